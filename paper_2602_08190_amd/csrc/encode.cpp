// Host encoders (Sec. 3: compression happens on the CPU and the compressed
// column stays in CPU memory).  Chunks are independent, so they are encoded in
// parallel across host threads.  FOR_BP, DICT_BP, DELTA_BP and RLE_DELTA_BP
// produce the canonical streams of the zf format byte for byte; the LZ77
// encoder additionally keeps every 64-sequence batch "flat" (see enc_lz77) so
// that the GPU can decode a batch with one sequence per lane.
#include <algorithm>
#include <atomic>
#include <functional>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <cstring>

#include "features.hpp"
#include "zf_internal.hpp"

namespace zf {

// ---------------------------------------------------------------- helpers
static inline uint32_t bit_width64(uint64_t v) { return v ? 64u - uint32_t(__builtin_clzll(v)) : 0u; }

static void parallel_for(uint64_t n, int threads, const std::function<void(uint64_t)> &fn);

// Append LSB-first w-bit fields into little-endian u32 words at `dst`.
struct BitPacker {
    uint8_t *dst;
    unsigned __int128 acc = 0;
    uint32_t nbits = 0;
    uint64_t words = 0;
    explicit BitPacker(uint8_t *d) : dst(d) {}
    inline void put(uint64_t v, uint32_t w) {
        if (w == 0) return;
        acc |= (unsigned __int128)v << nbits;
        nbits += w;
        while (nbits >= 32) {
            wr32(dst + 4 * words++, uint32_t(acc));
            acc >>= 32;
            nbits -= 32;
        }
    }
    inline void flush() {
        if (nbits) wr32(dst + 4 * words++, uint32_t(acc));
        acc = 0;
        nbits = 0;
    }
};

// ------------------------------------------------------------- FOR + BP
// Blocks of 2048 values; the reference is the block minimum and the width
// covers max - min (Sec. 2.1).
template <class T>
static void enc_for(std::vector<uint8_t> &s, const T *x, uint32_t n) {
    using U = std::make_unsigned_t<T>;
    const uint64_t nb = (n + kForBlock - 1) / kForBlock;
    std::vector<T> ref(nb);
    std::vector<uint32_t> w(nb), poff(nb);
    uint64_t pos = align_up(16 * nb, 16), end = pos;
    for (uint64_t b = 0; b < nb; b++) {
        const T *v = x + b * kForBlock;
        const uint32_t nv = uint32_t(std::min<uint64_t>(kForBlock, n - b * kForBlock));
        T lo = v[0], hi = v[0];
        for (uint32_t j = 1; j < nv; j++) {
            lo = std::min(lo, v[j]);
            hi = std::max(hi, v[j]);
        }
        ref[b] = lo;
        w[b] = bit_width64(uint64_t(U(U(hi) - U(lo))));
        poff[b] = uint32_t(pos);
        end = pos + 4 * ((uint64_t(nv) * w[b] + 31) / 32);
        pos = align_up(end, 16);
    }
    s.assign(end, 0);
    for (uint64_t b = 0; b < nb; b++) {
        wr64(s.data() + 16 * b, uint64_t(int64_t(ref[b])));
        wr32(s.data() + 16 * b + 8, w[b]);
        wr32(s.data() + 16 * b + 12, poff[b]);
        const T *v = x + b * kForBlock;
        const uint32_t nv = uint32_t(std::min<uint64_t>(kForBlock, n - b * kForBlock));
        BitPacker bp(s.data() + poff[b]);
        const U r = U(ref[b]);
        for (uint32_t j = 0; j < nv; j++) bp.put(uint64_t(U(U(v[j]) - r)), w[b]);
        bp.flush();
    }
}

// ----------------------------------------------------------- Float2Int
// Per block of 2048 float64 values, the decimal exponent e <= 18 whose
// integers d (bits(v) == bits(double(d) / 10^e)) pack into the fewest bits,
// counting 128 bits per value with no such d (an exception, stored raw);
// ties go to the smaller e.  The integers are then FOR + bit-packed.
static const double kF2iPow10[19] = {1e0,  1e1,  1e2,  1e3,  1e4,  1e5,  1e6,  1e7,  1e8, 1e9,
                                     1e10, 1e11, 1e12, 1e13, 1e14, 1e15, 1e16, 1e17, 1e18};

static inline bool f2i_fit(uint64_t vb, uint32_t e, int64_t &d) {
    double v;
    std::memcpy(&v, &vb, 8);
    const double m = v * kF2iPow10[e];
    if (!(std::fabs(m) < 4611686018427387904.0)) return false;  // 2^62; NaN fails too
    const int64_t k = int64_t(std::nearbyint(m));
    const double back = double(k) / kF2iPow10[e];
    uint64_t bb;
    std::memcpy(&bb, &back, 8);
    if (bb != vb) return false;
    d = k;
    return true;
}

static void enc_f2i(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n) {
    const uint64_t nb = (n + kForBlock - 1) / kForBlock;
    struct Blk {
        uint32_t e, w, nx;
        int64_t ref;
        uint64_t poff, xoff;
    };
    std::vector<Blk> blk(nb);
    std::vector<int64_t> d(n);
    std::vector<uint8_t> ok(n);
    uint64_t pos = align_up(32 * nb, 16), end = pos;
    for (uint64_t b = 0; b < nb; b++) {
        const uint64_t j0 = b * kForBlock;
        const uint32_t nv = uint32_t(std::min<uint64_t>(kForBlock, n - j0));
        uint64_t best_cost = ~0ull;
        uint32_t best_e = 0;
        for (uint32_t e = 0; e <= 18; e++) {
            uint32_t nx = 0;
            bool any = false;
            int64_t lo = 0, hi = 0, k = 0;
            for (uint32_t j = 0; j < nv; j++) {
                if (!f2i_fit(rd64(x + 8 * (j0 + j)), e, k)) {
                    nx++;
                    continue;
                }
                lo = any ? std::min(lo, k) : k;
                hi = any ? std::max(hi, k) : k;
                any = true;
            }
            const uint64_t cost = uint64_t(nv) * (any ? bit_width64(uint64_t(hi) - uint64_t(lo)) : 0) +
                                  128ull * nx;
            if (cost < best_cost) {
                best_cost = cost;
                best_e = e;
            }
        }
        Blk &B = blk[b];
        B.e = best_e;
        B.nx = 0;
        bool any = false;
        int64_t hi = 0;
        B.ref = 0;
        for (uint32_t j = 0; j < nv; j++) {
            ok[j0 + j] = f2i_fit(rd64(x + 8 * (j0 + j)), best_e, d[j0 + j]);
            if (!ok[j0 + j]) {
                B.nx++;
                continue;
            }
            B.ref = any ? std::min(B.ref, d[j0 + j]) : d[j0 + j];
            hi = any ? std::max(hi, d[j0 + j]) : d[j0 + j];
            any = true;
        }
        B.w = any ? bit_width64(uint64_t(hi) - uint64_t(B.ref)) : 0;
        B.poff = pos;
        B.xoff = align_up(pos + 4 * ((uint64_t(nv) * B.w + 31) / 32), 16);
        end = B.xoff + 16ull * B.nx;
        pos = align_up(end, 16);
    }
    s.assign(end, 0);
    for (uint64_t b = 0; b < nb; b++) {
        const Blk &B = blk[b];
        uint8_t *de = s.data() + 32 * b;
        wr64(de, uint64_t(B.ref));
        wr32(de + 8, B.w);
        wr32(de + 12, uint32_t(B.poff));
        wr32(de + 16, uint32_t(B.xoff));
        de[20] = uint8_t(B.nx);
        de[21] = uint8_t(B.nx >> 8);
        de[22] = uint8_t(B.e);
        const uint64_t j0 = b * kForBlock;
        const uint32_t nv = uint32_t(std::min<uint64_t>(kForBlock, n - j0));
        BitPacker bp(s.data() + B.poff);
        uint8_t *xr = s.data() + B.xoff;
        for (uint32_t j = 0; j < nv; j++) {
            if (ok[j0 + j]) {
                bp.put(uint64_t(d[j0 + j]) - uint64_t(B.ref), B.w);
            } else {
                bp.put(0, B.w);
                wr32(xr, j);
                wr64(xr + 8, rd64(x + 8 * (j0 + j)));
                xr += 16;
            }
        }
        bp.flush();
    }
}

// ------------------------------------------------------------------- ANS
// Range ANS over the chunk's bytes (static order-0 model, M = 4096), byte i
// coded by coder i mod 64.  Frequencies: floor(count * M / n), at least 1 for
// a present byte; a shortfall goes to the most frequent byte (ties: the
// smallest), an excess is taken one at a time from the largest frequency
// (ties: the smallest byte).  Each coder runs over its bytes backwards from
// x = 2^16, emitting the low 16 bits while x >= 2^20 * f; its words are
// stored in the order the decoder reads them (reversed).
static void ans_frequencies(const uint8_t *x, uint64_t n, uint32_t f[256]) {
    uint64_t cnt[256] = {0};
    for (uint64_t i = 0; i < n; i++) cnt[x[i]]++;
    uint32_t total = 0;
    for (int b = 0; b < 256; b++) {
        f[b] = cnt[b] ? std::max<uint32_t>(1, uint32_t(cnt[b] * kAnsM / n)) : 0;
        total += f[b];
    }
    if (total < kAnsM) {
        int top = 0;
        for (int b = 1; b < 256; b++)
            if (cnt[b] > cnt[top]) top = b;
        f[top] += kAnsM - total;
        total = kAnsM;
    }
    while (total > kAnsM) {
        int top = -1;
        for (int b = 0; b < 256; b++)
            if (f[b] > 1 && (top < 0 || f[b] > f[top])) top = b;
        f[top]--;
        total--;
    }
}

static void enc_ans(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n) {
    uint32_t f[256], cum[256];
    ans_frequencies(x, n, f);
    for (uint32_t b = 0, c = 0; b < 256; b++) {
        cum[b] = c;
        c += f[b];
    }
    // bytes from last to first, byte i into coder i mod 64; the words come
    // out in the reverse of the order the decoder takes them
    uint64_t st[kAnsLanes];
    for (uint32_t j = 0; j < kAnsLanes; j++) st[j] = kAnsL;
    std::vector<uint16_t> emitted;
    emitted.reserve(n / 4 + 16);
    for (uint32_t i = n; i-- > 0;) {
        uint64_t &x_ = st[i % kAnsLanes];
        const uint32_t b = x[i];
        const uint64_t lim = (uint64_t(kAnsL >> 12) << 16) * f[b];
        while (x_ >= lim) {
            emitted.push_back(uint16_t(x_));
            x_ >>= 16;
        }
        x_ = (x_ / f[b]) * kAnsM + x_ % f[b] + cum[b];
    }
    const uint64_t nw = emitted.size();
    s.assign(kAnsHdr + 2 * nw, 0);
    uint8_t *p = s.data();
    wr32(p, n);
    wr32(p + 4, uint32_t(nw));
    for (uint32_t b = 0; b < 256; b++) {
        p[16 + 2 * b] = uint8_t(f[b]);
        p[17 + 2 * b] = uint8_t(f[b] >> 8);
    }
    for (uint32_t j = 0; j < kAnsLanes; j++) wr32(p + 528 + 4 * j, uint32_t(st[j]));
    uint8_t *wp = p + kAnsHdr;
    for (uint64_t k = 0; k < nw; k++) {
        const uint16_t w = emitted[nw - 1 - k];
        wp[2 * k] = uint8_t(w);
        wp[2 * k + 1] = uint8_t(w >> 8);
    }
}

// ------------------------------------------------------------ dictionary
// Open-addressing set/map over keys of up to 16 bytes.
struct KeyTable {
    std::vector<uint64_t> k0, k1;
    std::vector<uint32_t> val;
    std::vector<uint8_t> used;
    uint64_t mask = 0, count = 0;
    static inline uint64_t mix(uint64_t a, uint64_t b) {
        uint64_t z = a * 0x9E3779B97F4A7C15ull ^ (b + 0x7F4A7C159E3779B9ull + (a << 6) + (a >> 2));
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    void init(uint64_t cap) {
        uint64_t c = 16;
        while (c < 2 * cap) c <<= 1;
        k0.assign(c, 0);
        k1.assign(c, 0);
        val.assign(c, 0);
        used.assign(c, 0);
        mask = c - 1;
        count = 0;
    }
    // returns slot; inserts when absent
    uint64_t insert(uint64_t a, uint64_t b) {
        if (2 * (count + 1) > mask + 1) grow();
        uint64_t h = mix(a, b) & mask;
        while (used[h]) {
            if (k0[h] == a && k1[h] == b) return h;
            h = (h + 1) & mask;
        }
        used[h] = 1;
        k0[h] = a;
        k1[h] = b;
        count++;
        return h;
    }
    int64_t find(uint64_t a, uint64_t b) const {
        uint64_t h = mix(a, b) & mask;
        while (used[h]) {
            if (k0[h] == a && k1[h] == b) return int64_t(h);
            h = (h + 1) & mask;
        }
        return -1;
    }
    void grow() {
        KeyTable t;
        t.init(2 * (mask + 1));
        for (uint64_t i = 0; i <= mask; i++)
            if (used[i]) t.insert(k0[i], k1[i]);
        *this = std::move(t);
    }
};

static inline void key_of(const uint8_t *v, uint32_t es, uint64_t &a, uint64_t &b) {
    a = b = 0;
    if (es == 4) a = uint64_t(int64_t(int32_t(rd32(v))));
    else if (es == 8) a = rd64(v);
    else { a = rd64(v); b = rd64(v + 8); }
}

struct Dictionary {
    std::vector<uint8_t> bytes;  // sorted unique entries
    uint32_t count = 0;
    uint32_t es = 0;
    KeyTable index;              // key -> code
};

// Sorted distinct values (integers by signed value, FIXED16 by memcmp).
// Returns false when there are more than max_count distinct values.
static bool build_dictionary(Dictionary &d, const uint8_t *x, uint64_t n, uint32_t dtype,
                             uint64_t max_count, int threads) {
    const uint32_t es = elem_size(dtype);
    d.es = es;
    const uint64_t parts = std::max<uint64_t>(1, std::min<uint64_t>(threads, (n + 65535) / 65536));
    std::vector<KeyTable> local(parts);
    std::atomic<bool> over{false};
    parallel_for(parts, threads, [&](uint64_t p) {
        uint64_t lo = n * p / parts, hi = n * (p + 1) / parts;
        local[p].init(1024);
        for (uint64_t i = lo; i < hi && !over.load(std::memory_order_relaxed); i++) {
            uint64_t a, b;
            key_of(x + i * es, es, a, b);
            local[p].insert(a, b);
            if (local[p].count > max_count) over = true;
        }
    });
    if (over) return false;
    KeyTable all;
    all.init(1024);
    for (auto &t : local)
        for (uint64_t i = 0; i <= t.mask; i++)
            if (t.used[i]) all.insert(t.k0[i], t.k1[i]);
    if (all.count > max_count) return false;
    std::vector<std::pair<uint64_t, uint64_t>> keys;
    keys.reserve(all.count);
    for (uint64_t i = 0; i <= all.mask; i++)
        if (all.used[i]) keys.emplace_back(all.k0[i], all.k1[i]);
    if (es == 16) {
        std::sort(keys.begin(), keys.end(), [](auto &p, auto &q) {
            uint8_t a[16], b[16];
            wr64(a, p.first); wr64(a + 8, p.second);
            wr64(b, q.first); wr64(b + 8, q.second);
            return std::memcmp(a, b, 16) < 0;
        });
    } else {
        std::sort(keys.begin(), keys.end(),
                  [](auto &p, auto &q) { return int64_t(p.first) < int64_t(q.first); });
    }
    d.count = uint32_t(keys.size());
    d.bytes.assign(uint64_t(d.count) * es, 0);
    d.index = std::move(all);
    for (uint32_t c = 0; c < d.count; c++) {
        uint8_t *e = d.bytes.data() + uint64_t(c) * es;
        if (es == 4) wr32(e, uint32_t(keys[c].first));
        else if (es == 8) wr64(e, keys[c].first);
        else { wr64(e, keys[c].first); wr64(e + 8, keys[c].second); }
        d.index.val[d.index.find(keys[c].first, keys[c].second)] = c;
    }
    return true;
}

static void enc_dict(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n, const Dictionary &d) {
    std::vector<int32_t> codes(n);
    for (uint32_t j = 0; j < n; j++) {
        uint64_t a, b;
        key_of(x + uint64_t(j) * d.es, d.es, a, b);
        int64_t h = d.index.find(a, b);
        if (h < 0) fail(ZF_E_INVALID, "value missing from the dictionary");
        codes[j] = int32_t(d.index.val[h]);
    }
    enc_for<int32_t>(s, codes.data(), n);
}

// ------------------------------------------------------- RLE / delta + BP
// Maximal runs (or unit runs for DELTA_BP); groups of 64 runs with their
// own output offset and value base; deltas of run values FOR-bit-packed.
template <class T>
static void enc_rle(std::vector<uint8_t> &s, const T *x, uint32_t n, bool unit_runs) {
    using U = std::make_unsigned_t<T>;
    std::vector<T> val;
    std::vector<uint32_t> len;
    val.reserve(unit_runs ? n : n / 4 + 16);
    len.reserve(unit_runs ? 0 : n / 4 + 16);
    for (uint32_t j = 0; j < n; j++) {
        if (!unit_runs && !val.empty() && val.back() == x[j]) len.back()++;
        else {
            val.push_back(x[j]);
            if (!unit_runs) len.push_back(1);
        }
    }
    const uint32_t nr = uint32_t(val.size());
    const uint32_t ng = (nr + kRleGroup - 1) / kRleGroup;
    // widths and offsets first
    std::vector<uint32_t> w(ng), doff(ng), out_off(ng);
    std::vector<T> dmin(ng);
    uint64_t pos = 16 + 32ull * ng;
    uint32_t produced = 0;
    for (uint32_t g = 0; g < ng; g++) {
        const uint32_t r0 = g * kRleGroup, cnt = std::min(kRleGroup, nr - r0);
        T mn = 0;
        U fmax = 0;
        for (uint32_t j = 1; j < cnt; j++) {
            T d = T(U(U(val[r0 + j]) - U(val[r0 + j - 1])));
            if (j == 1 || d < mn) mn = d;
        }
        for (uint32_t j = 1; j < cnt; j++) {
            U f = U(U(U(val[r0 + j]) - U(val[r0 + j - 1])) - U(mn));
            fmax = std::max(fmax, f);
        }
        dmin[g] = mn;
        w[g] = bit_width64(uint64_t(fmax));
        doff[g] = uint32_t(pos);
        out_off[g] = produced;
        pos += 4 * ((uint64_t(cnt - 1) * w[g] + 31) / 32);
        if (unit_runs) produced += cnt;
        else
            for (uint32_t j = 0; j < cnt; j++) produced += len[r0 + j];
    }
    const uint64_t roff = unit_runs ? 0 : align_up(pos, 16);
    s.assign(unit_runs ? pos : roff + 4ull * nr, 0);
    uint8_t *p = s.data();
    wr32(p, nr);
    wr32(p + 4, ng);
    wr32(p + 8, uint32_t(roff));
    for (uint32_t g = 0; g < ng; g++) {
        const uint32_t r0 = g * kRleGroup, cnt = std::min(kRleGroup, nr - r0);
        uint8_t *rec = p + 16 + 32ull * g;
        wr32(rec, out_off[g]);
        wr32(rec + 4, w[g]);
        wr32(rec + 8, doff[g]);
        wr64(rec + 16, uint64_t(int64_t(val[r0])));
        wr64(rec + 24, uint64_t(int64_t(dmin[g])));
        BitPacker bp(p + doff[g]);
        for (uint32_t j = 1; j < cnt; j++)
            bp.put(uint64_t(U(U(U(val[r0 + j]) - U(val[r0 + j - 1])) - U(dmin[g]))), w[g]);
        bp.flush();
    }
    if (!unit_runs)
        for (uint32_t j = 0; j < nr; j++) wr32(p + roff + 4ull * j, len[j]);
}

// ------------------------------------------------------------ DeltaStride
// Runs that are arithmetic progressions, maximal from the left (a run of one
// element only at the end); groups of 64 runs with their own output offset
// and first start; each later start is coded as its gap to the value the
// previous run would produce next; gaps and strides FOR-bit-packed.
template <class T>
static void enc_dstride(std::vector<uint8_t> &s, const T *x, uint32_t n) {
    using U = std::make_unsigned_t<T>;
    std::vector<U> st, sd;
    std::vector<uint32_t> len;
    for (uint32_t i = 0; i < n;) {
        U d = 0;
        uint32_t r = 1;
        if (i + 1 < n) {
            d = U(U(x[i + 1]) - U(x[i]));
            r = 2;
            while (i + r < n && U(U(x[i + r]) - U(x[i + r - 1])) == d) r++;
        }
        st.push_back(U(x[i]));
        sd.push_back(d);
        len.push_back(r);
        i += r;
    }
    const uint32_t nr = uint32_t(st.size()), ng = (nr + kRleGroup - 1) / kRleGroup;
    struct Grp { uint32_t out_off, poff, wg, wd; T gmin, dmin; };
    std::vector<Grp> G(ng);
    std::vector<U> gap(nr, 0);
    uint64_t pos = 16 + 32ull * ng;
    uint32_t produced = 0;
    for (uint32_t g = 0; g < ng; g++) {
        const uint32_t r0 = g * kRleGroup, cnt = std::min(kRleGroup, nr - r0);
        T gmin = 0, dmin = T(sd[r0]);
        for (uint32_t j = 1; j < cnt; j++) {
            gap[r0 + j] = U(st[r0 + j] - U(st[r0 + j - 1] + U(sd[r0 + j - 1] * U(len[r0 + j - 1]))));
            if (j == 1 || T(gap[r0 + j]) < gmin) gmin = T(gap[r0 + j]);
        }
        for (uint32_t j = 1; j < cnt; j++) dmin = std::min(dmin, T(sd[r0 + j]));
        U gmax = 0, dmax = 0;
        for (uint32_t j = 1; j < cnt; j++) gmax = std::max(gmax, U(gap[r0 + j] - U(gmin)));
        for (uint32_t j = 0; j < cnt; j++) dmax = std::max(dmax, U(sd[r0 + j] - U(dmin)));
        Grp &q = G[g];
        q.wg = bit_width64(uint64_t(gmax));
        q.wd = bit_width64(uint64_t(dmax));
        q.gmin = gmin;
        q.dmin = dmin;
        pos = align_up(pos, 8);
        q.poff = uint32_t(pos);
        q.out_off = produced;
        pos += 8 + 4 * ((uint64_t(cnt - 1) * q.wg + 31) / 32 + (uint64_t(cnt) * q.wd + 31) / 32);
        for (uint32_t j = 0; j < cnt; j++) produced += len[r0 + j];
    }
    const uint64_t roff = align_up(pos, 16);
    s.assign(roff + 4ull * nr, 0);
    uint8_t *p = s.data();
    wr32(p, nr);
    wr32(p + 4, ng);
    wr32(p + 8, uint32_t(roff));
    for (uint32_t g = 0; g < ng; g++) {
        const uint32_t r0 = g * kRleGroup, cnt = std::min(kRleGroup, nr - r0);
        const Grp &q = G[g];
        uint8_t *rec = p + 16 + 32ull * g;
        wr32(rec, q.out_off);
        wr32(rec + 4, q.poff);
        wr32(rec + 8, q.wg | (q.wd << 8));
        wr64(rec + 16, uint64_t(int64_t(T(st[r0]))));
        wr64(rec + 24, uint64_t(int64_t(q.dmin)));
        wr64(p + q.poff, uint64_t(int64_t(q.gmin)));
        BitPacker bg(p + q.poff + 8);
        for (uint32_t j = 1; j < cnt; j++) bg.put(uint64_t(U(gap[r0 + j] - U(q.gmin))), q.wg);
        bg.flush();
        BitPacker bd(p + q.poff + 8 + 4 * ((uint64_t(cnt - 1) * q.wg + 31) / 32));
        for (uint32_t j = 0; j < cnt; j++) bd.put(uint64_t(U(sd[r0 + j] - U(q.dmin))), q.wd);
        bd.flush();
    }
    for (uint32_t j = 0; j < nr; j++) wr32(p + roff + 4ull * j, len[j]);
}

// ------------------------------------ DeltaStride | [Delta | RLE | [BP, BP], BP]
// The chunk's stride d is its most frequent neighbour difference (ties to the
// smaller as unsigned); maximal runs of step d give the starts S and counts
// C; D = S[0], S[1] - S[0], ... is run-length coded into V (values) and L
// (lengths).  V, L and C are bit-packed per group of 64 against the group's
// smallest value; each group record holds its output offset (D's groups also
// the start before them), so both levels decode group-parallel.
template <class T>
static void enc_dstree(std::vector<uint8_t> &s, const T *x, uint32_t n) {
    using U = std::make_unsigned_t<T>;
    U d = 0;
    if (n > 1) {
        std::vector<U> df(n - 1);
        for (uint32_t i = 0; i + 1 < n; i++) df[i] = U(U(x[i + 1]) - U(x[i]));
        std::sort(df.begin(), df.end());
        uint32_t best = 0;
        for (uint32_t i = 0; i < n - 1;) {
            uint32_t k = i;
            while (k < n - 1 && df[k] == df[i]) k++;
            if (k - i > best) {
                best = k - i;
                d = df[i];
            }
            i = k;
        }
    }
    std::vector<U> S, V;
    std::vector<uint32_t> C, L;
    for (uint32_t i = 0; i < n;) {
        uint32_t r = 1;
        while (i + r < n && U(U(x[i + r]) - U(x[i + r - 1])) == d) r++;
        S.push_back(U(x[i]));
        C.push_back(r);
        i += r;
    }
    for (size_t k = 0; k < S.size(); k++) {
        const U dk = k == 0 ? S[0] : U(S[k] - S[k - 1]);
        if (!V.empty() && V.back() == dk) L.back()++;
        else {
            V.push_back(dk);
            L.push_back(1);
        }
    }
    const uint32_t R = uint32_t(S.size()), Q = uint32_t(V.size());
    const uint32_t ngA = (Q + 63) / 64, ngB = (R + 63) / 64;
    const uint64_t b_off = 32 + 32ull * ngA;
    auto words = [](uint32_t cnt, uint32_t w) { return (uint64_t(cnt) * w + 31) / 32; };
    struct GA { uint32_t wv, wl, lmin; T vmin; };
    struct GB { uint32_t wc, cmin; };
    std::vector<GA> ga(ngA);
    std::vector<GB> gb(ngB);
    uint64_t pos = b_off + 16ull * ngB;
    for (uint32_t g = 0; g < ngA; g++) {
        const uint32_t j0 = 64 * g, cnt = std::min(64u, Q - j0);
        T vmin = T(V[j0]);
        uint32_t lmin = L[j0], lmax = L[j0];
        for (uint32_t j = 1; j < cnt; j++) {
            vmin = std::min(vmin, T(V[j0 + j]));
            lmin = std::min(lmin, L[j0 + j]);
            lmax = std::max(lmax, L[j0 + j]);
        }
        U fmax = 0;
        for (uint32_t j = 0; j < cnt; j++) fmax = std::max(fmax, U(V[j0 + j] - U(vmin)));
        ga[g] = {bit_width64(uint64_t(fmax)), bit_width64(lmax - lmin), lmin, vmin};
        pos += 4 * (words(cnt, ga[g].wv) + words(cnt, ga[g].wl));
    }
    for (uint32_t g = 0; g < ngB; g++) {
        const uint32_t j0 = 64 * g, cnt = std::min(64u, R - j0);
        uint32_t lo = C[j0], hi = C[j0];
        for (uint32_t j = 1; j < cnt; j++) {
            lo = std::min(lo, C[j0 + j]);
            hi = std::max(hi, C[j0 + j]);
        }
        gb[g] = {bit_width64(hi - lo), lo};
        pos += 4 * words(cnt, gb[g].wc);
    }
    s.assign(pos, 0);
    uint8_t *p = s.data();
    wr32(p, R);
    wr32(p + 4, ngB);
    wr32(p + 8, Q);
    wr32(p + 12, ngA);
    wr64(p + 16, uint64_t(int64_t(T(d))));
    wr32(p + 24, uint32_t(b_off));
    pos = b_off + 16ull * ngB;
    uint32_t at = 0;
    for (uint32_t g = 0; g < ngA; g++) {
        const uint32_t j0 = 64 * g, cnt = std::min(64u, Q - j0);
        const GA &q = ga[g];
        uint8_t *rec = p + 32 + 32ull * g;
        wr32(rec, at);
        wr32(rec + 4, uint32_t(pos));
        wr32(rec + 8, q.wv | (q.wl << 8));
        wr32(rec + 12, q.lmin);
        wr64(rec + 16, at == 0 ? 0 : uint64_t(int64_t(T(S[at - 1]))));
        wr64(rec + 24, uint64_t(int64_t(q.vmin)));
        BitPacker bv(p + pos);
        for (uint32_t j = 0; j < cnt; j++) bv.put(uint64_t(U(V[j0 + j] - U(q.vmin))), q.wv);
        bv.flush();
        BitPacker bl(p + pos + 4 * words(cnt, q.wv));
        for (uint32_t j = 0; j < cnt; j++) bl.put(L[j0 + j] - q.lmin, q.wl);
        bl.flush();
        pos += 4 * (words(cnt, q.wv) + words(cnt, q.wl));
        for (uint32_t j = 0; j < cnt; j++) at += L[j0 + j];
    }
    uint32_t out = 0;
    for (uint32_t g = 0; g < ngB; g++) {
        const uint32_t j0 = 64 * g, cnt = std::min(64u, R - j0);
        uint8_t *rec = p + b_off + 16ull * g;
        wr32(rec, out);
        wr32(rec + 4, uint32_t(pos));
        wr32(rec + 8, gb[g].wc);
        wr32(rec + 12, gb[g].cmin);
        BitPacker bc(p + pos);
        for (uint32_t j = 0; j < cnt; j++) bc.put(C[j0 + j] - gb[g].cmin, gb[g].wc);
        bc.flush();
        pos += 4 * words(cnt, gb[g].wc);
        for (uint32_t j = 0; j < cnt; j++) out += C[j0 + j];
    }
}

// ------------------------------------------------------ String-dictionary
// Tokens end after a space or a period (at most 64 bytes; the chunk's last
// token may end without one); the distinct tokens, in order of first
// appearance, are the entries; entry indices bit-packed at the smallest
// width that holds the last index; one output offset per 64 tokens.
static void enc_sdict(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n) {
    struct Key {
        const uint8_t *p;
        uint32_t len;
        bool operator==(const Key &o) const { return len == o.len && std::memcmp(p, o.p, len) == 0; }
    };
    struct Hash {
        size_t operator()(const Key &k) const {
            uint64_t h = 0x9E3779B97F4A7C15ull ^ k.len;
            for (uint32_t i = 0; i < k.len; i++) h = (h ^ k.p[i]) * 0x100000001B3ull;
            return size_t(h ^ (h >> 29));
        }
    };
    std::unordered_map<Key, uint32_t, Hash> index;
    std::vector<Key> entries;
    std::vector<uint32_t> codes, starts;
    uint32_t nbytes = 0;
    for (uint32_t i = 0; i < n;) {
        uint32_t L = 0;
        while (i + L < n && L < kSdMaxToken) {
            const uint8_t c = x[i + L++];
            if (c == ' ' || c == '.') break;
        }
        const Key k{x + i, L};
        auto it = index.find(k);
        uint32_t code;
        if (it == index.end()) {
            code = uint32_t(entries.size());
            index.emplace(k, code);
            entries.push_back(k);
            nbytes += L;
        } else {
            code = it->second;
        }
        if (codes.size() % 64 == 0) starts.push_back(i);
        codes.push_back(code);
        i += L;
    }
    const uint32_t nt = uint32_t(codes.size()), ne = uint32_t(entries.size());
    const uint32_t w = ne > 1 ? bit_width64(ne - 1) : 0, ng = uint32_t(starts.size());
    const uint64_t eo = align_up(32 + 4ull * ng, 16), bo = eo + 4ull * ne;
    const uint64_t co = align_up(bo + nbytes + 4, 16);
    s.assign(co + 4 * ((uint64_t(nt) * w + 31) / 32), 0);
    uint8_t *p = s.data();
    const uint32_t hdr[8] = {nt, ne, w, ng, uint32_t(eo), uint32_t(bo), uint32_t(co), nbytes};
    for (int k = 0; k < 8; k++) wr32(p + 4 * k, hdr[k]);
    for (uint32_t g = 0; g < ng; g++) wr32(p + 32 + 4ull * g, starts[g]);
    uint32_t at = 0;
    for (uint32_t k = 0; k < ne; k++) {
        wr32(p + eo + 4ull * k, at | (entries[k].len << 24));
        std::memcpy(p + bo + at, entries[k].p, entries[k].len);
        at += entries[k].len;
    }
    BitPacker bp(p + co);
    for (uint32_t c : codes) bp.put(c, w);
    bp.flush();
}

// ----------------------------------- String-dictionary, column dictionary
// One dictionary for the column's SDICT_COL / SDICT_COL_ANS chunks: tokens
// end after a space, a period or a newline (the end of a row value), at most
// 64 bytes; entries by decreasing count, ties by first appearance in the
// column; in the container's dictionary area as {u32 n_bytes, 3 x u32 0,
// u32 entry[n] (offset | length << 24), entry bytes with at least 3 zero
// bytes on each side of every entry, zero padding to a multiple of 16}.  A chunk keeps its token count,
// width, group offsets and the bit-packed entry indices.
static inline uint32_t sdc_token_len(const uint8_t *x, uint32_t n, uint32_t i) {
    uint32_t L = 0;
    while (i + L < n && L < kSdMaxToken) {
        const uint8_t c = x[i + L++];
        if (c == ' ' || c == '.' || c == '\n') break;
    }
    return L;
}

// Open-addressing table of tokens (a pointer into the column and a length).
struct TokenTable {
    struct Slot {
        const uint8_t *p = nullptr;
        uint32_t len = 0, val = 0;  // val: count while counting, then the entry index
        uint64_t first = 0;         // first occurrence (byte offset in the column)
    };
    std::vector<Slot> slots;
    uint64_t mask = 0, count = 0;
    static inline uint64_t hash(const uint8_t *p, uint32_t len) {
        uint64_t h = 0x9E3779B97F4A7C15ull ^ len;
        uint32_t i = 0;
        for (; i + 8 <= len; i += 8) {
            uint64_t v;
            std::memcpy(&v, p + i, 8);
            h = (h ^ v) * 0xBF58476D1CE4E5B9ull;
            h ^= h >> 31;
        }
        uint64_t t = 0;
        for (uint32_t k = 0; i + k < len; k++) t |= uint64_t(p[i + k]) << (8 * k);
        h = (h ^ t) * 0x94D049BB133111EBull;
        return h ^ (h >> 29);
    }
    TokenTable() { init(1024); }
    void init(uint64_t cap) {
        uint64_t c = 16;
        while (c < 2 * cap) c <<= 1;
        slots.assign(c, Slot{});
        mask = c - 1;
        count = 0;
    }
    Slot *find(const uint8_t *p, uint32_t len) {
        uint64_t h = hash(p, len) & mask;
        while (slots[h].p) {
            if (slots[h].len == len && std::memcmp(slots[h].p, p, len) == 0) return &slots[h];
            h = (h + 1) & mask;
        }
        return nullptr;
    }
    const Slot *find(const uint8_t *p, uint32_t len) const { return const_cast<TokenTable *>(this)->find(p, len); }
    // add `cnt` occurrences of a token first seen at `first`
    void add(const uint8_t *p, uint32_t len, uint64_t first, uint32_t cnt) {
        if (2 * (count + 1) > mask + 1) grow();
        uint64_t h = hash(p, len) & mask;
        while (slots[h].p) {
            Slot &s = slots[h];
            if (s.len == len && std::memcmp(s.p, p, len) == 0) {
                s.val += cnt;
                s.first = std::min(s.first, first);
                return;
            }
            h = (h + 1) & mask;
        }
        slots[h] = Slot{p, len, cnt, first};
        count++;
    }
    void grow() {
        std::vector<Slot> old;
        old.swap(slots);
        init(2 * (mask + 1));
        for (const Slot &s : old)
            if (s.p) add(s.p, s.len, s.first, s.val);
    }
};

struct TokenDictionary {
    TokenTable table;            // token -> entry index
    std::vector<uint8_t> area;   // the dictionary area
    uint32_t count = 0, w = 0;
};

// Count the tokens of the chunks with codec SDICT_COL / SDICT_COL_ANS (in
// parallel), order them and lay out the dictionary area.
static void build_token_dictionary(TokenDictionary &d, const uint8_t *src, const std::vector<uint32_t> &ce,
                                   const std::vector<uint8_t> &cc, const std::vector<uint64_t> &first,
                                   int threads) {
    std::vector<uint64_t> todo;
    for (size_t i = 0; i < ce.size(); i++)
        if (cc[i] == C_SDICT_COL || cc[i] == C_SDICT_COL_ANS) todo.push_back(i);
    const int nt = int(std::max<uint64_t>(1, std::min<uint64_t>(uint64_t(threads), todo.size())));
    std::vector<TokenTable> part(nt);
    std::atomic<uint64_t> next{0};
    auto work = [&](int t) {
        for (uint64_t k; (k = next.fetch_add(1)) < todo.size();) {
            const uint64_t i = todo[k];
            const uint8_t *x = src + first[i];
            for (uint32_t a = 0; a < ce[i];) {
                const uint32_t L = sdc_token_len(x, ce[i], a);
                part[t].add(x + a, L, first[i] + a, 1);
                a += L;
            }
        }
    };
    {
        std::vector<std::thread> ts;
        for (int t = 1; t < nt; t++) ts.emplace_back(work, t);
        work(0);
        for (auto &th : ts) th.join();
    }
    for (int t = 1; t < nt; t++)
        for (const auto &s : part[t].slots)
            if (s.p) part[0].add(s.p, s.len, s.first, s.val);
    std::vector<const TokenTable::Slot *> ent;
    for (const auto &s : part[0].slots)
        if (s.p) ent.push_back(&s);
    ZF_REQUIRE(ent.size() <= (1u << 24), ZF_E_UNSUPPORTED,
               "%zu distinct tokens: a column dictionary holds at most 2^24", ent.size());
    std::sort(ent.begin(), ent.end(), [](const TokenTable::Slot *a, const TokenTable::Slot *b) {
        return a->val != b->val ? a->val > b->val : a->first < b->first;
    });
    // entry bytes with zero guards: 4 zero bytes, then each entry followed by
    // at least 3 zero bytes up to a multiple of 4 (a decoder may read whole
    // dwords around an entry)
    uint64_t nb = 4, last = 4;
    for (auto *e : ent) {
        last = nb;
        nb = align_up(nb + e->len + 3, 4);
    }
    nb = std::max(nb, last + 16);  // 16 bytes from the last entry's start
    ZF_REQUIRE(nb < (1u << 24), ZF_E_UNSUPPORTED,
               "%llu bytes of distinct tokens: a column dictionary holds at most 2^24 - 1",
               (unsigned long long)nb);
    d.count = uint32_t(ent.size());
    d.w = d.count > 1 ? bit_width64(d.count - 1) : 0;
    d.area.assign(16 + 4ull * d.count + align_up(nb, 16), 0);
    wr32(d.area.data(), uint32_t(nb));
    d.table.init(d.count);
    uint32_t at = 4;
    for (uint32_t k = 0; k < d.count; k++) {
        const TokenTable::Slot *e = ent[k];
        wr32(d.area.data() + 16 + 4ull * k, at | (e->len << 24));
        std::memcpy(d.area.data() + 16 + 4ull * d.count + at, e->p, e->len);
        at = uint32_t(align_up(at + e->len + 3, 4));
        d.table.add(e->p, e->len, e->first, k);
    }
}

static void enc_sdict_col(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n, const TokenDictionary &d) {
    std::vector<uint32_t> codes, starts;
    codes.reserve(n / 4 + 1);
    for (uint32_t i = 0; i < n;) {
        const uint32_t L = sdc_token_len(x, n, i);
        const TokenTable::Slot *e = d.table.find(x + i, L);
        if (!e) fail(ZF_E_INVALID, "token missing from the column dictionary");
        if (codes.size() % 64 == 0) starts.push_back(i);
        codes.push_back(e->val);
        i += L;
    }
    const uint32_t nt = uint32_t(codes.size()), ng = uint32_t(starts.size()), w = d.w;
    const uint64_t co = align_up(16 + 4ull * ng, 16);
    s.assign(co + 4 * ((uint64_t(nt) * w + 31) / 32), 0);
    uint8_t *p = s.data();
    wr32(p, nt);
    wr32(p + 4, w);
    wr32(p + 8, ng);
    wr32(p + 12, uint32_t(co));
    for (uint32_t g = 0; g < ng; g++) wr32(p + 16 + 4ull * g, starts[g]);
    BitPacker bp(p + co);
    for (uint32_t c : codes) bp.put(c, w);
    bp.flush();
}

// ------------------------------------------------------------------ LZ77
// Greedy LZ77 over a chunk of <= 64 KiB: hash chains of 4-byte prefixes
// (depth 16), longest match, nearest source on ties.
//
// Flat batches: sequences are grouped 64 at a time (one per lane of a
// wavefront).  Within a batch, every match may read only bytes written before
// the batch began, or bytes of its own sequence's literals.  Then all literal
// copies of a batch are independent, and so are all match copies once the
// literals are in place; the decoder needs no ordering inside the batch.  A
// candidate that would read another sequence of the same batch is shortened
// to end before the batch (or dropped).  Streams without this property are
// still valid and still decode (the GPU falls back to in-order copies).
struct LzScratch {
    std::vector<int32_t> head, prev;
    LzScratch() : head(1u << 16), prev(kLzMaxChunk) {}
};

static inline uint32_t lz_hash4(const uint8_t *p) {
    uint32_t v;
    std::memcpy(&v, p, 4);
    return (v * 2654435761u) >> 16;
}

static void enc_lz77(std::vector<uint8_t> &s, const uint8_t *x, uint32_t n, LzScratch &sc) {
    struct Seq { uint32_t ll, ml, off; };
    std::vector<Seq> seq;
    seq.reserve(n / 8 + 4);
    std::fill(sc.head.begin(), sc.head.end(), -1);
    int32_t *head = sc.head.data(), *prev = sc.prev.data();
    auto insert = [&](uint32_t k) {
        if (k + 4 <= n) {
            uint32_t h = lz_hash4(x + k);
            prev[k] = head[h];
            head[h] = int32_t(k);
        }
    };
    uint32_t i = 0, lit_start = 0, batch_start = 0;
    while (i < n) {
        uint32_t best = 0, best_off = 0;
        if (i + 4 <= n) {
            int32_t c = head[lz_hash4(x + i)];
            const uint32_t lim = n - i;
            for (int d = 0; d < 16 && c >= 0; d++, c = prev[c]) {
                const uint32_t cu = uint32_t(c);
                if (best > 0 && (best >= lim || x[cu + best] != x[i + best])) continue;
                uint32_t l = 0;
                while (l < lim && x[cu + l] == x[i + l]) l++;
                const uint32_t off = i - cu;
                if (cu < lit_start && cu + std::min(l, off) > batch_start)
                    l = batch_start > cu ? batch_start - cu : 0;
                if (l > best) {
                    best = l;
                    best_off = off;
                }
            }
        }
        if (best >= 4) {
            seq.push_back({i - lit_start, best, best_off});
            for (uint32_t k = i; k < i + best; k++) insert(k);
            i += best;
            lit_start = i;
            if (seq.size() % 64 == 0) batch_start = i;
        } else {
            insert(i);
            i++;
        }
    }
    if (lit_start < n) seq.push_back({n - lit_start, 0, 0});

    uint64_t next = 0, nlit = 0;
    for (auto &q : seq) {
        next += (q.ll >= 7) + (q.ml >= 34);
        nlit += q.ll;
    }
    const uint64_t ns = seq.size();
    s.assign(16 + 3 * ns + 2 * next + nlit, 0);
    uint8_t *p = s.data();
    wr32(p, uint32_t(ns));
    wr32(p + 4, uint32_t(nlit));
    wr32(p + 8, uint32_t(next));
    wr32(p + 12, n);
    uint8_t *offs = p + 16, *ext = offs + 2 * ns, *tags = ext + 2 * next, *lits = tags + ns;
    uint64_t e = 0, lp = 0, pos = 0;
    for (uint64_t k = 0; k < ns; k++) {
        const Seq &q = seq[k];
        uint32_t lc = q.ll, mc;
        if (q.ll >= 7) { lc = 7; wr16(ext + 2 * e++, uint16_t(q.ll - 7)); }
        if (q.ml == 0) mc = 0;
        else if (q.ml <= 33) mc = q.ml - 3;
        else { mc = 31; wr16(ext + 2 * e++, uint16_t(q.ml - 34)); }
        tags[k] = uint8_t(lc | (mc << 3));
        wr16(offs + 2 * k, uint16_t(q.off));
        std::memcpy(lits + lp, x + pos, q.ll);
        lp += q.ll;
        pos += q.ll + q.ml;
    }
}

// --------------------------------------------------------------- driver
static void parallel_for(uint64_t n, int threads, const std::function<void(uint64_t)> &fn) {
    if (n == 0) return;
    const int t = int(std::max<uint64_t>(1, std::min<uint64_t>(uint64_t(threads), n)));
    std::atomic<uint64_t> next{0};
    std::vector<Error> errs;
    std::mutex mu;
    auto work = [&] {
        try {
            for (uint64_t i; (i = next.fetch_add(1)) < n;) fn(i);
        } catch (const Error &e) {
            std::lock_guard<std::mutex> g(mu);
            errs.push_back(e);
            next = n;
        }
    };
    if (t == 1) work();
    else {
        std::vector<std::thread> ts;
        for (int k = 0; k < t; k++) ts.emplace_back(work);
        for (auto &th : ts) th.join();
    }
    if (!errs.empty()) throw errs[0];
}

static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The packed entry indices at co of a String-dictionary stream `sd`
// replaced by ANS streams of them in independent pieces of kSdAnsPiece
// bytes: u32 count, u32 stream ends, streams (each zero-padded to a multiple
// of 4 bytes).
static void ans_pieces(std::vector<uint8_t> &out, const std::vector<uint8_t> &sd, uint32_t co) {
    const uint64_t ncb = sd.size() - co;
    const uint32_t np = uint32_t((ncb + kSdAnsPiece - 1) / kSdAnsPiece);
    out.assign(sd.begin(), sd.begin() + co);
    if (!np) return;
    out.resize(co + 4 + 4ull * np, 0);
    wr32(out.data() + co, np);
    const uint64_t base = out.size();
    std::vector<uint8_t> a;
    for (uint32_t k = 0; k < np; k++) {
        const uint64_t lo = uint64_t(k) * kSdAnsPiece, hi = std::min<uint64_t>(lo + kSdAnsPiece, ncb);
        enc_ans(a, sd.data() + co + lo, uint32_t(hi - lo));
        out.insert(out.end(), a.begin(), a.end());
        out.resize(align_up(out.size(), 4), 0);  // the next stream starts 4-aligned
        wr32(out.data() + co + 4 + 4ull * k, uint32_t(out.size() - base));
    }
}

static void encode_chunk(std::vector<uint8_t> &out, uint32_t codec, uint32_t dtype, const uint8_t *x,
                         uint32_t n, const Dictionary *dict, const TokenDictionary *tdict, LzScratch &sc) {
    const uint32_t es = elem_size(dtype);
    switch (codec) {
    case C_PLAIN: out.assign(x, x + uint64_t(n) * es); return;
    case C_FOR_BP:
        if (dtype == D_I32) enc_for<int32_t>(out, reinterpret_cast<const int32_t *>(x), n);
        else enc_for<int64_t>(out, reinterpret_cast<const int64_t *>(x), n);
        return;
    case C_DICT_BP: enc_dict(out, x, n, *dict); return;
    case C_DELTA_BP:
    case C_RLE_DELTA_BP:
        if (dtype == D_I32) enc_rle<int32_t>(out, reinterpret_cast<const int32_t *>(x), n, codec == C_DELTA_BP);
        else enc_rle<int64_t>(out, reinterpret_cast<const int64_t *>(x), n, codec == C_DELTA_BP);
        return;
    case C_LZ77: enc_lz77(out, x, n * es, sc); return;
    case C_F2I_BP: enc_f2i(out, x, n); return;
    case C_ANS: enc_ans(out, x, n * es); return;
    case C_DSTRIDE_BP:
        if (dtype == D_I32) enc_dstride<int32_t>(out, reinterpret_cast<const int32_t *>(x), n);
        else enc_dstride<int64_t>(out, reinterpret_cast<const int64_t *>(x), n);
        return;
    case C_DSTREE:
        if (dtype == D_I32) enc_dstree<int32_t>(out, reinterpret_cast<const int32_t *>(x), n);
        else enc_dstree<int64_t>(out, reinterpret_cast<const int64_t *>(x), n);
        return;
    case C_SDICT_BP: enc_sdict(out, x, n); return;
    case C_SDICT_ANS: {
        std::vector<uint8_t> sd;
        enc_sdict(sd, x, n);
        ans_pieces(out, sd, rd32(sd.data() + 24));
        return;
    }
    case C_SDICT_COL: enc_sdict_col(out, x, n, *tdict); return;
    case C_SDICT_COL_ANS: {
        std::vector<uint8_t> sd;
        enc_sdict_col(sd, x, n, *tdict);
        ans_pieces(out, sd, rd32(sd.data() + 12));
        return;
    }
    }
    fail(ZF_E_INVALID, "unknown codec %u", codec);
}

double time_choice(const uint8_t *x, uint32_t n, uint32_t dtype, uint32_t codec, uint32_t sched, int device,
                   int threads);

// forced_sched (internal, nullable): the schedule stored for each chunk of an
// explicit chunking
void compress_host(const void *srcv, uint64_t n_elems, uint32_t dtype, uint32_t codec,
                   const zf_encode_opts &o, zf_column_t *col, const uint8_t *forced_sched) {
    const uint8_t *src = static_cast<const uint8_t *>(srcv);
    const uint32_t es = elem_size(dtype);
    ZF_REQUIRE(es, ZF_E_INVALID, "unknown dtype %u", dtype);
    ZF_REQUIRE(src || n_elems == 0, ZF_E_INVALID, "null source");
    ZF_REQUIRE(codec == 0 || codec_allows(codec, dtype), ZF_E_INVALID, "codec %u cannot encode dtype %u",
               codec, dtype);
    const int threads = o.n_threads > 0 ? o.n_threads : int(std::max(1u, std::thread::hardware_concurrency()));

    // chunking
    std::vector<uint32_t> ce;
    std::vector<uint8_t> cc;
    if (o.chunk_elems && o.n_chunk_elems) {
        uint64_t sum = 0;
        for (uint32_t i = 0; i < o.n_chunk_elems; i++) {
            ZF_REQUIRE(o.chunk_elems[i] > 0, ZF_E_INVALID, "empty chunk %u", i);
            ce.push_back(o.chunk_elems[i]);
            sum += o.chunk_elems[i];
            uint32_t c = o.chunk_codecs ? o.chunk_codecs[i] : codec;
            ZF_REQUIRE(c == 0 || codec_allows(c, dtype), ZF_E_INVALID, "chunk %u: codec %u", i, c);
            cc.push_back(uint8_t(c));
        }
        ZF_REQUIRE(sum == n_elems, ZF_E_INVALID, "chunk sizes sum to %llu, not %llu",
                   (unsigned long long)sum, (unsigned long long)n_elems);
    } else {
        // LZ77 chunks hold at most 64 KiB; ANS defaults to 64 KiB chunks (one
        // wave each) but takes any size; block codecs round to 2048 values
        const bool lz = codec == C_LZ77, bytewise = lz || codec == C_ANS;
        uint64_t lo = o.chunk_bytes_min ? o.chunk_bytes_min : (bytewise ? kLzMaxChunk : (1u << 20));
        uint64_t hi = std::max<uint64_t>(lo, o.chunk_bytes_max ? o.chunk_bytes_max : lo);
        uint64_t rs = o.seed ^ 0x5A17C0DEull;
        for (uint64_t at = 0; at < n_elems;) {
            uint64_t bytes = lo;
            if (hi > lo) {
                double u = double(splitmix(rs) >> 11) * (1.0 / 9007199254740992.0);
                bytes = uint64_t(std::exp(std::log(double(lo)) + u * (std::log(double(hi)) - std::log(double(lo)))));
            }
            uint64_t e = lz ? std::min<uint64_t>(bytes, kLzMaxChunk) / es
                         : bytewise ? bytes / es
                                    : std::max<uint64_t>(kForBlock, bytes / es / kForBlock * kForBlock);
            e = std::max<uint64_t>(1, std::min<uint64_t>(e, n_elems - at));
            e = std::min<uint64_t>(e, 0xFFFFFFFFull / es);
            ce.push_back(uint32_t(e));
            cc.push_back(uint8_t(codec));
            at += e;
        }
    }
    for (size_t i = 0; i < ce.size(); i++)
        if (cc[i] == C_LZ77)
            ZF_REQUIRE(uint64_t(ce[i]) * es <= kLzMaxChunk, ZF_E_INVALID,
                       "LZ77 chunk %zu holds %llu bytes (limit 65536)", i,
                       (unsigned long long)(uint64_t(ce[i]) * es));

    // dictionary, when any chunk may use it
    bool want_dict = false, any_auto = false;
    for (auto c : cc) {
        want_dict |= c == C_DICT_BP;
        any_auto |= c == 0;
    }
    Dictionary dict;
    bool have_dict = false;
    if (want_dict || (any_auto && dtype != D_BYTES && dtype != D_F64)) {
        const uint64_t limit = want_dict ? (1ull << 31) : (1ull << 16);
        have_dict = build_dictionary(dict, src, n_elems, dtype, limit, threads);
        ZF_REQUIRE(have_dict || !want_dict, ZF_E_UNSUPPORTED, "too many distinct values for DICT_BP");
    }

    // ZF_AUTO with a cost model: predicted (codec, schedule) per chunk
    std::vector<uint8_t> sched(ce.size(), 0);
    if (forced_sched)
        for (size_t i = 0; i < ce.size(); i++) sched[i] = forced_sched[i];
    if (any_auto) {
        CostModel model;
        std::string wpath = o.mlp_weights ? o.mlp_weights : "";
        if (wpath.empty())
            if (const char *e = std::getenv("ZF_MLP_WEIGHTS")) wpath = e;
        // the network's outputs cover the integer and byte codecs; float64
        // chunks keep the smallest stream
        if (!wpath.empty() && dtype != D_F64) {
            ZF_REQUIRE(model.load(wpath), ZF_E_INVALID, "cannot read cost model %s", wpath.c_str());
            std::vector<uint64_t> at(ce.size() + 1, 0);
            for (size_t i = 0; i < ce.size(); i++) at[i + 1] = at[i] + ce[i];
            std::vector<int> pick(ce.size(), -1), runner(ce.size(), -1);
            std::vector<float> gap(ce.size(), 0.f);
            parallel_for(ce.size(), threads, [&](uint64_t i) {
                if (cc[i] != 0) return;
                float x[kFeatures], y[kChoices];
                chunk_features(src + at[i] * es, ce[i], dtype, x);
                model.predict(x, y);
                int best = -1, second = -1;
                for (int c = 0; c < kChoices; c++) {
                    if (!choice_allowed(uint32_t(c), dtype, uint64_t(ce[i]) * es, have_dict)) continue;
                    if (best < 0 || y[c] < y[best]) {
                        second = best;
                        best = c;
                    } else if (second < 0 || y[c] < y[second]) {
                        second = c;
                    }
                }
                pick[i] = best;
                runner[i] = second;
                gap[i] = second >= 0 ? y[second] - y[best] : 0.f;
            });
            // near-ties (the two lowest predicted log times closer than the
            // margin): both candidates are timed on the device, the faster kept
            if (o.fallback_device >= 0 && o.fallback_margin > 0) {
                for (size_t i = 0; i < ce.size(); i++) {
                    if (pick[i] < 0 || runner[i] < 0 || !(gap[i] < o.fallback_margin)) continue;
                    const uint8_t *x = src + at[i] * es;
                    const int a = pick[i], b = runner[i];
                    const double ta = time_choice(x, ce[i], dtype, kChoiceCodec[a / 4], uint32_t(a % 4 + 1),
                                                  o.fallback_device, threads);
                    const double tb = time_choice(x, ce[i], dtype, kChoiceCodec[b / 4], uint32_t(b % 4 + 1),
                                                  o.fallback_device, threads);
                    if (tb < ta) pick[i] = b;
                }
            }
            std::vector<uint32_t> ce2;
            std::vector<uint8_t> cc2, sc2;
            for (size_t i = 0; i < ce.size(); i++) {
                if (pick[i] < 0) {
                    ce2.push_back(ce[i]);
                    cc2.push_back(cc[i]);
                    sc2.push_back(0);
                    continue;
                }
                const uint8_t codec = kChoiceCodec[pick[i] / 4], s = uint8_t(pick[i] % 4 + 1);
                if (codec == C_LZ77) {
                    // LZ77 schedules are chunk sizes: 8, 16, 32 or 64 KiB
                    const uint64_t per = std::max<uint64_t>(1, (8192ull << (s - 1)) / es);
                    for (uint64_t a = 0; a < ce[i]; a += per) {
                        ce2.push_back(uint32_t(std::min<uint64_t>(per, ce[i] - a)));
                        cc2.push_back(codec);
                        sc2.push_back(s);
                    }
                } else {
                    ce2.push_back(ce[i]);
                    cc2.push_back(codec);
                    sc2.push_back(s);
                }
            }
            ce.swap(ce2);
            cc.swap(cc2);
            sched.swap(sc2);
        }
    }

    // encode
    std::vector<uint64_t> first(ce.size() + 1, 0);
    for (size_t i = 0; i < ce.size(); i++) first[i + 1] = first[i] + ce[i];
    TokenDictionary tdict;
    bool want_tdict = false;
    for (auto c : cc) want_tdict |= c == C_SDICT_COL || c == C_SDICT_COL_ANS;
    if (want_tdict) build_token_dictionary(tdict, src, ce, cc, first, threads);
    std::vector<EncodedChunk> chunks(ce.size());
    parallel_for(ce.size(), threads, [&](uint64_t i) {
        static thread_local LzScratch sc_tl;
        LzScratch *sc = &sc_tl;
        const uint8_t *x = src + first[i] * es;
        EncodedChunk &out = chunks[i];
        out.n_elems = ce[i];
        out.sched = sched[i];
        if (cc[i] != 0) {
            out.codec = cc[i];
            encode_chunk(out.bytes, cc[i], dtype, x, ce[i], &dict, &tdict, *sc);
        } else {
            // smallest stream among the applicable codecs
            const uint32_t cands[] = {C_FOR_BP, C_DICT_BP, C_DELTA_BP, C_RLE_DELTA_BP, C_LZ77, C_F2I_BP, C_ANS,
                                      C_DSTRIDE_BP, C_SDICT_BP, C_SDICT_ANS};
            encode_chunk(out.bytes, C_PLAIN, dtype, x, ce[i], nullptr, nullptr, *sc);
            out.codec = C_PLAIN;
            std::vector<uint8_t> tmp;
            for (uint32_t c : cands) {
                if (!codec_allows(c, dtype)) continue;
                if (c == C_DICT_BP && !have_dict) continue;
                if (c == C_LZ77 && uint64_t(ce[i]) * es > kLzMaxChunk) continue;
                encode_chunk(tmp, c, dtype, x, ce[i], &dict, nullptr, *sc);
                if (tmp.size() < out.bytes.size()) {
                    out.bytes.swap(tmp);
                    out.codec = uint8_t(c);
                }
            }
        }
        ZF_REQUIRE(out.bytes.size() <= 0xFFFFFFFFull, ZF_E_UNSUPPORTED, "chunk stream above 4 GiB");
    });
    bool uses_dict = false;
    for (auto &c : chunks) uses_dict |= c.codec == C_DICT_BP;
    if (want_tdict)
        assemble_column(col->buf, o.pinned != 0, dtype, n_elems, chunks, tdict.area.data(), tdict.count,
                        tdict.area.size());
    else
        assemble_column(col->buf, o.pinned != 0, dtype, n_elems, chunks, uses_dict ? dict.bytes.data() : nullptr,
                        uses_dict ? dict.count : 0, uses_dict ? uint64_t(dict.count) * es : 0);
    col->view = parse_column(col->buf.p, col->buf.n);
}

}  // namespace zf
