// Decode kernels for gfx950 (wave64).  Every unit of work is owned by one
// wavefront; waves never wait for each other, so a workgroup is just a
// bundle of independent waves and there is no barrier anywhere.
//
//  Fully-Parallel (Sec. 3.1, Sec. 4 "Scheduling Fully-Parallel"):
//    FOR+BP and Dict+BP.  A lane owns 16 contiguous output bytes per step
//    (4 x int32, 2 x int64 or 1 x CHAR(16)): the paper's C, sized for one
//    16-byte store.  The packed words a lane needs (at most 5) are read
//    straight from HBM; neighbouring lanes share words, which the L1 absorbs,
//    so HBM sees each payload byte once.  Dictionary lookup is fused into the
//    unpack (Sec. 3.2, Eq. 2): no intermediate code array.
//  Group-Parallel (Sec. 4 "Scheduling Group-Parallel for load balance"):
//    RLE + delta + BP.  A wave takes one group of 64 runs: lane l loads run
//    l, an exclusive wave scan of the counts gives each run's output offset
//    (the paper's presum, fused), an inclusive wave scan of the unpacked
//    deltas gives the run values.  Output is written in 64-wide windows; the
//    runs that start inside a window are walked with uniform readlanes, so the
//    work per window is proportional to its run count and long runs cost no
//    more than short ones.  Units are balanced by output count on the host.
//  Non-Parallel (Sec. 4 "Scheduling Non-Parallel towards SIMT"): LZ77, one
//    chunk per wavefront.  Lane i holds sequence i of a batch of 64; wave
//    scans give every sequence's output and literal positions at once.  When
//    the batch is flat (no match reads another sequence of the same batch)
//    all literals, then all matches, are copied in lockstep; otherwise the
//    batch is replayed in order, one sequence at a time.
#include <hip/hip_runtime.h>

#include "zf_device.hpp"

namespace zf {

#define ZF_DEV __device__ __forceinline__

// ------------------------------------------------------------ wave helpers
ZF_DEV uint32_t lane_id() { return __lane_id(); }

ZF_DEV uint32_t rl32(uint32_t v, uint32_t lane) {
    return uint32_t(__builtin_amdgcn_readlane(int(v), int(lane)));
}
ZF_DEV uint64_t rl64(uint64_t v, uint32_t lane) {
    return uint64_t(rl32(uint32_t(v), lane)) | (uint64_t(rl32(uint32_t(v >> 32), lane)) << 32);
}
template <class T>
ZF_DEV T rlT(T v, uint32_t lane) {
    if constexpr (sizeof(T) == 8) return T(rl64(uint64_t(v), lane));
    else return T(rl32(uint32_t(v), lane));
}
ZF_DEV uint32_t first32(uint32_t v) { return uint32_t(__builtin_amdgcn_readfirstlane(int(v))); }

// inclusive prefix sums across the 64 lanes (wrapping)
ZF_DEV uint32_t scan_add32(uint32_t x) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (l >= uint32_t(d)) x += y;
    }
    return x;
}
ZF_DEV uint64_t scan_add64(uint64_t x) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (l >= uint32_t(d)) x += y;
    }
    return x;
}
template <class T>
ZF_DEV T scan_addT(T x) {
    if constexpr (sizeof(T) == 8) return T(scan_add64(uint64_t(x)));
    else return T(scan_add32(uint32_t(x)));
}
ZF_DEV uint32_t wave_max32(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = max(x, uint32_t(__shfl_xor(x, d, 64)));
    return x;
}
ZF_DEV bool any(bool p) { return __ballot(p) != 0; }

// Orders this wave's global memory accesses for the compiler.  Lanes of one
// wavefront share one in-order path to the L1, so a load issued after a
// store of the same wave observes it; the fence only stops reordering.
ZF_DEV void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

ZF_DEV void flag(uint32_t *err, uint32_t bits) {
    if (lane_id() == 0) atomicOr(err, bits);
}

ZF_DEV uint32_t ld32u(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }
ZF_DEV uint64_t ld64u(const uint8_t *p) {
    return uint64_t(ld32u(p)) | (uint64_t(ld32u(p + 4)) << 32);
}

ZF_DEV uint32_t mask32(uint32_t w) { return w >= 32 ? 0xFFFFFFFFu : ((1u << w) - 1u); }
ZF_DEV uint64_t mask64(uint32_t w) { return w >= 64 ? ~0ull : ((1ull << w) - 1ull); }

// A lane's window of five packed words, kept in named registers (an array
// indexed by a per-lane value would be demoted to LDS or scratch).
struct Win {
    uint32_t w0, w1, w2, w3, w4;
};

// Word d (0..6) of the window; words past the fifth read as zero.
ZF_DEV uint32_t pick(const Win &v, uint32_t d) {
    uint32_t r = 0;
    r = d == 0 ? v.w0 : r;
    r = d == 1 ? v.w1 : r;
    r = d == 2 ? v.w2 : r;
    r = d == 3 ? v.w3 : r;
    r = d == 4 ? v.w4 : r;
    return r;
}

// Load the 5 packed words starting at word k0 (zero past nwords).
ZF_DEV Win load_window(const uint32_t *words, uint64_t k0, uint64_t nwords) {
    Win v;
    if (k0 + 5 <= nwords) {
        uint4 q;
        __builtin_memcpy(&q, words + k0, 16);  // dword aligned: one dwordx4 load
        v.w0 = q.x;
        v.w1 = q.y;
        v.w2 = q.z;
        v.w3 = q.w;
        v.w4 = words[k0 + 4];
    } else {
        v.w0 = k0 < nwords ? words[k0] : 0u;
        v.w1 = k0 + 1 < nwords ? words[k0 + 1] : 0u;
        v.w2 = k0 + 2 < nwords ? words[k0 + 2] : 0u;
        v.w3 = k0 + 3 < nwords ? words[k0 + 3] : 0u;
        v.w4 = k0 + 4 < nwords ? words[k0 + 4] : 0u;
    }
    return v;
}

// Field at bit `pos` (0 <= pos < 128) of the window, width w <= 32.
ZF_DEV uint32_t field32(const Win &wv, uint32_t pos, uint32_t w) {
    const uint32_t d = pos >> 5, s = pos & 31u;
    const uint64_t pair = uint64_t(pick(wv, d)) | (uint64_t(pick(wv, d + 1)) << 32);
    return uint32_t(pair >> s) & mask32(w);
}
// Field at bit `pos` (0 <= pos < 96) of the window, width w <= 64.
ZF_DEV uint64_t field64(const Win &wv, uint32_t pos, uint32_t w) {
    const uint32_t d = pos >> 5, s = pos & 31u;
    const uint64_t lo = uint64_t(pick(wv, d)) | (uint64_t(pick(wv, d + 1)) << 32);
    const uint64_t hi = pick(wv, d + 2);
    const uint64_t v = s ? ((lo >> s) | (hi << (64 - s))) : lo;
    return v & mask64(w);
}

// ====================================================== Fully-Parallel
// One wave decodes blocks [t.a, t.a + t.b) of a FOR_BP or DICT_BP chunk.
// ES = output bytes per value; DICT = dictionary lookup fused after unpack.
template <int ES, bool DICT>
ZF_DEV void unit_fp(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    constexpr uint32_t VPL = 16 / ES;              // values per lane per step
    constexpr uint32_t BITS = (ES == 8 && !DICT) ? 64 : 32;
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t n = ck.n_elems, clen = ck.comp_len;
    const uint32_t nb = (n + kForBlock - 1) / kForBlock;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    const uint8_t *dict = A.dict + ck.dict_off;
    const uint32_t lane = lane_id();
    if (16ull * nb > clen || t.a + t.b > nb) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    bool bad = false;
    for (uint32_t b = t.a; b < t.a + t.b; b++) {
        const uint8_t *d = s + 16ull * b;
        const uint64_t ref = ld64u(d);
        const uint32_t w = ld32u(d + 8), poff = ld32u(d + 12);
        const uint32_t j0 = b * kForBlock;
        const uint32_t nv = min(kForBlock, n - j0);
        const uint64_t nwords = (uint64_t(nv) * w + 31) / 32;
        if (w > BITS || (poff & 15u) || poff < 16ull * nb || poff + 4 * nwords > clen) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t *words = reinterpret_cast<const uint32_t *>(s + poff);
        uint8_t *ob = out + uint64_t(j0) * ES;
        const bool vec = (reinterpret_cast<uintptr_t>(ob) & 15u) == 0;
        for (uint32_t v0 = lane * VPL; v0 < nv; v0 += 64 * VPL) {
            const uint64_t bit0 = uint64_t(v0) * w;
            const Win wv = load_window(words, bit0 >> 5, nwords);
            const uint32_t sh = uint32_t(bit0 & 31u);
            if constexpr (ES == 4) {
                uint32_t v[4];
#pragma unroll
                for (uint32_t i = 0; i < 4; i++) {
                    const uint32_t f = field32(wv, sh + i * w, w);
                    if constexpr (DICT) {
                        const uint32_t code = uint32_t(ref) + f;
                        const bool ok = code < ck.dict_count && v0 + i < nv;
                        bad |= (v0 + i < nv) && !ok;
                        v[i] = ok ? ld32u(dict + 4ull * code) : 0u;
                    } else {
                        v[i] = uint32_t(ref) + f;
                    }
                }
                if (vec && v0 + 4 <= nv) {
                    *reinterpret_cast<uint4 *>(ob + 4ull * v0) = make_uint4(v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (uint32_t i = 0; i < 4; i++)
                        if (v0 + i < nv) *reinterpret_cast<uint32_t *>(ob + 4ull * (v0 + i)) = v[i];
                }
            } else if constexpr (ES == 8) {
                uint64_t v[2];
#pragma unroll
                for (uint32_t i = 0; i < 2; i++) {
                    if constexpr (DICT) {
                        const uint32_t code = uint32_t(ref) + field32(wv, sh + i * w, w);
                        const bool ok = code < ck.dict_count && v0 + i < nv;
                        bad |= (v0 + i < nv) && !ok;
                        v[i] = ok ? ld64u(dict + 8ull * code) : 0ull;
                    } else {
                        v[i] = ref + field64(wv, sh + i * w, w);
                    }
                }
                if (vec && v0 + 2 <= nv) {
                    *reinterpret_cast<uint4 *>(ob + 8ull * v0) =
                        make_uint4(uint32_t(v[0]), uint32_t(v[0] >> 32), uint32_t(v[1]), uint32_t(v[1] >> 32));
                } else {
#pragma unroll
                    for (uint32_t i = 0; i < 2; i++)
                        if (v0 + i < nv) {
                            uint32_t *o = reinterpret_cast<uint32_t *>(ob + 8ull * (v0 + i));
                            o[0] = uint32_t(v[i]);
                            o[1] = uint32_t(v[i] >> 32);
                        }
                }
            } else {  // ES == 16: dictionary of CHAR(16)
                const uint32_t code = uint32_t(ref) + field32(wv, sh, w);
                const bool ok = code < ck.dict_count;
                bad |= !ok;
                uint4 e = make_uint4(0, 0, 0, 0);
                if (ok) e = *reinterpret_cast<const uint4 *>(dict + 16ull * code);
                if (vec) {
                    *reinterpret_cast<uint4 *>(ob + 16ull * v0) = e;
                } else {
                    uint32_t *o = reinterpret_cast<uint32_t *>(ob + 16ull * v0);
                    o[0] = e.x;
                    o[1] = e.y;
                    o[2] = e.z;
                    o[3] = e.w;
                }
            }
        }
    }
    if (any(bad)) flag(A.err, ERR_CORRUPT);
}

// ===================================================== Group-Parallel
// One wave writes elements [t.b, t.c) of an RLE_DELTA_BP / DELTA_BP chunk,
// starting at group t.a.
template <class T>
ZF_DEV void unit_rle(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    using U = T;  // unsigned value type: uint32_t or uint64_t
    constexpr uint32_t BITS = sizeof(T) * 8;
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t n = ck.n_elems, clen = ck.comp_len, lane = lane_id();
    const bool unit_runs = ck.codec == C_DELTA_BP;
    U *out = reinterpret_cast<U *>(A.out_tab[ck.col] + ck.out_off);
    if (clen < 16) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t nr = ld32u(s), ng = ld32u(s + 4), roff = ld32u(s + 8);
    bool hdr_ok = ng == (uint64_t(nr) + kRleGroup - 1) / kRleGroup && 16ull + 32ull * ng <= clen;
    if (unit_runs) hdr_ok = hdr_ok && nr == n && roff == 0;
    else hdr_ok = hdr_ok && (roff & 3u) == 0 && roff >= 16ull + 32ull * ng && roff + 4ull * nr <= clen;
    const uint32_t e0 = t.b, e1 = t.c;
    if (!hdr_ok || e1 > n || e0 >= e1) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t *runs = reinterpret_cast<const uint32_t *>(s + roff);
    for (uint32_t g = t.a;; g++) {
        if (g >= ng) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint8_t *rec = s + 16 + 32ull * g;
        const uint32_t goff = ld32u(rec), w = ld32u(rec + 4), doff = ld32u(rec + 8);
        const U base = U(ld64u(rec + 16)), dmin = U(ld64u(rec + 24));
        const uint32_t cnt = min(kRleGroup, nr - g * kRleGroup);
        const uint64_t nwords = (uint64_t(cnt - 1) * w + 31) / 32;
        const uint32_t next_off = (g + 1 < ng) ? ld32u(rec + 32) : n;
        if (w > BITS || (doff & 3u) || doff + 4 * nwords > clen || (g == t.a && goff > e0) ||
            next_off > n) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        // run lengths -> output offsets (exclusive scan = presum)
        const bool act = lane < cnt;
        const uint32_t r = act ? (unit_runs ? 1u : runs[uint64_t(g) * kRleGroup + lane]) : 0u;
        const uint64_t incl = scan_add64(r);
        const uint64_t total = rl64(incl, cnt - 1);
        if (any(act && r == 0) || uint64_t(goff) + total != next_off) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t end_abs = goff + uint32_t(incl);  // end of run `lane`
        // run values: base, then base + prefix sums of (dmin + field)
        U delta = base;
        if (lane >= 1 && act) {
            const uint64_t bit = uint64_t(lane - 1) * w;
            const uint32_t *words = reinterpret_cast<const uint32_t *>(s + doff);
            const uint64_t k = bit >> 5;
            const uint32_t sh = uint32_t(bit & 31u);
            const uint32_t w0 = k < nwords ? words[k] : 0u;
            const uint32_t w1 = k + 1 < nwords ? words[k + 1] : 0u;
            U f;
            if constexpr (BITS == 32) {
                f = uint32_t((uint64_t(w0) | (uint64_t(w1) << 32)) >> sh) & mask32(w);
            } else {
                const uint32_t w2 = k + 2 < nwords ? words[k + 2] : 0u;
                const uint64_t lo = uint64_t(w0) | (uint64_t(w1) << 32);
                f = (sh ? ((lo >> sh) | (uint64_t(w2) << (64 - sh))) : lo) & mask64(w);
            }
            delta = U(dmin + f);
        }
        const U v = scan_addT<U>(act ? delta : U(0));
        // expand the part of this group inside [e0, e1)
        const uint32_t a = max(e0, goff), bnd = min(e1, next_off);
        if (a < bnd) {
            uint32_t j = uint32_t(__popcll(__ballot(act && end_abs <= a)));  // run holding a
            for (uint32_t W0 = a; W0 < bnd; W0 += 64) {
                const uint32_t wend = W0 + 64, p = W0 + lane;
                U val = rlT<U>(v, j);
                uint32_t k = j;
                while (k + 1 < cnt) {
                    const uint32_t st = rl32(end_abs, k);  // start of run k+1
                    if (st >= wend) break;
                    k++;
                    if (p >= st) val = rlT<U>(v, k);
                }
                if (p < bnd) out[p] = val;
                j = (rl32(end_abs, k) <= wend) ? k + 1 : k;
            }
        }
        if (next_off >= e1) return;
    }
}

// ======================================================== Non-Parallel
// One wave decodes one whole LZ77 chunk.
ZF_DEV void unit_lz(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t clen = ck.comp_len, lane = lane_id();
    const uint32_t es = ck.dtype == D_I32 ? 4 : ck.dtype == D_I64 ? 8 : ck.dtype == D_FIXED16 ? 16 : 1;
    const uint32_t plain = ck.n_elems * es;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    if (clen < 16) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t nseq = ld32u(s), nlit = ld32u(s + 4), next = ld32u(s + 8), plen = ld32u(s + 12);
    if (plen != plain || plain > kLzMaxChunk ||
        16ull + 3ull * nseq + 2ull * next + nlit != uint64_t(clen)) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint16_t *offs = reinterpret_cast<const uint16_t *>(s + 16);
    const uint16_t *ext = offs + nseq;
    const uint8_t *tags = reinterpret_cast<const uint8_t *>(ext + next);
    const uint8_t *lits = tags + nseq;
    uint32_t pos = 0, lp = 0, ep = 0;
    for (uint32_t base = 0; base < nseq; base += 64) {
        const uint32_t i = base + lane;
        const bool act = i < nseq;
        const uint32_t tag = act ? tags[i] : 0u;
        const uint32_t off = act ? offs[i] : 0u;
        const uint32_t lc = tag & 7u, mc = tag >> 3;
        const uint32_t ne = (lc == 7u) + (mc == 31u);
        const uint32_t eincl = scan_add32(ne);
        const uint32_t eex = ep + eincl - ne, etot = rl32(eincl, 63);
        if (uint64_t(ep) + etot > next) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        uint32_t ll = lc, ml = 0;
        if (lc == 7u) ll = 7u + ext[eex];
        if (mc == 31u) ml = 34u + ext[eex + (lc == 7u)];
        else if (mc) ml = mc + 3u;
        const uint32_t len = ll + ml;
        const uint32_t pincl = scan_add32(len), lincl = scan_add32(ll);
        const uint32_t P = pos + pincl - len, LP = lp + lincl - ll;
        const uint32_t total = rl32(pincl, 63), ltot = rl32(lincl, 63);
        const uint32_t D = P + ll;
        const bool bad = act && (uint64_t(P) + len > plain || uint64_t(LP) + ll > nlit ||
                                 (ml == 0 ? off != 0 : (off == 0 || off > D)));
        if (any(bad)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t q0 = D - off;  // first source byte of the match
        const bool flat = ml == 0 || q0 + min(ml, off) <= pos || q0 >= P;
        if (!any(!flat)) {
            // literals of all 64 sequences, in lockstep, 4 bytes per round
            const uint32_t mll = wave_max32(ll);
            for (uint32_t t0 = 0; t0 < mll; t0 += 4) {
                uint8_t b[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; u++)
                    if (t0 + u < ll) b[u] = lits[LP + t0 + u];
#pragma unroll
                for (uint32_t u = 0; u < 4; u++)
                    if (t0 + u < ll) out[P + t0 + u] = b[u];
            }
            wave_fence();
            // then all matches; sources are final bytes (before the batch or
            // this sequence's literals), so loads never wait on this pass
            const uint32_t mml = wave_max32(ml);
            uint32_t src = q0;
            for (uint32_t t0 = 0; t0 < mml; t0 += 4) {
                uint8_t b[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; u++) {
                    if (t0 + u < ml) b[u] = out[src];
                    src = (src + 1 == D) ? q0 : src + 1;  // repeat the period
                }
#pragma unroll
                for (uint32_t u = 0; u < 4; u++)
                    if (t0 + u < ml) out[D + t0 + u] = b[u];
            }
            wave_fence();
        } else {
            // in-order replay of this batch
            const uint32_t cntb = min(64u, nseq - base);
            for (uint32_t k = 0; k < cntb; k++) {
                const uint32_t Pk = rl32(P, k), llk = rl32(ll, k), LPk = rl32(LP, k);
                const uint32_t mlk = rl32(ml, k), offk = rl32(off, k), Dk = Pk + llk;
                for (uint32_t x = lane; x < llk; x += 64) out[Pk + x] = lits[LPk + x];
                wave_fence();
                const uint32_t step = min(offk, 64u);
                for (uint32_t j0 = 0; j0 < mlk; j0 += step) {
                    const uint32_t j = j0 + lane;
                    if (lane < step && j < mlk) out[Dk + j] = out[Dk - offk + j];
                    wave_fence();
                }
            }
        }
        pos += total;
        lp += ltot;
        ep += etot;
    }
    if (pos != plain || lp != nlit || ep != next) flag(A.err, ERR_CORRUPT);
}

// ================================================================ PLAIN
ZF_DEV void unit_plain(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    const uint8_t *src = A.comp + ck.comp_off;
    uint8_t *dst = A.out_tab[ck.col] + ck.out_off;
    const uint32_t a = t.a, b = min(t.b, ck.comp_len), lane = lane_id();
    if (((reinterpret_cast<uintptr_t>(src + a) | reinterpret_cast<uintptr_t>(dst + a)) & 15u) == 0) {
        const uint32_t nvec = (b - a) / 16;
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src + a);
        uint4 *d4 = reinterpret_cast<uint4 *>(dst + a);
        for (uint32_t i = lane; i < nvec; i += 64) d4[i] = s4[i];
        for (uint32_t i = a + nvec * 16 + lane; i < b; i += 64) dst[i] = src[i];
    } else {
        for (uint32_t i = a + lane; i < b; i += 64) dst[i] = src[i];
    }
}

// ============================================================== dispatch
ZF_DEV void run_unit(const LaunchArgs &A, uint32_t kind, uint32_t u) {
    const Tile t = A.tiles[u];
    const ChunkDesc ck = A.chunks[t.chunk];
    switch (kind) {
    case K_PLAIN: unit_plain(A, t, ck); break;
    case K_FOR32: unit_fp<4, false>(A, t, ck); break;
    case K_FOR64: unit_fp<8, false>(A, t, ck); break;
    case K_DICT32: unit_fp<4, true>(A, t, ck); break;
    case K_DICT64: unit_fp<8, true>(A, t, ck); break;
    case K_DICT128: unit_fp<16, true>(A, t, ck); break;
    case K_RLE32: unit_rle<uint32_t>(A, t, ck); break;
    case K_RLE64: unit_rle<uint64_t>(A, t, ck); break;
    case K_LZ: unit_lz(A, t, ck); break;
    }
}

// One launch per kind: wave w of block b takes unit begin + b*waves + w.
template <uint32_t KIND>
__global__ __launch_bounds__(1024) void k_decode_kind(LaunchArgs A) {
    const uint32_t waves = blockDim.x / 64;
    const uint32_t u = A.kind_begin[KIND] + blockIdx.x * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[KIND + 1]) return;
    run_unit(A, KIND, u);
}

// Persistent: every wave pulls units from one queue until it is empty.
// Units are ordered by kind, the costliest kinds first.
__global__ __launch_bounds__(256) void k_decode_persistent(LaunchArgs A) {
    const uint32_t n = A.kind_begin[K_COUNT];
    for (;;) {
        uint32_t u = 0;
        if (lane_id() == 0) u = atomicAdd(A.counter, 1u);
        u = first32(u);
        if (u >= n) return;
        uint32_t kind = 0;
        while (kind + 1 < K_COUNT && u >= A.kind_begin[kind + 1]) kind++;
        run_unit(A, kind, u);
    }
}

__global__ void k_zero_counter(uint32_t *c) { *c = 0; }

struct OutTable {
    uint8_t *p[kMaxCols];
};
__global__ void k_set_out_tab(uint8_t **tab, OutTable t, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tab[i] = t.p[i];
}

// ============================================================ host side
hipError_t launch_set_out_tab(uint8_t **d_tab, uint8_t *const *ptrs, uint32_t n, hipStream_t st) {
    OutTable t{};
    for (uint32_t i = 0; i < n && i < kMaxCols; i++) t.p[i] = ptrs[i];
    hipLaunchKernelGGL(k_set_out_tab, dim3(1), dim3(kMaxCols), 0, st, d_tab, t, n);
    return hipGetLastError();
}

template <uint32_t K>
static void launch_kind(const LaunchArgs &A, uint32_t waves, hipStream_t st) {
    const uint32_t n = A.kind_begin[K + 1] - A.kind_begin[K];
    if (!n) return;
    hipLaunchKernelGGL(k_decode_kind<K>, dim3((n + waves - 1) / waves), dim3(64 * waves), 0, st, A);
}

// Enqueue the decode of one launch's units.  persistent_waves > 0 selects
// the persistent kernel with that many waves in flight.
hipError_t launch_decode(const LaunchArgs &A, uint32_t persistent_waves, uint32_t waves_per_block,
                         hipStream_t st) {
    if (A.kind_begin[K_COUNT] == 0) return hipSuccess;
    if (persistent_waves) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, A.counter);
        const uint32_t blocks = (persistent_waves + 3) / 4;
        hipLaunchKernelGGL(k_decode_persistent, dim3(blocks), dim3(256), 0, st, A);
        return hipGetLastError();
    }
    const uint32_t wpb = waves_per_block ? waves_per_block : 4;
    launch_kind<K_LZ>(A, wpb, st);
    launch_kind<K_RLE32>(A, wpb, st);
    launch_kind<K_RLE64>(A, wpb, st);
    launch_kind<K_DICT128>(A, wpb, st);
    launch_kind<K_DICT64>(A, wpb, st);
    launch_kind<K_DICT32>(A, wpb, st);
    launch_kind<K_FOR64>(A, wpb, st);
    launch_kind<K_FOR32>(A, wpb, st);
    launch_kind<K_PLAIN>(A, wpb, st);
    return hipGetLastError();
}

}  // namespace zf
