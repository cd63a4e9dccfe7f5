// Chunk statistics for the learned (codec, schedule) choice, and the host
// side of the cost model: the network's forward pass and the argmin over the
// codecs a chunk admits.  Statistics come from the first 65,536 values (64 KiB
// for byte columns) of the chunk, so they cost a bounded amount per chunk.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <unordered_map>
#include <vector>

#include "features.hpp"

namespace zf {

static inline uint32_t bitw(uint64_t v) { return v ? 64u - uint32_t(__builtin_clzll(v)) : 0u; }
static inline float lg2(double x) { return float(std::log2(x)); }

// 64-bit key of element j (FIXED16 folded by a multiplicative hash).
static inline uint64_t key_at(const uint8_t *p, uint32_t es, uint64_t j) {
    const uint8_t *e = p + j * es;
    if (es == 4) return uint64_t(int64_t(int32_t(rd32(e))));
    if (es == 8) return rd64(e);
    if (es == 1) return e[0];
    return rd64(e) * 0x9E3779B97F4A7C15ull ^ rd64(e + 8);
}

void chunk_features(const void *srcv, uint64_t n, uint32_t dtype, float *f) {
    std::fill(f, f + kFeatures, 0.f);
    const uint8_t *src = static_cast<const uint8_t *>(srcv);
    const uint32_t es = elem_size(dtype);
    const bool is_int = dtype == D_I32 || dtype == D_I64;
    const bool text = dtype == D_BYTES;
    const uint64_t m = std::min<uint64_t>(n, text ? 65536 : 65536);  // sampled values
    f[0] = lg2(double(n) + 1);
    f[1] = lg2(es);
    f[2] = text ? 1.f : 0.f;
    f[3] = lg2(double(m) + 1);
    f[28] = lg2(double(n) * es + 1);
    if (m == 0) return;

    // value range and FOR widths (integers, signed)
    if (is_int) {
        int64_t lo = int64_t(key_at(src, es, 0)), hi = lo;
        double wsum = 0;
        uint32_t wmax = 0, nb = 0;
        for (uint64_t b = 0; b < m; b += kForBlock) {
            int64_t bl = int64_t(key_at(src, es, b)), bh = bl;
            for (uint64_t j = b; j < std::min<uint64_t>(m, b + kForBlock); j++) {
                const int64_t v = int64_t(key_at(src, es, j));
                bl = std::min(bl, v);
                bh = std::max(bh, v);
            }
            lo = std::min(lo, bl);
            hi = std::max(hi, bh);
            const uint32_t w = bitw(uint64_t(bh) - uint64_t(bl));
            wsum += w;
            wmax = std::max(wmax, w);
            nb++;
        }
        f[4] = float(bitw(uint64_t(hi) - uint64_t(lo)));
        f[5] = float(wsum / nb);
        f[6] = float(wmax);
        f[24] = float((wsum / nb) / (8.0 * es));  // FOR_BP bits per plain bit
    }

    // distinct values, top frequencies, value entropy
    std::unordered_map<uint64_t, uint32_t> hist;
    hist.reserve(size_t(std::min<uint64_t>(m, 1 << 16)) * 2);
    for (uint64_t j = 0; j < m; j++) hist[key_at(src, es, j)]++;
    std::vector<uint32_t> counts;
    counts.reserve(hist.size());
    for (auto &kv : hist) counts.push_back(kv.second);
    std::sort(counts.begin(), counts.end(), std::greater<uint32_t>());
    const double dm = double(m);
    double ent = 0, top8 = 0;
    for (size_t i = 0; i < counts.size(); i++) {
        const double p = counts[i] / dm;
        ent -= p * std::log2(p);
        if (i < 8) top8 += p;
    }
    f[7] = lg2(double(counts.size()) + 1);
    f[8] = float(counts.size() / dm);
    f[9] = float(counts[0] / dm);
    f[10] = float(top8);
    f[12] = float(ent);
    f[25] = float((bitw(counts.size() > 1 ? counts.size() - 1 : 0) + 0.0) / (8.0 * es));

    // order-0 byte entropy over the sampled bytes
    {
        uint64_t bh[256] = {0};
        const uint64_t nbytes = m * es;
        for (uint64_t i = 0; i < nbytes; i++) bh[src[i]]++;
        double e = 0;
        for (int i = 0; i < 256; i++)
            if (bh[i]) {
                const double p = double(bh[i]) / double(nbytes);
                e -= p * std::log2(p);
            }
        f[11] = float(e);
    }

    // order, runs, deltas
    {
        uint64_t nondec = 0, runs = 1, run = 1, maxrun = 1, zeros = 0;
        int64_t dlo = 0, dhi = 0;
        double dabs = 0;
        for (uint64_t j = 1; j < m; j++) {
            const uint64_t a = key_at(src, es, j - 1), b = key_at(src, es, j);
            if (is_int ? int64_t(b) >= int64_t(a) : b >= a) nondec++;
            if (a == b) {
                run++;
                zeros++;
            } else {
                runs++;
                maxrun = std::max(maxrun, run);
                run = 1;
            }
            if (is_int) {
                const int64_t d = int64_t(b - a);
                if (j == 1) dlo = dhi = d;
                dlo = std::min(dlo, d);
                dhi = std::max(dhi, d);
                dabs += std::fabs(double(d));
            }
        }
        maxrun = std::max(maxrun, run);
        const double pairs = std::max<double>(1, double(m - 1));
        f[13] = float(nondec / pairs);
        f[14] = float(double(runs) / dm);
        f[15] = lg2(dm / double(runs));
        f[16] = lg2(double(maxrun));
        if (is_int) {
            const uint32_t dbits = bitw(uint64_t(dhi) - uint64_t(dlo));
            f[17] = float(dbits);
            f[18] = lg2(dabs / pairs + 1);
            f[26] = float(dbits / (8.0 * es));                          // DELTA_BP
            f[27] = float((double(runs) / dm) * (4.0 + dbits / 8.0) / es);  // RLE_DELTA_BP
        }
        f[19] = float(zeros / pairs);
    }

    // text shape and repeats of 4-byte prefixes (over the sampled bytes)
    {
        const uint64_t nbytes = m * es;
        uint64_t spaces = 0, tokens = 0;
        for (uint64_t i = 0; i < nbytes; i++) {
            const bool sp = src[i] == ' ' || src[i] == '\n';
            spaces += sp;
            if (!sp && (i == 0 || src[i - 1] == ' ' || src[i - 1] == '\n')) tokens++;
        }
        f[20] = tokens ? float(double(nbytes - spaces) / double(tokens)) : 0.f;
        f[21] = float(double(spaces) / double(nbytes));
        if (nbytes >= 8) {
            std::vector<uint32_t> seen(1u << 16, 0xFFFFFFFFu);
            uint64_t rep = 0;
            std::unordered_map<uint32_t, uint32_t> grams;
            for (uint64_t i = 0; i + 4 <= nbytes; i++) {
                uint32_t v;
                std::memcpy(&v, src + i, 4);
                const uint32_t h = (v * 2654435761u) >> 16;
                if (seen[h] != 0xFFFFFFFFu && std::memcmp(src + seen[h], src + i, 4) == 0) rep++;
                seen[h] = uint32_t(i);
            }
            f[22] = float(double(rep) / double(nbytes - 3));
            f[23] = float(std::max(0.05, 1.0 - 0.75 * f[22]));  // crude LZ77 size ratio
        }
    }
}

// ------------------------------------------------------------ the network
bool CostModel::load(const std::string &path) {
    std::ifstream in(path, std::ios::binary);
    if (!in) return false;
    char magic[8] = {0};
    in.read(magic, 8);
    if (std::memcmp(magic, "ZFMLP1\0\0", 8) != 0) return false;
    mean.resize(kFeatures);
    scale.resize(kFeatures);
    params.resize(kMlpParams);
    in.read(reinterpret_cast<char *>(mean.data()), sizeof(float) * kFeatures);
    in.read(reinterpret_cast<char *>(scale.data()), sizeof(float) * kFeatures);
    in.read(reinterpret_cast<char *>(params.data()), sizeof(float) * kMlpParams);
    ok = bool(in);
    return ok;
}

void CostModel::predict(const float *x, float *y) const {
    constexpr int NI = kFeatures, NH = 64, NO = kChoices;
    float z[NI], h1[NH], h2[NH];
    for (int i = 0; i < NI; i++) z[i] = (x[i] - mean[i]) * scale[i];
    const float *W1 = params.data(), *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH,
                *W3 = b2 + NH, *b3 = W3 + NO * NH;
    for (int j = 0; j < NH; j++) {
        float a = b1[j];
        for (int i = 0; i < NI; i++) a += W1[j * NI + i] * z[i];
        h1[j] = a > 0 ? a : 0;
    }
    for (int j = 0; j < NH; j++) {
        float a = b2[j];
        for (int i = 0; i < NH; i++) a += W2[j * NH + i] * h1[i];
        h2[j] = a > 0 ? a : 0;
    }
    for (int o = 0; o < NO; o++) {
        float a = b3[o];
        for (int i = 0; i < NH; i++) a += W3[o * NH + i] * h2[i];
        y[o] = a;
    }
}

// Codec of output column c (4 schedules each).
const uint8_t kChoiceCodec[6] = {C_PLAIN, C_FOR_BP, C_DICT_BP, C_DELTA_BP, C_RLE_DELTA_BP, C_LZ77};

bool choice_allowed(uint32_t choice, uint32_t dtype, uint64_t chunk_bytes, bool have_dict) {
    const uint32_t codec = kChoiceCodec[choice / 4];
    if (!codec_allows(codec, dtype)) return false;
    if (codec == C_DICT_BP && !have_dict) return false;
    (void)chunk_bytes;
    return true;
}

}  // namespace zf
