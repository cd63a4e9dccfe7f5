// Decode routines for gfx950 (wave64), shared by the kernel translation units.  Every unit of work is owned by one
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
//    deltas gives the run values.  Output is written in windows of 64 lanes x
//    16 bytes: every run starting in a window marks its start in an LDS slot,
//    a wave max-scan carries the latest run over the window and each lane
//    fetches its run's value with a cross-lane permute, so a window costs the
//    same whatever its run count.  Units are balanced by output count on the
//    host.
//  String dictionary (Sec. 5.3) is a Group-Parallel expansion too: a wave
//    takes groups of 64 tokens, scans their lengths for output offsets and
//    gathers each token's bytes into a per-wave LDS staging buffer that is
//    written back in aligned 16-byte stores.
//  Non-Parallel (Sec. 4 "Scheduling Non-Parallel towards SIMT"): LZ77, one
//    chunk per wavefront.  Lane i holds sequence i of a batch of 64; wave
//    scans give every sequence's output and literal positions at once.  When
//    the batch is flat (no match reads another sequence of the same batch)
//    all literals, then all matches, are copied in lockstep; otherwise the
//    batch is replayed in order, one sequence at a time.
#pragma once
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
// A pointer that every lane holds the same value of, moved to scalar
// registers: a buffer resource built from a pointer the compiler cannot
// prove uniform (one read from memory) is otherwise wrapped in a loop over
// the distinct values, around every load through it.
template <class T>
ZF_DEV T *uniform_ptr(T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint64_t u = (uint64_t(first32(uint32_t(v >> 32))) << 32) | first32(uint32_t(v));
    return reinterpret_cast<T *>(u);
}

// Inclusive prefix sums across the 64 lanes (wrapping), with DPP lane moves:
// row_shr 1, 2, 4, 8 inside each row of 16 lanes, then row_bcast 15 and 31
// carry the row totals into the rows above (GCN / CDNA DPP controls).
template <int CTRL, int ROWS>
ZF_DEV uint32_t dpp(uint32_t x) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROWS, 0xF, true));
}
ZF_DEV uint32_t scan_add32(uint32_t x) {
    x += dpp<0x111, 0xF>(x);   // row_shr:1
    x += dpp<0x112, 0xF>(x);   // row_shr:2
    x += dpp<0x114, 0xF>(x);   // row_shr:4
    x += dpp<0x118, 0xF>(x);   // row_shr:8
    x += dpp<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}
// 64-bit version: the same moves on both halves, with the carry of each add.
template <int CTRL, int ROWS>
ZF_DEV void add64_dpp(uint32_t &lo, uint32_t &hi) {
    const uint32_t ylo = dpp<CTRL, ROWS>(lo), yhi = dpp<CTRL, ROWS>(hi);
    const uint32_t nlo = lo + ylo;
    hi = hi + yhi + (nlo < lo ? 1u : 0u);
    lo = nlo;
}
ZF_DEV uint64_t scan_add64(uint64_t x) {
    uint32_t lo = uint32_t(x), hi = uint32_t(x >> 32);
    add64_dpp<0x111, 0xF>(lo, hi);
    add64_dpp<0x112, 0xF>(lo, hi);
    add64_dpp<0x114, 0xF>(lo, hi);
    add64_dpp<0x118, 0xF>(lo, hi);
    add64_dpp<0x142, 0xA>(lo, hi);
    add64_dpp<0x143, 0xC>(lo, hi);
    return uint64_t(lo) | (uint64_t(hi) << 32);
}
template <class T>
ZF_DEV T scan_addT(T x) {
    if constexpr (sizeof(T) == 8) return T(scan_add64(uint64_t(x)));
    else return T(scan_add32(uint32_t(x)));
}
// The x of the highest lane below this one whose x is nonzero, or `carry`
// where there is none; `carry` then becomes the x of the wave's highest lane
// with a nonzero x (unchanged if there is none).  A ballot finds the lane,
// one cross-lane read fetches its x.
ZF_DEV uint32_t last_nonzero_below(uint32_t x, uint32_t &carry) {
    const uint64_t m = __ballot(x != 0);
    const uint64_t b = m & ((uint64_t(1) << __lane_id()) - 1);
    const uint32_t hi = uint32_t(b >> 32), lo = uint32_t(b);
    const uint32_t src = hi ? 63u - uint32_t(__clz(int(hi))) : 31u - uint32_t(__clz(int(lo)));
    const uint32_t got = uint32_t(__builtin_amdgcn_ds_bpermute(int(src * 4), int(x)));
    const uint32_t r = b ? got : carry;
    if (m) carry = uint32_t(__builtin_amdgcn_readlane(int(x), 63 - __builtin_clzll(m)));
    return r;
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
// Cache policy of a buffer store that bypasses the caches' normal
// retention (the nt bit of the instruction).
constexpr int kNonTemporal = 2;

ZF_DEV void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

ZF_DEV void flag(uint32_t *err, uint32_t bits) {
    if (lane_id() == 0) atomicOr(err, bits);
}

ZF_DEV uint32_t ld32u(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }
ZF_DEV uint64_t ld64u(const uint8_t *p) {
    return uint64_t(ld32u(p)) | (uint64_t(ld32u(p + 4)) << 32);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
#define ZF_GLOBAL __attribute__((address_space(1)))
// Every buffer the kernels touch is device global memory; saying so lets the
// compiler use global (not flat) loads and stores.
template <class T>
ZF_DEV ZF_GLOBAL T *gp(T *p) {
    return (ZF_GLOBAL T *)(p);
}
template <class T>
ZF_DEV const ZF_GLOBAL T *gp(const T *p) {
    return (const ZF_GLOBAL T *)(p);
}
// 16-byte store of streaming output (not read again by this kernel).
ZF_DEV void st16_nt(uint8_t *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    u32x4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, gp(reinterpret_cast<u32x4 *>(p)));
}
ZF_DEV void st4(uint8_t *p, uint32_t v) { *gp(reinterpret_cast<uint32_t *>(p)) = v; }

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
ZF_DEV uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// A Float2Int integer (two's complement in 64 bits) as the bits of the
// float64 (double)d / div: IEEE conversion and division, round to nearest.
ZF_DEV uint64_t f2i_value(uint64_t d, double div) {
    const double v = double(int64_t(d)) / div;
    return uint64_t(__double_as_longlong(v));
}

// The NW packed words starting at word k0 (NW <= 5, known per width);
// zero past nwords.
template <uint32_t NW>
ZF_DEV Win load_words(const uint32_t *words, uint64_t k0, uint64_t nwords) {
    Win v{0, 0, 0, 0, 0};
    const ZF_GLOBAL uint32_t *g = gp(words) + k0;
    if (k0 + NW <= nwords) {
        if constexpr (NW >= 4) {
            u32x4 q;
            __builtin_memcpy(&q, (const uint32_t *)g, 16);
            v.w0 = q.x; v.w1 = q.y; v.w2 = q.z; v.w3 = q.w;
            if constexpr (NW == 5) v.w4 = g[4];
        } else if constexpr (NW == 3) {
            u32x3 q;
            __builtin_memcpy(&q, (const uint32_t *)g, 12);
            v.w0 = q.x; v.w1 = q.y; v.w2 = q.z;
        } else if constexpr (NW == 2) {
            u32x2 q;
            __builtin_memcpy(&q, (const uint32_t *)g, 8);
            v.w0 = q.x; v.w1 = q.y;
        } else if constexpr (NW == 1) {
            v.w0 = g[0];
        }
    } else {
        if constexpr (NW >= 1) v.w0 = k0 < nwords ? g[0] : 0u;
        if constexpr (NW >= 2) v.w1 = k0 + 1 < nwords ? g[1] : 0u;
        if constexpr (NW >= 3) v.w2 = k0 + 2 < nwords ? g[2] : 0u;
        if constexpr (NW >= 4) v.w3 = k0 + 3 < nwords ? g[3] : 0u;
        if constexpr (NW >= 5) v.w4 = k0 + 4 < nwords ? g[4] : 0u;
    }
    return v;
}

// Word K (compile time) of the 128-bit value Y = window >> sh.
template <uint32_t K>
ZF_DEV uint32_t yword(const Win &v, uint32_t sh) {
    if constexpr (K == 0) return alignbit(v.w1, v.w0, sh);
    else if constexpr (K == 1) return alignbit(v.w2, v.w1, sh);
    else if constexpr (K == 2) return alignbit(v.w3, v.w2, sh);
    else if constexpr (K == 3) return alignbit(v.w4, v.w3, sh);
    else return 0u;
}
// Field I of width W (W <= 32) of Y: bits [I*W, I*W + W).
template <uint32_t W, uint32_t I>
ZF_DEV uint32_t yfield32(const Win &v, uint32_t sh) {
    if constexpr (W == 0) {
        return 0u;
    } else {
        constexpr uint32_t pos = I * W, k = pos >> 5, s = pos & 31;
        constexpr uint32_t m = W == 32 ? 0xFFFFFFFFu : ((1u << W) - 1u);
        if constexpr (s + W <= 32) return (yword<k>(v, sh) >> s) & m;
        else return alignbit(yword<k + 1>(v, sh), yword<k>(v, sh), s) & m;
    }
}
// Field I of width W (W <= 64) of Y, as 64 bits.
template <uint32_t W, uint32_t I>
ZF_DEV uint64_t yfield64(const Win &v, uint32_t sh) {
    if constexpr (W == 0) {
        return 0ull;
    } else {
        constexpr uint32_t pos = I * W, k = pos >> 5, s = pos & 31;
        constexpr uint64_t m = W == 64 ? ~0ull : ((1ull << W) - 1ull);
        const uint32_t lo = s ? alignbit(yword<k + 1>(v, sh), yword<k>(v, sh), s) : yword<k>(v, sh);
        const uint32_t hi = s ? alignbit(yword<k + 2>(v, sh), yword<k + 1>(v, sh), s) : yword<k + 1>(v, sh);
        return (uint64_t(lo) | (uint64_t(hi) << 32)) & m;
    }
}

// Decode one block of nv values, width W known at compile time.  A lane owns
// 16 output bytes per step; the packed words of UNR steps are loaded before
// any is used, so each wave keeps UNR x 1 KiB of output's loads in flight.
// F2I: the 64-bit values are Float2Int integers, written as the float64
// (double)int64(value) / div.
// LDS: the dictionary was copied into this wave's LDS (dict points there).
template <int ES, bool DICT, uint32_t UNR, uint32_t W, bool F2I = false, bool LDS = false>
ZF_DEV void fp_block(const uint32_t *words, uint64_t nwords, uint64_t ref, uint32_t nv,
                     uint8_t *ob, bool vec, const uint8_t *dict, uint32_t dict_count, bool &bad,
                     double div = 1.0) {
    constexpr uint32_t VPL = 16 / ES;
    constexpr uint32_t NW = (31 + VPL * W + 31) / 32;  // words a lane may need
    const uint32_t lane = lane_id();
    const uint32_t steps = (nv + 64 * VPL - 1) / (64 * VPL);
    const ZF_GLOBAL uint8_t *gd = gp(dict);
    for (uint32_t g = 0; g < steps; g += UNR) {
        Win wv[UNR];
#pragma unroll
        for (uint32_t u = 0; u < UNR; u++) {
            const uint32_t v0 = ((g + u) * 64 + lane) * VPL;
            if (v0 < nv) wv[u] = load_words<NW>(words, (uint64_t(v0) * W) >> 5, nwords);
        }
#pragma unroll
        for (uint32_t u = 0; u < UNR; u++) {
            const uint32_t v0 = ((g + u) * 64 + lane) * VPL;
            if (v0 >= nv) continue;
            const uint32_t sh = uint32_t((uint64_t(v0) * W) & 31u);
            if constexpr (ES == 4) {
                uint32_t f[4] = {yfield32<W, 0>(wv[u], sh), yfield32<W, 1>(wv[u], sh),
                                 yfield32<W, 2>(wv[u], sh), yfield32<W, 3>(wv[u], sh)};
                uint32_t v[4];
#pragma unroll
                for (uint32_t i = 0; i < 4; i++) {
                    if constexpr (DICT && LDS) {
                        const uint32_t code = uint32_t(ref) + f[i];
                        const bool in = v0 + i < nv, ok = code < dict_count;
                        bad |= in && !ok;
                        const uint32_t x = *reinterpret_cast<const uint32_t *>(dict + 4 * (ok ? code : 0u));
                        v[i] = (in && ok) ? x : 0u;
                    } else if constexpr (DICT) {
                        const uint32_t code = uint32_t(ref) + f[i];
                        const bool in = v0 + i < nv, ok = code < dict_count;
                        bad |= in && !ok;
                        v[i] = (in && ok) ? *reinterpret_cast<const ZF_GLOBAL uint32_t *>(gd + 4ull * code) : 0u;
                    } else {
                        v[i] = uint32_t(ref) + f[i];
                    }
                }
                if (vec && v0 + 4 <= nv) {
                    st16_nt(ob + 4ull * v0, v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (uint32_t i = 0; i < 4; i++)
                        if (v0 + i < nv) st4(ob + 4ull * (v0 + i), v[i]);
                }
            } else if constexpr (ES == 8) {
                uint64_t v[2];
                if constexpr (DICT) {
                    const uint32_t f[2] = {yfield32<W, 0>(wv[u], sh), yfield32<W, 1>(wv[u], sh)};
#pragma unroll
                    for (uint32_t i = 0; i < 2; i++) {
                        const uint32_t code = uint32_t(ref) + f[i];
                        const bool in = v0 + i < nv, ok = code < dict_count;
                        bad |= in && !ok;
                        if constexpr (LDS) {
                            const uint64_t x = *reinterpret_cast<const uint64_t *>(dict + 8 * (ok ? code : 0u));
                            v[i] = (in && ok) ? x : 0ull;
                        } else {
                            v[i] = (in && ok) ? *reinterpret_cast<const ZF_GLOBAL uint64_t *>(gd + 8ull * code) : 0ull;
                        }
                    }
                } else {
                    v[0] = ref + yfield64<W, 0>(wv[u], sh);
                    v[1] = ref + yfield64<W, 1>(wv[u], sh);
                    if constexpr (F2I) {
                        v[0] = f2i_value(v[0], div);
                        v[1] = f2i_value(v[1], div);
                    }
                }
                if (vec && v0 + 2 <= nv) {
                    st16_nt(ob + 8ull * v0, uint32_t(v[0]), uint32_t(v[0] >> 32), uint32_t(v[1]),
                            uint32_t(v[1] >> 32));
                } else {
#pragma unroll
                    for (uint32_t i = 0; i < 2; i++)
                        if (v0 + i < nv) {
                            st4(ob + 8ull * (v0 + i), uint32_t(v[i]));
                            st4(ob + 8ull * (v0 + i) + 4, uint32_t(v[i] >> 32));
                        }
                }
            } else {  // ES == 16: dictionary of CHAR(16)
                const uint32_t code = uint32_t(ref) + yfield32<W, 0>(wv[u], sh);
                const bool ok = code < dict_count;
                bad |= !ok;
                u32x4 e = {0, 0, 0, 0};
                if constexpr (LDS) {
                    const u32x4 x = *reinterpret_cast<const u32x4 *>(dict + 16 * (ok ? code : 0u));
                    e = ok ? x : e;
                } else if (ok) {
                    e = *reinterpret_cast<const ZF_GLOBAL u32x4 *>(gd + 16ull * code);
                }
                if (vec) {
                    st16_nt(ob + 16ull * v0, e.x, e.y, e.z, e.w);
                } else {
                    st4(ob + 16ull * v0, e.x);
                    st4(ob + 16ull * v0 + 4, e.y);
                    st4(ob + 16ull * v0 + 8, e.z);
                    st4(ob + 16ull * v0 + 12, e.w);
                }
            }
        }
    }
}


// ---- runtime-width variant (persistent kernel): the same steps with the
// field positions computed at run time (uniform across the wave).
ZF_DEV uint32_t ysel(uint32_t y0, uint32_t y1, uint32_t y2, uint32_t y3, uint32_t k) {
    return k == 0 ? y0 : k == 1 ? y1 : k == 2 ? y2 : k == 3 ? y3 : 0u;
}
ZF_DEV uint64_t yfield_rt(uint32_t y0, uint32_t y1, uint32_t y2, uint32_t y3, uint32_t pos, uint32_t w) {
    const uint32_t k = pos >> 5, s = pos & 31;
    const uint32_t a = ysel(y0, y1, y2, y3, k), b = ysel(y0, y1, y2, y3, k + 1),
                   c = ysel(y0, y1, y2, y3, k + 2);
    const uint32_t lo = alignbit(b, a, s), hi = alignbit(c, b, s);
    const uint64_t v = uint64_t(lo) | (uint64_t(hi) << 32);
    return w >= 64 ? v : (v & ((1ull << w) - 1ull));
}

template <int ES, bool DICT, bool F2I = false>
ZF_DEV void fp_block_rt(uint32_t w, const uint32_t *words, uint64_t nwords, uint64_t ref, uint32_t nv,
                        uint8_t *ob, bool vec, const uint8_t *dict, uint32_t dict_count, bool &bad,
                        double div = 1.0) {
    constexpr uint32_t VPL = 16 / ES;
    const uint32_t lane = lane_id();
    const ZF_GLOBAL uint8_t *gd = gp(dict);
    for (uint32_t v0 = lane * VPL; v0 < nv; v0 += 64 * VPL) {
        const Win wv = load_words<5>(words, (uint64_t(v0) * w) >> 5, nwords);
        const uint32_t sh = uint32_t((uint64_t(v0) * w) & 31u);
        const uint32_t y0 = yword<0>(wv, sh), y1 = yword<1>(wv, sh), y2 = yword<2>(wv, sh),
                       y3 = yword<3>(wv, sh);
        uint64_t v[VPL];
#pragma unroll
        for (uint32_t i = 0; i < VPL; i++) {
            const uint64_t f = yfield_rt(y0, y1, y2, y3, i * w, w);
            if constexpr (DICT) {
                const uint32_t code = uint32_t(ref) + uint32_t(f);
                const bool in = v0 + i < nv, ok = code < dict_count;
                bad |= in && !ok;
                v[i] = 0;
                if (in && ok) {
                    if constexpr (ES == 4) v[i] = *reinterpret_cast<const ZF_GLOBAL uint32_t *>(gd + 4ull * code);
                    if constexpr (ES == 8) v[i] = *reinterpret_cast<const ZF_GLOBAL uint64_t *>(gd + 8ull * code);
                }
                if constexpr (ES == 16) {
                    u32x4 e = {0, 0, 0, 0};
                    if (ok) e = *reinterpret_cast<const ZF_GLOBAL u32x4 *>(gd + 16ull * code);
                    if (vec) st16_nt(ob + 16ull * v0, e.x, e.y, e.z, e.w);
                    else {
                        st4(ob + 16ull * v0, e.x);
                        st4(ob + 16ull * v0 + 4, e.y);
                        st4(ob + 16ull * v0 + 8, e.z);
                        st4(ob + 16ull * v0 + 12, e.w);
                    }
                }
            } else {
                v[i] = ref + f;
                if constexpr (F2I) v[i] = f2i_value(v[i], div);
            }
        }
        if constexpr (ES == 4) {
            if (vec && v0 + 4 <= nv) st16_nt(ob + 4ull * v0, uint32_t(v[0]), uint32_t(v[1]), uint32_t(v[2]), uint32_t(v[3]));
            else
                for (uint32_t i = 0; i < 4; i++)
                    if (v0 + i < nv) st4(ob + 4ull * (v0 + i), uint32_t(v[i]));
        } else if constexpr (ES == 8) {
            if (vec && v0 + 2 <= nv)
                st16_nt(ob + 8ull * v0, uint32_t(v[0]), uint32_t(v[0] >> 32), uint32_t(v[1]), uint32_t(v[1] >> 32));
            else
                for (uint32_t i = 0; i < 2; i++)
                    if (v0 + i < nv) {
                        st4(ob + 8ull * (v0 + i), uint32_t(v[i]));
                        st4(ob + 8ull * (v0 + i) + 4, uint32_t(v[i] >> 32));
                    }
        }
    }
}

// Uniform dispatch on the block's width to its specialised decoder.
template <int ES, bool DICT, uint32_t UNR, uint32_t W, uint32_t WMAX, bool F2I = false, bool LDS = false>
ZF_DEV void fp_dispatch(uint32_t w, const uint32_t *words, uint64_t nwords, uint64_t ref, uint32_t nv,
                        uint8_t *ob, bool vec, const uint8_t *dict, uint32_t dict_count, bool &bad,
                        double div = 1.0) {
    if constexpr (W <= WMAX) {
        if (w == W)
            fp_block<ES, DICT, UNR, W, F2I, LDS>(words, nwords, ref, nv, ob, vec, dict, dict_count, bad, div);
        else
            fp_dispatch<ES, DICT, UNR, W + 1, WMAX, F2I, LDS>(w, words, nwords, ref, nv, ob, vec, dict, dict_count,
                                                            bad, div);
    }
}

// One wave decodes blocks [t.a, t.a + t.b) of a FOR_BP or DICT_BP chunk.
// ES = output bytes per value; DICT = dictionary lookup fused after unpack.
// MAXUNR = 0 selects the runtime-width variant.
// A dictionary of up to kDictLds bytes is copied into the wave's LDS (lds,
// when given) and gathered from there: gathers from global memory would
// share the wave's in-order memory counter with its stores.
constexpr uint32_t kDictLds = 4096;

template <int ES, bool DICT, uint32_t MAXUNR>
ZF_DEV void unit_fp(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint8_t *lds = nullptr) {
    constexpr uint32_t VPL = 16 / ES;                     // values per lane per step
    constexpr uint32_t STEPS = kForBlock / (64 * VPL);    // lane-steps per block
    constexpr uint32_t UNR = STEPS < MAXUNR ? STEPS : (MAXUNR ? MAXUNR : 1);
    constexpr uint32_t BITS = (ES == 8 && !DICT) ? 64 : 32;
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t n = ck.n_elems, clen = ck.comp_len;
    const uint32_t nb = (n + kForBlock - 1) / kForBlock;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    const uint8_t *dict = A.dict + ck.dict_off;
    if (16ull * nb > clen || t.a + t.b > nb) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    bool bad = false;
    bool in_lds = false;
    if constexpr (DICT && MAXUNR > 0) {
        if (lds && uint64_t(ck.dict_count) * ES <= kDictLds) {
            // 16 bytes per lane, through a view of the dictionary (a read past
            // it gives zeros)
            const uint32_t nbytes = ck.dict_count * ES;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(uniform_ptr(dict)), 0, int(nbytes), 0x00020000);
            for (uint32_t k = lane_id(); 16 * k < nbytes; k += 64)
                *reinterpret_cast<u32x4 *>(lds + 16 * k) = __builtin_amdgcn_raw_buffer_load_b128(rs, int(16 * k), 0, 0);
            wave_fence();
            in_lds = true;
        }
    }
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
        if constexpr (MAXUNR == 0)
            fp_block_rt<ES, DICT>(first32(w), words, nwords, ref, nv, ob, vec, dict, ck.dict_count, bad);
        else if (DICT && in_lds)
            fp_dispatch<ES, DICT, UNR, 0, BITS, false, true>(first32(w), words, nwords, ref, nv, ob, vec, lds,
                                                             ck.dict_count, bad);
        else
            fp_dispatch<ES, DICT, UNR, 0, BITS>(first32(w), words, nwords, ref, nv, ob, vec, dict,
                                                ck.dict_count, bad);
    }
    if (any(bad)) flag(A.err, ERR_CORRUPT);
}

// One wave decodes blocks [t.a, t.a + t.b) of a Float2Int + bit-packing
// chunk: the FOR + bit-packing unpack of the block's integers, each written
// as (double)d / 10^e (fused: no intermediate integer array), then the
// block's exceptions, stored raw over their slots by the same wave.
template <uint32_t MAXUNR>
ZF_DEV void unit_f2i(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    constexpr uint32_t STEPS = kForBlock / 128;  // lane-steps per block (2 values each)
    constexpr uint32_t UNR = STEPS < MAXUNR ? STEPS : (MAXUNR ? MAXUNR : 1);
    constexpr double kPow10[19] = {1e0,  1e1,  1e2,  1e3,  1e4,  1e5,  1e6,  1e7,  1e8, 1e9,
                                   1e10, 1e11, 1e12, 1e13, 1e14, 1e15, 1e16, 1e17, 1e18};
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t n = ck.n_elems, clen = ck.comp_len, lane = lane_id();
    const uint32_t nb = (n + kForBlock - 1) / kForBlock;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    if (32ull * nb > clen || t.a + t.b > nb) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    bool bad = false;
    for (uint32_t b = t.a; b < t.a + t.b; b++) {
        const uint8_t *d = s + 32ull * b;
        const uint64_t ref = ld64u(d);
        const uint32_t w = ld32u(d + 8), poff = ld32u(d + 12), xoff = ld32u(d + 16);
        const uint32_t nx = ld32u(d + 20) & 0xFFFFu, e = (ld32u(d + 20) >> 16) & 0xFFu;
        const uint32_t j0 = b * kForBlock;
        const uint32_t nv = min(kForBlock, n - j0);
        const uint64_t nwords = (uint64_t(nv) * min(w, 64u) + 31) / 32;
        if (w > 64 || e > 18 || nx > nv || (poff & 15u) || poff < 32ull * nb || poff + 4 * nwords > clen ||
            (xoff & 15u) || xoff < 32ull * nb || xoff + 16ull * nx > clen) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t *words = reinterpret_cast<const uint32_t *>(s + poff);
        uint8_t *ob = out + uint64_t(j0) * 8;
        const bool vec = (reinterpret_cast<uintptr_t>(ob) & 15u) == 0;
        const double div = kPow10[first32(e)];
        if constexpr (MAXUNR == 0)
            fp_block_rt<8, false, true>(first32(w), words, nwords, ref, nv, ob, vec, nullptr, 0, bad, div);
        else
            fp_dispatch<8, false, UNR, 0, 64, true>(first32(w), words, nwords, ref, nv, ob, vec, nullptr, 0,
                                                  bad, div);
        // exceptions (issued after the block's stores by the same wave, so
        // they land last)
        for (uint32_t i = lane; i < nx; i += 64) {
            const uint8_t *r = s + xoff + 16ull * i;
            const uint32_t j = ld32u(r);
            const bool ok = j < nv && (i == 0 || j > ld32u(r - 16));
            bad |= !ok;
            if (ok) {
                const u32x2 q = {ld32u(r + 8), ld32u(r + 12)};
                __builtin_nontemporal_store(q, gp(reinterpret_cast<u32x2 *>(ob + 8ull * j)));
            }
        }
    }
    if (any(bad)) flag(A.err, ERR_CORRUPT);
}

// ===================================================== Group-Parallel
// One wave writes elements [t.b, t.c) of an RLE_DELTA_BP / DELTA_BP chunk,
// starting at group t.a.  Per group of 64 runs, lane j holds run j: an
// exclusive scan of the run lengths gives the run starts (the paper's presum,
// fused), an inclusive scan of dmin + field gives the run values.  The next
// group's record, run lengths and packed words are loaded while this one is
// expanded.  Expansion goes by windows of 64 lanes x 16 bytes of output:
// each run starting in the window writes its index into an LDS slot at its
// start, a wave scan carries the latest index over the window, and each lane
// takes its values with cross-lane permutes — no per-run loop.  slot: this
// wave's 256 dwords.
// One group's record and this lane's run length and packed words.  For
// DeltaStride, w/doff/w0..w2 are the gap field's and wd/dw0..dw2 the stride
// field's.
template <class T>
struct RleGroup {
    uint32_t goff, w, doff, next_off, r, w0, w1, w2;
    uint32_t wd, dw0, dw1, dw2;
    T base, dmin, gmin;
    bool ok;
};

// Field of width w at bit `bit` of a packed stream, from the three words
// starting at word bit / 32.
template <class U>
ZF_DEV U field_of(uint32_t w0, uint32_t w1, uint32_t w2, uint64_t bit, uint32_t w) {
    const uint32_t sh = uint32_t(bit & 31u);
    if constexpr (sizeof(U) == 4) {
        return uint32_t((uint64_t(w0) | (uint64_t(w1) << 32)) >> sh) & mask32(w);
    } else {
        const uint64_t lo = uint64_t(w0) | (uint64_t(w1) << 32);
        return (sh ? ((lo >> sh) | (uint64_t(w2) << (64 - sh))) : lo) & mask64(w);
    }
}

// Expansion of one group of up to 64 runs into out[a, bnd): lane j holds run
// j (act), its output range [start_abs, end_abs) and its value: v for RLE
// (DS = false), v + dstr * p at element p for progressions (DS = true).
// Output goes by windows of 64 lanes x 16 bytes: each run starting in the
// window writes its index into an LDS slot at its start, a wave scan carries
// the latest index over the window, and each lane takes its values with
// cross-lane permutes — no per-run loop.  slot: this wave's 256 dwords.
template <class U, bool DS>
ZF_DEV void expand_runs(U *out, uint32_t a, uint32_t bnd, bool act, uint32_t start_abs, uint32_t end_abs, U v,
                        U dstr, uint32_t *slot) {
    constexpr uint32_t BITS = sizeof(U) * 8;
    const uint32_t lane = lane_id();
    // R outputs per lane per window (16 bytes: one aligned store when whole)
    constexpr uint32_t R = 16 / sizeof(U), SPAN = 64 * R;
    if (a < bnd) {
        // window grid aligned so that out + W0 + R * lane is 16-byte aligned
        // (signed: the first window may start before element 0)
        const int32_t mis = int32_t((reinterpret_cast<uintptr_t>(out + a) & 15u) / sizeof(U));
        const int32_t ia = int32_t(a), ib = int32_t(bnd);
        // 1 + index of the run holding a (a run index, plus one, marks a start)
        uint32_t carry = 1 + uint32_t(__popcll(__ballot(act && end_abs <= a)));
        for (int32_t W0 = ia - mis; W0 < ib; W0 += int32_t(SPAN)) {
#pragma unroll
            for (uint32_t i = 0; i < R; i++) slot[64 * i + lane] = 0;
            wave_fence();
            // element W0 + R l + i has slot 64 i + l
            const uint32_t rel = start_abs - uint32_t(W0);
            if (act && rel < SPAN && start_abs >= a) slot[64 * (rel % R) + rel / R] = lane + 1;
            wave_fence();
            uint32_t m[R], last = 0;
#pragma unroll
            for (uint32_t i = 0; i < R; i++) {
                m[i] = slot[64 * i + lane];
                last = m[i] ? m[i] : last;
            }
            uint32_t cur1 = last_nonzero_below(last, carry);
            U val[R];
#pragma unroll
            for (uint32_t i = 0; i < R; i++) {
                cur1 = m[i] ? m[i] : cur1;
                const int src = int((cur1 - 1) * 4);
                if constexpr (BITS == 32) {
                    val[i] = uint32_t(__builtin_amdgcn_ds_bpermute(src, int(v)));
                } else {
                    const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(src, int(uint32_t(v))));
                    const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(src, int(uint32_t(v >> 32))));
                    val[i] = uint64_t(lo) | (uint64_t(hi) << 32);
                }
                if constexpr (DS) {
                    // plus stride * element index
                    U dd;
                    if constexpr (BITS == 32) {
                        dd = uint32_t(__builtin_amdgcn_ds_bpermute(src, int(dstr)));
                    } else {
                        const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(src, int(uint32_t(dstr))));
                        const uint32_t hi =
                            uint32_t(__builtin_amdgcn_ds_bpermute(src, int(uint32_t(dstr >> 32))));
                        dd = uint64_t(lo) | (uint64_t(hi) << 32);
                    }
                    val[i] = U(val[i] + dd * U(uint32_t(W0 + int32_t(R * lane + i))));
                }
            }
            const int32_t p = W0 + int32_t(R * lane);
            if (p >= ia && p + int32_t(R) <= ib) {
                u32x4 q;
                if constexpr (BITS == 32) q = u32x4{val[0], val[1], val[2], val[3]};
                else q = u32x4{uint32_t(val[0]), uint32_t(val[0] >> 32), uint32_t(val[1]), uint32_t(val[1] >> 32)};
                __builtin_nontemporal_store(q, gp(reinterpret_cast<u32x4 *>(out + p)));
            } else {
#pragma unroll
                for (int32_t i = 0; i < int32_t(R); i++)
                    if (p + i >= ia && p + i < ib) out[p + i] = val[i];
            }
            wave_fence();
        }
    }
}

// Group-Parallel decode of RLE_DELTA_BP / DELTA_BP (DS = false) and
// DSTRIDE_BP (DS = true) chunks: one wave expands the groups that meet its
// tile's element range [t.b, t.c), starting with group t.a.
template <class T, bool DS>
ZF_DEV void unit_rle(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *slot) {
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
    if (!hdr_ok || e1 > n || e0 >= e1 || t.a >= ng) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t *runs = reinterpret_cast<const uint32_t *>(s + roff);
    // record, run length and packed words of group g (bounds checked before
    // any load that depends on the record)
    auto load = [&](uint32_t g, RleGroup<U> &G) {
        const uint8_t *rec = s + 16 + 32ull * g;
        G.goff = ld32u(rec);
        G.base = U(ld64u(rec + 16));
        G.dmin = U(ld64u(rec + 24));
        G.next_off = (g + 1 < ng) ? ld32u(rec + 32) : n;
        const uint32_t cnt = min(kRleGroup, nr - g * kRleGroup);
        uint64_t nwords, dwords = 0;
        if constexpr (DS) {
            const uint32_t poff = ld32u(rec + 4), widths = ld32u(rec + 8);
            G.w = widths & 0xFFu;
            G.wd = (widths >> 8) & 0xFFu;
            G.doff = poff + 8;
            nwords = (uint64_t(cnt - 1) * min(G.w, 64u) + 31) / 32;
            dwords = (uint64_t(cnt) * min(G.wd, 64u) + 31) / 32;
            G.ok = G.w <= BITS && G.wd <= BITS && (widths >> 16) == 0 && (poff & 7u) == 0 &&
                   poff + 8 + 4 * (nwords + dwords) <= clen && G.next_off <= n;
            G.gmin = G.ok ? U(ld64u(s + poff)) : U(0);
        } else {
            G.w = ld32u(rec + 4);
            G.doff = ld32u(rec + 8);
            nwords = (uint64_t(cnt - 1) * min(G.w, 64u) + 31) / 32;
            G.ok = G.w <= BITS && (G.doff & 3u) == 0 && G.doff + 4 * nwords <= clen && G.next_off <= n;
        }
        const bool act = lane < cnt;
        G.r = act ? (unit_runs ? 1u : runs[uint64_t(g) * kRleGroup + lane]) : 0u;
        G.w0 = G.w1 = G.w2 = 0;
        const uint32_t *words = reinterpret_cast<const uint32_t *>(s + G.doff);
        if (G.ok && lane >= 1 && act) {
            const uint64_t k = (uint64_t(lane - 1) * G.w) >> 5;
            G.w0 = k < nwords ? words[k] : 0u;
            G.w1 = k + 1 < nwords ? words[k + 1] : 0u;
            if constexpr (BITS == 64) G.w2 = k + 2 < nwords ? words[k + 2] : 0u;
        }
        if constexpr (DS) {
            G.dw0 = G.dw1 = G.dw2 = 0;
            if (G.ok && act) {
                const uint32_t *dw = words + nwords;
                const uint64_t k = (uint64_t(lane) * G.wd) >> 5;
                G.dw0 = k < dwords ? dw[k] : 0u;
                G.dw1 = k + 1 < dwords ? dw[k + 1] : 0u;
                if constexpr (BITS == 64) G.dw2 = k + 2 < dwords ? dw[k + 2] : 0u;
            }
        }
    };
    RleGroup<U> cur, nxt;
    load(t.a, cur);
    for (uint32_t g = t.a;; g++) {
        if (!cur.ok || (g == t.a && cur.goff > e0)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const bool more = cur.next_off < e1;
        if (more) {
            if (g + 1 >= ng) {
                flag(A.err, ERR_CORRUPT);
                return;
            }
            load(g + 1, nxt);  // in flight while this group is expanded
        }
        const uint32_t cnt = min(kRleGroup, nr - g * kRleGroup);
        // run lengths -> output offsets (exclusive scan = presum)
        const bool act = lane < cnt;
        const uint32_t r = cur.r;
        const uint64_t incl = scan_add64(r);
        const uint64_t total = rl64(incl, cnt - 1);
        if (any(act && r == 0) || uint64_t(cur.goff) + total != cur.next_off) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t end_abs = cur.goff + uint32_t(incl);  // end of run `lane`
        const uint32_t start_abs = end_abs - r;
        // RLE: run values are base, then base + prefix sums of (dmin + field).
        // DeltaStride: run j writes c_j + d_j * p at element p, with stride
        // d_j = dmin + field, start s_j = s_{j-1} + d_{j-1} r_{j-1} + gap_j
        // (gap_j = gmin + field, s_0 = base) and c_j = s_j - d_j * start_j.
        U v, dstr = 0;
        if constexpr (DS) {
            dstr = act ? U(cur.dmin + field_of<U>(cur.dw0, cur.dw1, cur.dw2, uint64_t(lane) * cur.wd, cur.wd))
                       : U(0);
            // start_j = base + sum_{k<j} stride_k count_k + sum_{k<=j} gap_k:
            // an exclusive and an inclusive wave scan, no cross-lane reads
            const U f = act ? U(dstr * U(r)) : U(0);
            const U gap = (act && lane >= 1)
                              ? U(cur.gmin + field_of<U>(cur.w0, cur.w1, cur.w2, uint64_t(lane - 1) * cur.w, cur.w))
                              : U(0);
            const U F = scan_addT<U>(f), Gs = scan_addT<U>(gap);
            const U st = U(cur.base + (F - f) + Gs);
            v = U(st - dstr * U(start_abs));
        } else {
            U delta = cur.base;
            if (lane >= 1 && act)
                delta = U(cur.dmin + field_of<U>(cur.w0, cur.w1, cur.w2, uint64_t(lane - 1) * cur.w, cur.w));
            v = scan_addT<U>(act ? delta : U(0));
        }
        expand_runs<U, DS>(out, max(e0, cur.goff), min(e1, cur.next_off), act, start_abs, end_abs, v, dstr, slot);
        if (!more) return;
        cur = nxt;
    }
}

// ============================= DeltaStride | [Delta | RLE | [BP, BP], BP]
// Two Group-Parallel stages (Sec. 5's order-key scheme).  The first expands
// the runs of D (values V, lengths L, both bit-packed per group) into the run
// starts S, written to the scratch area: S is the running sum of D, so run j
// of D is the progression P_j + V_j (p - a_j + 1) over its positions p, P_j
// the sum before it (the group's base plus an exclusive wave scan of V L).
// The second expands the DeltaStride runs (start S_k from the scratch area,
// count C_k bit-packed per group, the chunk's stride d) into the output.

// Field j (width w <= 32) of packed words at p, from two bounds-checked loads.
ZF_DEV uint32_t field32_at(const uint8_t *p, uint64_t nwords, uint32_t j, uint32_t w) {
    const uint64_t bit = uint64_t(j) * w, k = bit >> 5;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(p);
    const uint32_t w0 = k < nwords ? words[k] : 0u, w1 = k + 1 < nwords ? words[k + 1] : 0u;
    return field_of<uint32_t>(w0, w1, 0u, bit, w);
}
template <class U>
ZF_DEV U fieldU_at(const uint8_t *p, uint64_t nwords, uint32_t j, uint32_t w) {
    const uint64_t bit = uint64_t(j) * w, k = bit >> 5;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(p);
    const uint32_t w0 = k < nwords ? words[k] : 0u, w1 = k + 1 < nwords ? words[k + 1] : 0u;
    uint32_t w2 = 0;
    if constexpr (sizeof(U) == 8) w2 = k + 2 < nwords ? words[k + 2] : 0u;
    return field_of<U>(w0, w1, w2, bit, w);
}

// First stage: S[t.b, t.c) of a chunk (ck.n_elems = R starts, written at
// out_tab[kScratchCol] + ck.out_off), starting with D's group t.a.
template <class U>
ZF_DEV void unit_tree_starts(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *slot) {
    constexpr uint32_t BITS = sizeof(U) * 8;
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t R = ck.n_elems, clen = ck.comp_len, lane = lane_id();
    U *out = reinterpret_cast<U *>(A.out_tab[kScratchCol] + ck.out_off);
    if (clen < 32) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t Q = ld32u(s + 8), ngA = ld32u(s + 12);
    const uint32_t e0 = t.b, e1 = t.c;
    if (ld32u(s) != R || Q == 0 || Q > R || ngA != (uint64_t(Q) + 63) / 64 || 32ull + 32ull * ngA > clen ||
        e1 > R || e0 >= e1 || t.a >= ngA) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    for (uint32_t g = t.a;; g++) {
        const uint8_t *rec = s + 32 + 32ull * g;
        const uint32_t goff = ld32u(rec), poff = ld32u(rec + 4), widths = ld32u(rec + 8), lmin = ld32u(rec + 12);
        const U base = U(ld64u(rec + 16)), vmin = U(ld64u(rec + 24));
        const uint32_t next_off = g + 1 < ngA ? ld32u(rec + 32) : R;
        const uint32_t cnt = min(64u, Q - 64 * g), wv = widths & 0xFFu, wl = (widths >> 8) & 0xFFu;
        const uint64_t vw = (uint64_t(cnt) * min(wv, 64u) + 31) / 32, lw = (uint64_t(cnt) * min(wl, 64u) + 31) / 32;
        if (wv > BITS || wl > 32 || (widths >> 16) != 0 || (poff & 3u) != 0 || poff + 4 * (vw + lw) > clen ||
            next_off > R || (g == t.a && goff > e0)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const bool act = lane < cnt;
        const U vj = act ? U(vmin + fieldU_at<U>(s + poff, vw, lane, wv)) : U(0);
        const uint32_t r = act ? lmin + field32_at(s + poff + 4 * vw, lw, lane, wl) : 0u;
        const uint64_t incl = scan_add64(r);
        const uint64_t total = rl64(incl, cnt - 1);
        if (any(act && r == 0) || uint64_t(goff) + total != next_off) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t end_abs = goff + uint32_t(incl), start_abs = end_abs - r;
        // run j: value P_j + V_j at its first position, then + V_j per position
        const U f = act ? U(vj * U(r)) : U(0);
        const U F = scan_addT<U>(f);
        const U first = U(base + (F - f) + vj);
        const U c = U(first - vj * U(start_abs));
        expand_runs<U, true>(out, max(e0, goff), min(e1, next_off), act, start_abs, end_abs, c, vj, slot);
        if (next_off >= e1) return;
        if (g + 1 >= ngA) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
    }
}

// Second stage: output elements [t.b, t.c) of a chunk, starting with run
// group t.a; the starts S are in the scratch area at ck.aux_off.
template <class U>
ZF_DEV void unit_tree(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *slot) {
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t n = ck.n_elems, clen = ck.comp_len, lane = lane_id();
    U *out = reinterpret_cast<U *>(A.out_tab[ck.col] + ck.out_off);
    const U *S = reinterpret_cast<const U *>(A.out_tab[kScratchCol] + ck.aux_off);
    if (clen < 32) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t R = ld32u(s), ngB = ld32u(s + 4), ngA = ld32u(s + 12), b_off = ld32u(s + 24);
    const U d = U(ld64u(s + 16));
    const uint32_t e0 = t.b, e1 = t.c;
    if (R == 0 || R > n || ngB != (uint64_t(R) + 63) / 64 || b_off != 32ull + 32ull * ngA ||
        uint64_t(b_off) + 16ull * ngB > clen || e1 > n || e0 >= e1 || t.a >= ngB) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    for (uint32_t g = t.a;; g++) {
        const uint8_t *rec = s + b_off + 16ull * g;
        const uint32_t goff = ld32u(rec), poff = ld32u(rec + 4), wc = ld32u(rec + 8), cmin = ld32u(rec + 12);
        const uint32_t next_off = g + 1 < ngB ? ld32u(rec + 16) : n;
        const uint32_t cnt = min(64u, R - 64 * g);
        const uint64_t cw = (uint64_t(cnt) * min(wc, 64u) + 31) / 32;
        if (wc > 32 || (poff & 3u) != 0 || poff + 4 * cw > clen || next_off > n || (g == t.a && goff > e0)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const bool act = lane < cnt;
        const uint32_t r = act ? cmin + field32_at(s + poff, cw, lane, wc) : 0u;
        const U st = act ? S[64ull * g + lane] : U(0);
        const uint64_t incl = scan_add64(r);
        const uint64_t total = rl64(incl, cnt - 1);
        if (any(act && r == 0) || uint64_t(goff) + total != next_off) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t end_abs = goff + uint32_t(incl), start_abs = end_abs - r;
        const U c = U(st - d * U(start_abs));
        expand_runs<U, true>(out, max(e0, goff), min(e1, next_off), act, start_abs, end_abs, c, d, slot);
        if (next_off >= e1) return;
        if (g + 1 >= ngB) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
    }
}

// ======================================================== Non-Parallel
// One wave decodes one LZ77 chunk.  Lane i holds sequence i of a batch of 64;
// wave scans give every sequence's output position, literal position and
// extension index.  Tags, offsets and a 128-entry window of extension words
// are loaded one batch ahead, so the only loads on the parse's critical path
// are the copy sources.

// Extension words e0 + lane and e0 + 64 + lane (0 past the array), packed.
ZF_DEV uint32_t ext_window(const uint16_t *ext, uint32_t e0, uint32_t next, uint32_t lane) {
    const uint32_t lo = e0 + lane < next ? ext[e0 + lane] : 0u;
    const uint32_t hi = e0 + 64 + lane < next ? ext[e0 + 64 + lane] : 0u;
    return lo | (hi << 16);
}

// Entry k (0..127) of a window (entry k in lane k % 64, low half for k < 64);
// every lane of the wave must take part.
ZF_DEV uint32_t ext_pick(uint32_t ew, uint32_t k) {
    const uint32_t v = uint32_t(__builtin_amdgcn_ds_bpermute(int((k & 63u) * 4u), int(ew)));
    return (k & 64u) ? v >> 16 : v & 0xFFFFu;
}


// Copies output bytes [pos, end) of a flat batch of segments (no source byte
// at or after pos), in steps of 64 * BLK bytes:
//  * a byte's source is p + delta, with delta constant over a segment; bit 31
//    of the source set means "index into the second view";
//  * scatter(w0, span, put) calls put(a, delta) for the start a of every
//    segment of the calling lane, and may skip those outside [w0, w0 + span);
//    put records the delta at the segment's first byte in an LDS row of BLK
//    dwords per block (entry k of block b at row[64k + b]; zero = no segment
//    starts here; no delta is ever zero);
//  * each block lane carries the last delta forward over its bytes, taking
//    the delta in force at its first byte from the blocks before it (a
//    ballot over the wave) or from the previous step;
//  * each run of equal delta inside a 4-byte quarter of a block is read as
//    one unaligned dword through two bounds-checked buffer views (the output
//    and the second view), one of which is out of range and reads 0; a dword
//    that would reach past its view sends the block down a byte path; each
//    block is written with one aligned store (bytes at the edges one by one).
// plain4 / nlit4: sizes of the views less 3 (0 if below 4); mis: the output
// pointer's misalignment modulo BLK.  OUT_SRC = false: no segment reads the
// output (only the bytes of a partial first block before pos do, and those
// are not stored), so the output view is never read, and the caller
// guarantees that the dword at every segment byte lies inside the second
// view, so no block needs the byte path.
template <uint32_t BLK, bool OUT_SRC = true, class Scatter>
ZF_DEV void copy_segments(uint32_t *row, uint8_t *out, __amdgpu_buffer_rsrc_t rs_out,
                          __amdgpu_buffer_rsrc_t rs_lit, uint32_t plain4, uint32_t nlit4, uint32_t mis,
                          uint32_t pos, uint32_t end, Scatter &&scatter) {
    const uint32_t lane = lane_id();
    const int32_t B0 = int32_t(pos) - int32_t((mis + pos) & (BLK - 1));
    uint32_t carry = 0;  // delta in force before the step (0: none yet)
    for (int32_t W = B0; W < int32_t(end); W += int32_t(64 * BLK)) {
        const uint32_t w0 = uint32_t(W), span = 64 * BLK;
#pragma unroll
        for (uint32_t k = 0; k < BLK; k++) row[64 * k + lane] = 0;
        wave_fence();
        // scatter the segment starts that fall in the step
        auto put = [&](uint32_t a, uint32_t d) {
            const uint32_t r = a - w0;
            if (r < span) row[64 * (r & (BLK - 1)) + r / BLK] = d;
        };
        scatter(w0, span, put);
        wave_fence();
        // gather: block lane b owns bytes [w0 + BLK b, w0 + BLK b + BLK)
        uint32_t v[BLK];
        uint32_t last = 0;
#pragma unroll
        for (uint32_t k = 0; k < BLK; k++) {
            v[k] = row[64 * k + lane];
            last = v[k] ? v[k] : last;
        }
        uint32_t cur = last_nonzero_below(last, carry);
        const uint32_t Bb = w0 + BLK * lane;
        const int32_t Bi = W + int32_t(BLK * lane);
        // a block wholly outside [pos, end) has no segment start; its
        // reads are sent out of range of both views (no memory traffic)
        const bool live = Bi + int32_t(BLK) > int32_t(pos) && Bi < int32_t(end);
        if (!live) cur = 0x7FFFFFF0u - Bb;
        // one unaligned dword read per run of equal delta inside each
        // 4-byte quarter of the block: at the quarter's first byte and
        // at every segment start.  Byte t of a run sits t bytes into
        // the run's dword.  A dword that would reach past the end of
        // its view is not read; its block takes the byte path below.
        const uint32_t cur0 = cur;
        uint32_t ro[BLK], rl[BLK];
        bool slow = false;
        // all reads first (every lane issues every read; a lane with no
        // run start at byte k reads nothing), then the bytes
#pragma unroll
        for (uint32_t k = 0; k < BLK; k++) {
            cur = v[k] ? v[k] : cur;
            const bool start = (k & 3u) == 0 || v[k] != 0;
            const uint32_t x = Bb + k + cur;
            const uint32_t xl = x ^ 0x80000000u;
            const bool in_out = OUT_SRC && start && x < plain4, in_lit = start && xl < nlit4;
            // (a byte of a partial block outside [pos, end) may send its
            // block down the byte path needlessly; that is rare)
            if constexpr (OUT_SRC) slow = slow || (live && start && !in_out && !in_lit);
            ro[k] = OUT_SRC ? __builtin_amdgcn_raw_buffer_load_b32(rs_out, int(in_out ? x : 0x7FFFFFF0u), 0, 0)
                            : 0u;
            rl[k] = __builtin_amdgcn_raw_buffer_load_b32(rs_lit, int(in_lit ? xl : 0x7FFFFFF0u), 0, 0);
        }
        uint32_t wv[BLK / 4];
#pragma unroll
        for (uint32_t d = 0; d < BLK / 4; d++) {
            uint32_t word = 0, run = 0;
#pragma unroll
            for (uint32_t t = 0; t < 4; t++) {
                const uint32_t k = 4 * d + t;
                run = (t == 0 || v[k] != 0) ? (ro[k] | rl[k]) : run >> 8;
                word |= (run & 0xFFu) << (8 * t);
            }
            wv[d] = word;
        }
        if (OUT_SRC && any(slow)) {
            // byte by byte through the views (the chunk's last bytes,
            // the literal array's last bytes)
            if (slow) {
                uint32_t c = cur0;
#pragma unroll
                for (uint32_t d = 0; d < BLK / 4; d++) {
                    uint32_t word = 0;
#pragma unroll
                    for (uint32_t t = 0; t < 4; t++) {
                        const uint32_t k = 4 * d + t;
                        c = v[k] ? v[k] : c;
                        const uint32_t x = Bb + k + c;
                        word |= (__builtin_amdgcn_raw_buffer_load_b8(rs_out, int(x), 0, 0) |
                                 __builtin_amdgcn_raw_buffer_load_b8(rs_lit, int(x ^ 0x80000000u), 0, 0))
                                << (8 * t);
                    }
                    wv[d] = word;
                }
            }
        }
        if (Bi >= int32_t(pos) && Bi + int32_t(BLK) <= int32_t(end)) {
            if constexpr (BLK == 16) {
                const u32x4 vv = {wv[0], wv[1], wv[2], wv[3]};
                *gp(reinterpret_cast<u32x4 *>(out + Bi)) = vv;
            } else if constexpr (BLK == 8) {
                const u32x2 vv = {wv[0], wv[1]};
                *gp(reinterpret_cast<u32x2 *>(out + Bi)) = vv;
            } else {
                *gp(reinterpret_cast<uint32_t *>(out + Bi)) = wv[0];
            }
        } else if (Bi < int32_t(end) && Bi + int32_t(BLK) > int32_t(pos)) {
            const uint32_t p0 = uint32_t(max(Bi, int32_t(pos)));
            const uint32_t pe = min(uint32_t(Bi) + BLK, end);
            for (uint32_t p = p0; p < pe; p++) {
                const uint32_t k = p - uint32_t(Bi);
                uint32_t wd = wv[0];
#pragma unroll
                for (uint32_t d = 1; d < BLK / 4; d++) wd = k >= 4 * d ? wv[d] : wd;
                gp(out)[p] = uint8_t(wd >> (8 * (k & 3)));
            }
        }
        wave_fence();
    }
}

// Flat batches (every match reads bytes before the batch or its own
// literals; the product encoder keeps every batch flat) are copied by
// copy_segments without any per-lane walk: a literal run is one segment
// whose source is in the literal view, a match one segment (or one per
// period when it overlaps itself) whose source is earlier output.  Other
// batches are replayed in order, one sequence at a time.
// BLK: bytes per block (4, 8 or 16); row: this wave's 64 * BLK dwords.
template <uint32_t BLK>
ZF_DEV void unit_lz(const LaunchArgs &A, const ChunkDesc &ck, uint32_t *row) {
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t clen = ck.comp_len, lane = lane_id();
    const uint32_t es = ck.dtype == D_I32 ? 4 : ck.dtype == D_I64 ? 8 : ck.dtype == D_FIXED16 ? 16 : 1;
    const uint32_t plain = ck.n_elems * es;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    if (clen < 16) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    // the header is the same for every lane: keep it in scalar registers
    const uint32_t nseq = first32(ld32u(s)), nlit = first32(ld32u(s + 4));
    const uint32_t next = first32(ld32u(s + 8)), plen = first32(ld32u(s + 12));
    if (plen != plain || plain > kLzMaxChunk ||
        16ull + 3ull * nseq + 2ull * next + nlit != uint64_t(clen)) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint16_t *offs = reinterpret_cast<const uint16_t *>(s + 16);
    const uint16_t *ext = offs + nseq;
    const uint8_t *tags = reinterpret_cast<const uint8_t *>(ext + next);
    const uint8_t *lits = tags + nseq;
    // byte-granular bounds-checked views of the output and the literals
    // (raw buffers, 32-bit offsets; descriptor word 3 as for gfx9)
    const __amdgpu_buffer_rsrc_t rs_out = __builtin_amdgcn_make_buffer_rsrc(out, 0, int(plain), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs_lit =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(lits), 0, int(nlit), 0x00020000);
    // misalignment of the chunk's output, for BLK-aligned stores
    const uint32_t mis = uint32_t(reinterpret_cast<uintptr_t>(out) & (BLK - 1));
    // a dword read at offset x stays inside a view when x < view size - 3
    const uint32_t plain4 = plain >= 4 ? plain - 3 : 0, nlit4 = nlit >= 4 ? nlit - 3 : 0;
    uint32_t pos = 0, lp = 0, ep = 0;
    uint32_t tag = lane < nseq ? tags[lane] : 0u;
    uint32_t off = lane < nseq ? offs[lane] : 0u;
    uint32_t ew = ext_window(ext, 0, next, lane);
    for (uint32_t base = 0; base < nseq; base += 64) {
        const uint32_t i = base + lane;
        const bool act = i < nseq;
        // prefetch the next batch's headers
        const uint32_t ni = i + 64;
        const uint32_t ntag = ni < nseq ? tags[ni] : 0u;
        const uint32_t noff = ni < nseq ? offs[ni] : 0u;

        const uint32_t lc = tag & 7u, mc = tag >> 3;
        const uint32_t ne = (lc == 7u) + (mc == 31u);
        const uint32_t eincl = scan_add32(ne);
        const uint32_t eex = ep + eincl - ne, etot = rl32(eincl, 63);
        if (uint64_t(ep) + etot > next) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        const uint32_t k1 = eex - ep, k2 = k1 + (lc == 7u);
        const uint32_t x1 = ext_pick(ew, k1), x2 = ext_pick(ew, k2);
        ew = ext_window(ext, ep + etot, next, lane);  // next batch's window
        uint32_t ll = lc, ml = 0;
        if (lc == 7u) ll = 7u + x1;
        if (mc == 31u) ml = 34u + x2;
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
        const uint32_t cnt = min(64u, nseq - base);
        const uint32_t end = pos + total;
        if (!any(!flat)) {
            // segment deltas of this lane's sequence: src = p + delta
            const uint32_t dL = 0x80000000u + (LP - P);        // literal run
            uint32_t dM = q0 - D;                              // match, first period
            if (q0 >= P) dM += 0x80000000u + (LP - P);         // source in own literals
            copy_segments<BLK>(row, out, rs_out, rs_lit, plain4, nlit4, mis, pos, end,
                               [&](uint32_t w0, uint32_t span, auto &&put) {
                if (act && ll) put(P, dL);
                if (act && ml) {
                    if (off >= ml) {
                        put(D, dM);
                    } else {
                        // self-overlapping match: one segment per period of
                        // length off, the delta falling by off each period;
                        // only the periods that start inside the step
                        uint32_t m = 0;
                        if (w0 > D && int32_t(w0) > 0) m = (w0 - D + off - 1) / off;
                        for (uint32_t a = D + m * off; a < D + ml && a - w0 < span; a += off, m++)
                            put(a, dM - m * off);
                    }
                }
            });
        } else {
            // in-order replay of this batch
            for (uint32_t k = 0; k < cnt; k++) {
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
        pos = end;
        lp += ltot;
        ep += etot;
        tag = ntag;
        off = noff;
    }
    if (pos != plain || lp != nlit || ep != next) flag(A.err, ERR_CORRUPT);
}

// ======================================================= String-dictionary
// Group-Parallel (Sec. 5: each word is a group that expands to its entry's
// bytes).  One wave takes whole groups of 64 tokens [t.a, t.b): lane i reads
// token i's entry index from the packed codes, then the entry {offset,
// length}; a wave scan of the lengths gives each token's output position.
// The tokens' bytes are assembled in the wave's LDS buffer, laid on the
// output's 16-byte grid: each lane ORs the dwords its token covers (read as
// unaligned dwords from the entry bytes and masked to the token) into the
// zeroed buffer, which starts on the output's 128-byte grid.  After each
// group the wave writes out the whole 128-byte lines done (one 16-byte store
// per lane and block, one store instruction per group) and carries the
// unfinished line to the buffer's front; at the unit's end it writes out the
// rest.  Bytes of a block outside the unit's output range belong to the
// neighbouring units and are left alone.
// Entries and entry bytes are the chunk's (SDICT_BP, SDICT_ANS) or the
// column dictionary's (SDICT_COL, SDICT_COL_ANS); the packed indices are the
// chunk's, or were ANS-decoded into the scratch area by an earlier launch
// (the *_ANS codecs).  Every header field is checked against the stream or
// dictionary size before use; the wave checks every index and entry and each
// group's length.
// buf: this wave's kSdBufAlloc dwords (16-byte aligned): kSdBufWords of
// buffer and 4 that only ever receive ORs of zero.
constexpr uint32_t kSdBufAlloc = 1280;    // 5120 bytes: 32 one-wave workgroups fill a CU's LDS
constexpr uint32_t kSdBufWords = kSdBufAlloc - 4;
// Before a group the buffer holds at most kSdHold bytes (the whole lines are
// written out after each pair of groups, or sooner); a group adds at most 64
// tokens of kSdMaxToken bytes, so every token position of a checked group
// lies in the buffer, and the four dwords from a position's dword end at
// most 3 dwords past it.
constexpr uint32_t kSdHold = 1008;
static_assert(kSdHold + 64 * kSdMaxToken <= 4 * kSdBufWords, "String-dictionary buffer");
static_assert(kSdBufAlloc % 256 == 0, "String-dictionary buffers: 16-byte aligned, zeroed in 64 lanes x 16 bytes");

// COL: a column dictionary (SDICT_COL, SDICT_COL_ANS), whose entries have
// at least three zero bytes on each side, so a dword read around a token
// needs no mask; else the chunk's own dictionary (SDICT_BP, SDICT_ANS).
// PAIR: two groups per loop iteration (the per-kind kernel); one group per
// iteration keeps the persistent kernel, which holds every kind's routine,
// within its register budget.
// BUFW: the buffer's dwords (kSdBufAlloc, or fewer: a group that does not
// fit then bypasses it).  HOT (COL only): hot[1 + r] holds record r of the
// column dictionary for r < hot_n, in LDS, and hot[0] is zero; those records
// are read there.
template <bool COL, bool PAIR, uint32_t BUFW = kSdBufAlloc, bool HOT = false>
ZF_DEV void unit_sdict_t(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *buf,
                         const u32x4 *hot = nullptr, uint32_t hot_n = 0) {
    static_assert(BUFW % 256 == 0 && 4 * (BUFW - 4) >= kSdHold + 1024, "String-dictionary buffer");
    constexpr uint32_t kWords = BUFW - 4;
    // may a checked group not fit behind the bytes the buffer holds?
    constexpr bool kSmall = kSdHold + 64 * kSdMaxToken > 4 * kWords;
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t lane = lane_id(), plain = ck.n_elems, clen = ck.comp_len;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    constexpr bool coldict = COL;
    const bool staged = ck.codec == C_SDICT_ANS || ck.codec == C_SDICT_COL_ANS;
    uint32_t nt = 0, ne = 0, w = 0, ng = 0, co = 0, nb = 0, go = 0;
    const uint8_t *ebase = nullptr, *bbase = nullptr;  // entries, entry bytes
    bool ok;
    if constexpr (coldict) {
        // header {n_tokens, w, n_groups, codes_off}; the dictionary area
        // {n_bytes, 0, 0, 0, entries, bytes (zero-guarded, ending in zeros)}
        const uint8_t *D = A.dict + ck.dict_off;
        ok = clen >= 16 && ck.dict_bytes >= 16;
        if (ok) {
            nt = first32(ld32u(s));
            w = first32(ld32u(s + 4));
            ng = first32(ld32u(s + 8));
            co = first32(ld32u(s + 12));
            nb = first32(ld32u(D));
        }
        ne = ck.dict_count;
        go = 16;
        ebase = D + 16;
        bbase = D + 16 + 4ull * ne;
        ok = ok && ne >= 1 && 16ull + 4ull * ne + nb <= ck.dict_bytes && co >= 16ull + 4ull * ng;
    } else {
        // header {n_tokens, n_entries, w, n_groups, ent_off, bytes_off,
        // codes_off, n_bytes}; entries, bytes and >= 4 bytes of padding
        // inside the chunk, in that order
        uint32_t eo = 0, bo = 0;
        ok = clen >= 32;
        if (ok) {
            nt = first32(ld32u(s));
            ne = first32(ld32u(s + 4));
            w = first32(ld32u(s + 8));
            ng = first32(ld32u(s + 12));
            eo = first32(ld32u(s + 16));
            bo = first32(ld32u(s + 20));
            co = first32(ld32u(s + 24));
            nb = first32(ld32u(s + 28));
        }
        go = 32;
        ebase = s + eo;
        bbase = s + bo;
        ok = ok && ne >= 1 && (eo & 3u) == 0 && eo >= 32ull + 4ull * ng && uint64_t(eo) + 4ull * ne <= bo &&
             uint64_t(bo) + nb + 4 <= co;
    }
    const uint64_t ncw = (uint64_t(nt) * w + 31) / 32;
    ok = ok && w <= 32 && ng == (uint64_t(nt) + 63) / 64 && co <= clen && (staged || uint64_t(co) + 4 * ncw <= clen);
    if (!ok || t.b > ng || t.a >= t.b) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    // Index words, entries and group offsets are read through bounds-checked
    // views (a read past a view returns 0), so no load sits behind a branch
    // and loads stay in flight until their values are used.
    const uint8_t *codes = uniform_ptr(staged ? A.out_tab[kScratchCol] + ck.aux_off : s + co);
    const __amdgpu_buffer_rsrc_t rs_codes =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(codes), 0, int(4 * ncw), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs_ents =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(ebase), 0, int(4 * ne), 0x00020000);
    // COL: the plan's 16-byte records of the column dictionary's entries
    const __amdgpu_buffer_rsrc_t rs_fat = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(COL ? uniform_ptr(A.fat + ck.fat_off) : ebase), 0, COL ? int(kFatBytes * ne) : 0,
        0x00020000);
    const __amdgpu_buffer_rsrc_t rs_gofs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(s + go), 0, int(4 * ng), 0x00020000);
    // the entry bytes, shifted by 4 so that the dword before a token is at a
    // non-negative offset, with the 4 bytes before them (entries or header)
    // and 4 after (padding, or the last guard of a column dictionary): every
    // dword read below lies inside this view
    const __amdgpu_buffer_rsrc_t rs_ent =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(bbase - 4), 0, int(nb + (COL ? 4 : 8)), 0x00020000);
    // output offsets of groups t.a + l (l = 0..63; plain past the last
    // group), one per lane; the planner gives a unit at most 63 groups
    if (t.b - t.a > 63) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t gwin = t.a + lane < ng ? __builtin_amdgcn_raw_buffer_load_b32(rs_gofs, int(4 * (t.a + lane)), 0, 0)
                                          : plain;
    auto goff = [&](uint32_t g) { return rl32(gwin, min(g - t.a, 63u)); };  // (past t.b: unused)
    const uint32_t ua = goff(t.a), ub = goff(t.b);
    if (ua >= ub || ub > plain) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t oa = uint32_t(reinterpret_cast<uintptr_t>(out) & 127u);
    // buffer byte k holds output byte sbase + k; out + sbase lies on the
    // output's 128-byte grid
    int64_t sbase = int64_t(ua) - int64_t((oa + ua) & 127u);
    // the chunk's output (stores past it are dropped)
    const __amdgpu_buffer_rsrc_t rs_out =
        __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(out), 0, int(plain), 0x00020000);
    const u32x4 zero4 = {0u, 0u, 0u, 0u};
#pragma unroll
    for (uint32_t k = 0; k < BUFW / 256; k++) *reinterpret_cast<u32x4 *>(buf + 4 * (64 * k + lane)) = zero4;
    wave_fence();
    // output bytes below lo are written already (the unit before this one
    // writes those of its last line; a group that bypassed the buffer wrote
    // its own)
    int64_t lo = ua;

    // Three stages run ahead of the group being written: the packed index
    // words of group g + 2 and the entries of group g + 1 are loaded, and
    // group g + 1's token positions are computed and its entry bytes loaded,
    // before group g's bytes are ORed into the buffer.
    // group g's packed indices: 64 tokens of w bits start on a dword, so the
    // group's bits are the 2w dwords from dword 2wg; lane l loads dword
    // 2wg + l (one coalesced load)
    auto words_of = [&](uint32_t g) -> uint32_t {
        const bool act = g < t.b && lane < 2 * w;
        return __builtin_amdgcn_raw_buffer_load_b32(rs_codes, int(act ? 4 * (2 * w * g + lane) : 0x7FFFFFF0u), 0,
                                                    0);
    };
    // entry of group g's token from the group's index dwords (win): the
    // token's w bits start at bit lane * w of them; bad: index past the
    // entries.  (The second dword is read from lane k + 1 < 2w whenever the
    // token reaches into it; lane 63's token at w = 32 lies in dword 63.)
    // (COL: the entry's 16-byte record from the plan's copy of the column
    // dictionary, one load for a token of up to 15 bytes and its length)
    struct Entry {
        u32x4 f;        // COL: the record; else f.x = the entry {offset, length}
        u32x4 h;        // HOT: the record from LDS (zero when f holds it)
        uint32_t code;  // the entry index
        bool bad;
    };
    auto entry_of = [&](uint32_t g, uint32_t win) -> Entry {
        const uint32_t i = 64 * g + lane;
        const bool act = g < t.b && i < nt;
        const uint32_t bit = lane * w, k = bit >> 5;
        const uint32_t w0 = uint32_t(__builtin_amdgcn_ds_bpermute(int(4 * k), int(win)));
        const uint32_t w1 = uint32_t(__builtin_amdgcn_ds_bpermute(int(4 * k + 4), int(win)));
        Entry en;
        en.code = w ? uint32_t((uint64_t(w0) | (uint64_t(w1) << 32)) >> (bit & 31u)) & mask32(w) : 0u;
        en.bad = act && en.code >= ne;
        const bool use = act && !en.bad;
        if constexpr (COL) {
            // (HOT: a record in the LDS copy is read there, and the global
            // read returns zero; the two are ORed where they are used)
            const bool h = HOT && use && en.code < hot_n;
            en.f = __builtin_amdgcn_raw_buffer_load_b128(rs_fat, int(use && !h ? kFatBytes * en.code : 0x7FFFFFF0u),
                                                         0, 0);
            if constexpr (HOT) en.h = hot[h ? en.code + 1 : 0u];
        } else {
            en.f.x = __builtin_amdgcn_raw_buffer_load_b32(rs_ents, int(use ? 4 * en.code : 0x7FFFFFF0u), 0, 0);
        }
        return en;
    };
    struct Grp {
        uint32_t len, eoff, P, end;  // token length and entry offset (COL: the entry index), token start, group end
        uint32_t v0, v1, v2, v3;     // the first four dwords of the token's bytes (COL: of its record)
        bool live;                   // a checked group of the unit, to be staged
    };
    // A corrupt group ends the wave's work: it and every later group are not
    // staged (the loop still runs to the unit's end, so that no exit from
    // its middle keeps loads in flight across the loop's back edge).
    bool dead = false;
    // positions and checks of group g from its entries, then its first loads;
    // a group past the unit (g >= t.b, whose entries read as zero), a corrupt
    // group and the groups after it are not live: they take the previous
    // group's end (prev_end) as their position and end.  Returns false for a
    // corrupt group of the unit.
    auto prepare = [&](uint32_t g, const Entry &en, Grp &G, uint32_t prev_end) -> bool {
        const bool act = g < t.b && 64 * g + lane < nt;
        const bool bad_code = en.bad;
        u32x4 f = en.f;
        if constexpr (HOT) f |= en.h;
        if constexpr (COL) {
            G.len = f.w >> 24;
            G.eoff = en.code;
        } else {
            G.len = en.f.x >> 24;
            G.eoff = en.f.x & 0xFFFFFFu;
        }
        const uint32_t incl = scan_add32(G.len), total = rl32(incl, 63);
        const uint32_t pos = goff(g);
        G.end = goff(g + 1);
        G.P = pos + incl - G.len;
        // token byte 4j - ((oa + P) & 3) begins buffer dword j of the token;
        // the loads go out before the checks (they cannot leave the view), so
        // that no branch stands between them and their use
        const uint32_t m = (oa + G.P) & 3u, nd = act ? (m + G.len + 3) >> 2 : 0u;
        if constexpr (COL) {
            // the record's token bytes (its last byte, the length, cleared);
            // the dwords are shifted into the buffer's alignment when they
            // are ORed
            G.v0 = f.x;
            G.v1 = f.y;
            G.v2 = f.z;
            G.v3 = f.w & 0x00FFFFFFu;
        } else {
            const uint32_t at = G.eoff - m + 4;
            G.v0 = __builtin_amdgcn_raw_buffer_load_b32(rs_ent, int(0 < nd ? at : 0x7FFFFFF0u), 0, 0);
            G.v1 = __builtin_amdgcn_raw_buffer_load_b32(rs_ent, int(1 < nd ? at + 4 : 0x7FFFFFF0u), 0, 0);
            G.v2 = __builtin_amdgcn_raw_buffer_load_b32(rs_ent, int(2 < nd ? at + 8 : 0x7FFFFFF0u), 0, 0);
            G.v3 = __builtin_amdgcn_raw_buffer_load_b32(rs_ent, int(3 < nd ? at + 12 : 0x7FFFFFF0u), 0, 0);
        }
        // an entry's bytes (and the dword read at each) lie in the entry bytes;
        // the group's tokens fill exactly its output range
        // (bitwise, not short-circuit: no branch per condition)
        const bool bad_lane =
            bad_code | (act & (((G.len - 1u) >= kSdMaxToken) | (!COL && G.eoff + G.len > nb)));
        const bool bad_grp = (uint64_t(pos) + total != G.end) | (G.end > ub) | (pos < ua);
        const bool ok = !((any(bad_lane) | bad_grp) & (g < t.b));
        G.live = ok & !dead & (g < t.b);
        G.P = G.live ? G.P : prev_end;
        G.end = G.live ? G.end : prev_end;
        return ok;
    };
    // OR group G's token bytes into the buffer: dword j of the token's span
    // holds token bytes [4j - m, 4j - m + 4) clipped to [0, len); every lane
    // ORs (a zero where it has nothing) so that no branch splits the wave
    auto stage = [&](const Grp &G, uint32_t g) {
        const bool act = G.live && 64 * g + lane < nt;
        const uint32_t o = uint32_t(int64_t(G.P) - sbase), m = o & 3u;
        const uint32_t nd = act ? (m + G.len + 3) >> 2 : 0u;
        const uint32_t head = 0xFFFFFFFFu << (8 * m);            // bytes from the token's start
        const uint32_t endb = m + G.len;                         // buffer byte after the token, from o & ~3
        auto tail = [&](uint32_t j) {                            // bytes before the token's end
            const uint32_t r = endb - 4 * j;
            return r >= 4 ? 0xFFFFFFFFu : ((1u << (8 * r)) - 1u);
        };
        // a staged group's positions lie inside the buffer (o < 4 kWords),
        // so dwords d0 .. d0 + 3 lie inside the allocation; lanes with nothing
        // to OR at dword j OR a zero
        const uint32_t d0 = o >> 2;
        uint32_t *at = buf + d0;
        uint32_t v0, v1, v2, v3;
        if constexpr (COL) {
            // buffer dword j = token bytes [4j - m, 4j - m + 4): bytes 4 - m ..
            // 7 - m of the record's dwords j - 1 (low) and j (high), one byte
            // permute each (the record is zero past the token, so only
            // dwords past the token need clearing)
            const uint32_t sel = 0x07060504u - 0x01010101u * m;
            v0 = 0 < nd ? __builtin_amdgcn_perm(G.v0, 0u, sel) : 0u;
            v1 = 1 < nd ? __builtin_amdgcn_perm(G.v1, G.v0, sel) : 0u;
            v2 = 2 < nd ? __builtin_amdgcn_perm(G.v2, G.v1, sel) : 0u;
            v3 = 3 < nd ? __builtin_amdgcn_perm(G.v3, G.v2, sel) : 0u;
            __hip_atomic_fetch_or(at, v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 1, v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 2, v2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 3, v3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            // a token of 14 or 15 bytes reaching a fifth dword: the record's rest
            const bool longer = act && G.len > kFatInline;
            const bool fifth = act && !longer && nd > 4;
            if (any(fifth))
                __hip_atomic_fetch_or(at + 4, fifth ? __builtin_amdgcn_perm(0u, G.v3, sel) : 0u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            // a token of more than 15 bytes: dword 3 on from the dictionary's
            // entry bytes (the record's dword 2 is the entry's dword 2), after
            // checking the entry against the record and the entry bytes
            if (any(longer)) {
                const uint32_t e = __builtin_amdgcn_raw_buffer_load_b32(rs_ents, int(longer ? 4 * G.eoff : 0x7FFFFFF0u),
                                                                        0, 0);
                const uint32_t off = e & 0xFFFFFFu;
                const bool bad = longer && ((e >> 24) != G.len || off + G.len > nb);
                if (any(bad)) flag(A.err, ERR_CORRUPT);
                const bool go = longer && !bad;
                uint32_t prev = G.v2;
                for (uint32_t j = 3; any(go && j < nd); j++) {
                    const uint32_t cur = __builtin_amdgcn_raw_buffer_load_b32(
                        rs_ent, int(go && j < nd ? off + 4 * j + 4 : 0x7FFFFFF0u), 0, 0);
                    const uint32_t v = __builtin_amdgcn_perm(cur, prev, sel);
                    prev = cur;
                    if (go && j < nd) __hip_atomic_fetch_or(at + j, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        } else {
            // (a dword past nd was read out of range as 0)
            v0 = G.v0 & head & tail(0);
            v1 = G.v1 & tail(1);
            v2 = G.v2 & tail(2);
            v3 = G.v3 & tail(3);
            __hip_atomic_fetch_or(at, v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 1, v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 2, v2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_or(at + 3, v3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (uint32_t j = 4; any(j < nd); j++) {  // tokens of more than 13 bytes
                const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(
                    rs_ent, int(j < nd ? G.eoff - m + 4 * j + 4 : 0x7FFFFFF0u), 0, 0);
                if (j < nd) __hip_atomic_fetch_or(at + j, v & tail(j), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    };

    // OR group g (cur, whose bytes were loaded one group earlier) into the
    // buffer, and write out the whole blocks when enough are done and
    // everything at the unit's end (a group past the unit writes nothing).
    // slot (a constant at each call): this group issues the store of its
    // pair of groups (every group, in the one-group loop)
    // A checked group that does not fit behind the bytes the buffer holds
    // (a small buffer only): the buffer's bytes before it are written out,
    // then its tokens byte by byte from the entry bytes, and the buffer
    // starts again empty at the group's end.
    auto spill = [&](uint32_t g, const Grp &cur) {
        const int64_t p0 = goff(g);
        wave_fence();
        const uint32_t nbk = uint32_t(p0 - sbase + 15) >> 4;  // blocks holding bytes below p0
        for (uint32_t b = lane; b < nbk; b += 64) {
            const int64_t q = sbase + 16 * int64_t(b);
            const u32x4 v = *reinterpret_cast<const u32x4 *>(buf + 4 * b);
            if (q >= lo && q + 16 <= p0) {
                __builtin_nontemporal_store(v, gp(reinterpret_cast<u32x4 *>(out + q)));
            } else {
                for (uint32_t k = 0; k < 16; k++)
                    if (q + k >= lo && q + k < p0) gp(out)[q + k] = uint8_t(v[k >> 2] >> (8 * (k & 3u)));
            }
        }
        const bool act = cur.live && 64 * g + lane < nt;
        uint32_t off = cur.eoff;  // the token's first byte in the entry bytes
        bool go = act;
        if constexpr (COL) {
            const uint32_t e = __builtin_amdgcn_raw_buffer_load_b32(rs_ents, int(act ? 4 * cur.eoff : 0x7FFFFFF0u), 0, 0);
            off = e & 0xFFFFFFu;
            const bool bad = act && ((e >> 24) != cur.len || off + cur.len > nb);
            if (any(bad)) flag(A.err, ERR_CORRUPT);
            go = act && !bad;
        }
        for (uint32_t k = 0; any(go && k < cur.len); k++) {
            const uint8_t c = __builtin_amdgcn_raw_buffer_load_b8(rs_ent, int(go && k < cur.len ? off + 4 + k : 0x7FFFFFF0u),
                                                                  0, 0);
            if (go && k < cur.len) gp(out)[cur.P + k] = c;
        }
#pragma unroll
        for (uint32_t k = 0; k < BUFW / 256; k++) *reinterpret_cast<u32x4 *>(buf + 4 * (64 * k + lane)) = zero4;
        wave_fence();
        lo = cur.end;
        sbase = int64_t(cur.end) - int64_t((oa + cur.end) & 127u);
    };
    auto finish = [&](uint32_t g, const Grp &cur, bool slot) {
        if constexpr (kSmall) {
            if (int64_t(cur.end) - sbase > int64_t(4 * kWords)) {
                spill(g, cur);
                return;
            }
        }
        stage(cur, g);
        const uint32_t fill = uint32_t(int64_t(cur.end) - sbase);
        const bool last = g + 1 == t.b;
        // every store slot (a group past the unit too) issues exactly one
        // store instruction: the whole 128-byte lines ready, at most eight
        // (lane l writes block l); a variable number of stores between a load
        // and its use would make the compiler's wait for that load also wait
        // for every store and later load.  One slot per pair of groups halves
        // the address work of the stores (each writes about twice as much).
        const uint32_t nl = slot && g < t.b ? min(fill >> 7, 8u) : 0u;
        wave_fence();
        if (slot) {
            // (read and written back by every lane, without a branch, so
            // that the store stays one instruction)
            const bool mine = lane < 8 * nl;
            const u32x4 v = *reinterpret_cast<const u32x4 *>(buf + 4 * lane);
            *reinterpret_cast<u32x4 *>(buf + 4 * lane) = mine ? zero4 : v;
            const int64_t q = sbase + 16 * int64_t(lane);
            const bool whole = mine && q >= lo && q + 16 <= int64_t(ub);
            // nontemporal: the output is not read back here, and keeping it
            // out of the L2's way leaves that to the dictionary (0.85 against
            // 0.56 ms per GiB)
            // (the offset passed through an empty asm statement: the store
            // is not duplicated into branches on whether the lane writes)
            uint32_t off = whole ? uint32_t(q) : 0x7FFFFFF0u;
            asm volatile("" : "+v"(off));
            __builtin_amdgcn_raw_buffer_store_b128(v, rs_out, int(off), 0, kNonTemporal);
            // a block partly written already (shared with the unit before,
            // or with a group that bypassed the buffer): its bytes from lo on
            const bool part = mine && !whole && q + 16 > lo && q < int64_t(ub);
            if (any(part) && part)
                for (uint32_t k = 0; k < 16; k++)
                    if (q + k >= lo && q + k < int64_t(ub))
                        gp(out)[q + k] = uint8_t(v[k >> 2] >> (8 * (k & 3u)));
        }
        uint32_t done = nl;  // lines written
        // the buffer holds at most kSdHold bytes before a group
        if (g < t.b && (last || fill >= 128 * nl + (slot ? 128 : kSdHold + 1))) {
            // the unit's end (everything, the last block cut at ub), or more
            // than the buffer may keep before the next group: the rest of
            // the whole lines
            const uint32_t nb = last ? (fill + 15) >> 4 : (fill >> 7) << 3;
            for (uint32_t b = 8 * nl + lane; b < nb; b += 64) {
                const int64_t q = sbase + 16 * int64_t(b);
                const u32x4 v = *reinterpret_cast<const u32x4 *>(buf + 4 * b);
                *reinterpret_cast<u32x4 *>(buf + 4 * b) = zero4;
                if (q >= lo && q + 16 <= int64_t(ub)) {
                    __builtin_nontemporal_store(v, gp(reinterpret_cast<u32x4 *>(out + q)));
                } else {
                    for (uint32_t k = 0; k < 16; k++)
                        if (q + k >= lo && q + k < int64_t(ub))
                            gp(out)[q + k] = uint8_t(v[k >> 2] >> (8 * (k & 3u)));
                }
            }
            done = fill >> 7;
        }
        if (!last && done) {
            // carry the unfinished line (fewer than 128 bytes; its bytes from
            // the next group are still to come) to the front
            wave_fence();
            u32x4 c = zero4;
            if (lane < 8) {
                c = *reinterpret_cast<const u32x4 *>(buf + 4 * (8 * done + lane));
                *reinterpret_cast<u32x4 *>(buf + 4 * (8 * done + lane)) = zero4;
            }
            wave_fence();
            if (lane < 8) *reinterpret_cast<u32x4 *>(buf + 4 * lane) = c;
            wave_fence();
            sbase += 128 * int64_t(done);
        }
    };
    // One group.  Run ahead: take group g + 2's entries from its index
    // dwords (wc, loaded two groups earlier) and load them (into en), take
    // group g + 1's positions from its entries (ec, loaded one group earlier)
    // and load its bytes (into nxt), load group g + 4's index dwords (into
    // wc); then finish group g.  The index dwords come from the chunk or the
    // scratch area, often from HBM, hence the longer run ahead; entries and
    // entry bytes are the dictionary's and stay in the caches.  A wave's
    // loads complete in issue order, so the index dwords go last: waiting
    // for the entries and bytes needed one group later does not wait for
    // them.
    auto step = [&](uint32_t g, uint32_t &wc, Entry &en, const Entry &ec, const Grp &cur, Grp &nxt, bool slot) {
        en = entry_of(g + 2, wc);
        dead |= !prepare(g + 1, ec, nxt, cur.end);
        wc = words_of(g + 4);
        finish(g, cur, slot);
    };
    Grp ga, gb;
    Entry ea, eb;
    if constexpr (PAIR) {
        // the loads in the order that leaves, at the loop's first waits, as
        // many later loads as the loop itself does (the index dwords of
        // groups t.a + 2 and t.a + 3 around the entries and bytes)
        const uint32_t w0 = words_of(t.a), w1 = words_of(t.a + 1);
        uint32_t wa = words_of(t.a + 2);
        ea = entry_of(t.a, w0);
        eb = entry_of(t.a + 1, w1);
        asm volatile("" ::: "memory");  // (keeps the entry loads before the ones below)
        if (!prepare(t.a, ea, ga, ua)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        uint32_t wb = words_of(t.a + 3);
        {
            // a store that writes nothing, in the place of a group's store
            uint32_t off = 0x7FFFFFF0u;
            asm volatile("" : "+v"(off));
            __builtin_amdgcn_raw_buffer_store_b128(zero4, rs_out, int(off), 0, kNonTemporal);
        }
        // two groups per iteration, the run-ahead state alternating between
        // the a and b copies, so that no copy waits for the loads in flight
        // into the next group's state; an odd unit ends with a group past it
        for (uint32_t g = t.a;; g += 2) {
            step(g, wa, ea, eb, ga, gb, false);
            step(g + 1, wb, eb, ea, gb, ga, true);
            if (g + 2 >= t.b) break;
        }
        if (dead) flag(A.err, ERR_CORRUPT);
    } else {
        // one copy of each run-ahead value, the index dwords one group ahead
        // of their use; a corrupt group ends the unit at once
        uint32_t wa = words_of(t.a);
        ea = entry_of(t.a, wa);
        wa = words_of(t.a + 1);
        eb = entry_of(t.a + 1, wa);
        wa = words_of(t.a + 2);
        if (!prepare(t.a, ea, ga, ua)) {
            flag(A.err, ERR_CORRUPT);
            return;
        }
        for (uint32_t g = t.a;; g++) {
            if (!prepare(g + 1, eb, gb, ga.end)) {
                flag(A.err, ERR_CORRUPT);
                return;
            }
            eb = entry_of(g + 2, wa);
            wa = words_of(g + 3);
            finish(g, ga, true);
            if (g + 1 >= t.b) break;
            ga = gb;
        }
    }
}

template <bool PAIR>
ZF_DEV void unit_sdict(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *buf) {
    if (ck.codec == C_SDICT_COL || ck.codec == C_SDICT_COL_ANS) unit_sdict_t<true, PAIR>(A, t, ck, buf);
    else unit_sdict_t<false, PAIR>(A, t, ck, buf);
}
// A unit over a column dictionary with a buffer of kSdSmallBuf dwords and
// the workgroup's LDS copy of the dictionary's hottest records (hot_n of
// them; 0 when the copy is of another dictionary).
constexpr uint32_t kSdSmallBuf = 512;
ZF_DEV void unit_sdict_hot(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck, uint32_t *buf, const u32x4 *hot,
                           uint32_t hot_n) {
    unit_sdict_t<true, true, kSdSmallBuf, true>(A, t, ck, buf, hot, hot_n);
}

// ===================================================================== ANS
// One wave decodes one chunk: lane j runs coder j, which holds bytes j,
// j + 64, j + 128, ... (Sec. 3.1 sees ANS as one serial state chain per chunk;
// the 64 interleaved chains of a chunk advance in lockstep).  Per wave the LDS
// holds the model: slot -> byte (4096 bytes) and byte -> {f, cum} (256 dwords).
// The coders share one stream of 16-bit words, read in byte order: at each
// step the lanes whose state fell below L take the next words in lane order
// (a ballot and a count of the set bits below each lane).  The wave keeps a
// window of 128 words in registers (lane l: words base + l and base + 64 + l,
// packed in one dword) and reads a lane's word with one cross-lane permute;
// the 64 words after the window are loaded one slide ahead, so the stream is
// read once, in coalesced 128-byte loads.
// lds: this wave's kAnsLdsWords dwords (the last 256: output staging).
ZF_DEV void unit_ans(const LaunchArgs &A, const ChunkDesc &ck, uint32_t *lds) {
    const uint8_t *s = A.comp + ck.comp_off;
    const uint32_t lane = lane_id();
    const uint32_t es = ck.dtype == D_I32 ? 4 : (ck.dtype == D_I64 || ck.dtype == D_F64) ? 8
                        : ck.dtype == D_FIXED16 ? 16 : 1;
    const uint32_t n = ck.n_elems * es;
    uint8_t *out = A.out_tab[ck.col] + ck.out_off;
    // sizes, the frequency total and every coder's word range are checked
    // here before any of them is used (the host checked them too)
    if (ck.comp_len < kAnsHdr) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    const uint32_t nw = first32(ld32u(s + 4));
    if (first32(ld32u(s)) != n || uint64_t(kAnsHdr) + 2ull * nw > ck.comp_len) {
        flag(A.err, ERR_CORRUPT);
        return;
    }
    uint8_t *sym = reinterpret_cast<uint8_t *>(lds);
    uint32_t *fc = lds + kAnsM / 4;
    // model: lane l owns bytes 4l .. 4l + 3
    const uint32_t f2 = ld32u(s + 16 + 8 * lane), f3 = ld32u(s + 20 + 8 * lane);
    const uint32_t f[4] = {f2 & 0xFFFFu, f2 >> 16, f3 & 0xFFFFu, f3 >> 16};
    const uint32_t tot = f[0] + f[1] + f[2] + f[3];
    const uint32_t cincl = scan_add32(tot);
    if (rl32(cincl, 63) != kAnsM) {  // the slot walk below needs the exact total
        flag(A.err, ERR_CORRUPT);
        return;
    }
    uint32_t c = cincl - tot;  // cum of byte 4l
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) {
        fc[4 * lane + k] = f[k] | (c << 16);
        c += f[k];
    }
    wave_fence();
    // slot -> byte: lane l fills slots [64 l, 64 l + 64), walking the bytes
    // from the one holding slot 64 l (a binary search over cum)
    {
        const uint32_t s0 = 64 * lane;
        uint32_t lo = 0, hi = 256;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((fc[mid] >> 16) <= s0) lo = mid;
            else hi = mid;
        }
        uint32_t b = lo, e = (fc[b] >> 16) + (fc[b] & 0xFFFFu);
        for (uint32_t k = 0; k < 64; k += 4) {
            uint32_t word = 0;
#pragma unroll
            for (uint32_t i = 0; i < 4; i++) {
                while (s0 + k + i >= e) {  // next byte with a nonzero frequency
                    b++;
                    e = (fc[b] >> 16) + (fc[b] & 0xFFFFu);
                }
                word |= b << (8 * i);
            }
            *reinterpret_cast<uint32_t *>(sym + s0 + k) = word;
        }
    }
    wave_fence();
    // this coder's state; the shared words through a bounds-checked view of
    // the stream (0 past its end, which only a corrupt stream reaches)
    uint32_t x = ld32u(s + 528 + 4 * lane);
    const __amdgpu_buffer_rsrc_t rw =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(s + kAnsHdr), 0, int(2 * nw), 0x00020000);
    auto ld16 = [&](uint32_t at) { return uint32_t(__builtin_amdgcn_raw_buffer_load_b16(rw, int(2 * at), 0, 0)); };
    // window: words [base, base + 128) in win (lane l: base + l low, base + 64
    // + l high); ahead: word base + 128 + l.  pos - base < 64 at every step's
    // start, so a step's at most 64 words lie inside the window.
    uint32_t pos = 0, base = 0;
    uint32_t win = ld16(lane) | (ld16(64 + lane) << 16);
    uint32_t ahead = ld16(128 + lane);
    auto step = [&](uint32_t &b, bool act) {
        const uint32_t slot = x & (kAnsM - 1);
        b = sym[slot];
        const uint32_t e = fc[b];
        const uint32_t xn = (e & 0xFFFFu) * (x >> 12) + slot - (e >> 16);
        x = act ? xn : x;
        const bool need = act && x < kAnsL;  // one word at most: x >= 1 * 2^4 before the shift
        const uint64_t m = __ballot(need);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
        const uint32_t j = pos - base + rank;  // < 128
        // (the permute reads lane (address / 4) mod 64)
        const uint32_t pair = uint32_t(__builtin_amdgcn_ds_bpermute(int(j << 2), int(win)));
        // (x << 16) | (the low or high half of pair) in one byte permute
        const uint32_t sel = 0x05040100u + ((j >> 5) & 2u) * 0x0101u;
        // (computed by every lane and selected: a branch around it costs more)
        uint32_t xp = __builtin_amdgcn_perm(x, pair, sel);
        asm volatile("" : "+v"(xp));
        x = need ? xp : x;
        pos += uint32_t(__popcll(m));
        if (pos - base >= 64) {  // slide by 64 words
            base += 64;
            win = (win >> 16) | (ahead << 16);
            ahead = ld16(base + 128 + lane);
        }
    };
    bool bad = false;
    const uint32_t steps = (n + kAnsLanes - 1) / kAnsLanes;
    uint32_t t = 0;
    if ((reinterpret_cast<uintptr_t>(out) & 15u) == 0) {
        // 16 steps at a time: each lane's 16 bytes (one per step, 64 apart)
        // gathered in LDS, then written back as 16 contiguous bytes per lane
        uint8_t *stg = reinterpret_cast<uint8_t *>(lds + kAnsLdsWords - 256);
        for (; t + 16 <= n / kAnsLanes; t += 16) {
#pragma unroll
            for (uint32_t jj = 0; jj < 16; jj++) {
                uint32_t b;
                step(b, true);
                stg[64 * jj + lane] = uint8_t(b);
            }
            wave_fence();
            const u32x4 v = *reinterpret_cast<const u32x4 *>(stg + 16 * lane);
            __builtin_nontemporal_store(v, gp(reinterpret_cast<u32x4 *>(out + uint64_t(t) * kAnsLanes + 16 * lane)));
            wave_fence();
        }
    }
    for (; t < steps; t++) {
        const uint32_t i = t * kAnsLanes + lane;
        uint32_t b;
        step(b, i < n);
        if (i < n) __builtin_nontemporal_store(uint8_t(b), gp(out) + i);  // never read back here
    }
    bad = x != kAnsL || pos != nw;
    if (any(bad)) flag(A.err, ERR_CORRUPT);
}

// ================================================================ PLAIN
ZF_DEV void unit_plain(const LaunchArgs &A, const Tile &t, const ChunkDesc &ck) {
    const uint8_t *src = A.comp + ck.comp_off;
    uint8_t *dst = A.out_tab[ck.col] + ck.out_off;
    const uint32_t a = t.a, b = min(t.b, ck.comp_len), lane = lane_id();
    if (((reinterpret_cast<uintptr_t>(src + a) | reinterpret_cast<uintptr_t>(dst + a)) & 15u) == 0) {
        const uint32_t nvec = (b - a) / 16;
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src + a);
        uint8_t *d8 = dst + a;
        uint32_t i = lane;
        for (; i + 7 * 64 < nvec; i += 8 * 64) {
            uint4 v[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) v[u] = s4[i + u * 64];
#pragma unroll
            for (uint32_t u = 0; u < 8; u++)
                st16_nt(d8 + 16ull * (i + u * 64), v[u].x, v[u].y, v[u].z, v[u].w);
        }
        for (; i < nvec; i += 64) {
            const uint4 v = s4[i];
            st16_nt(d8 + 16ull * i, v.x, v.y, v.z, v.w);
        }
        for (uint32_t k = a + nvec * 16 + lane; k < b; k += 64) dst[k] = src[k];
    } else {
        for (uint32_t k = a + lane; k < b; k += 64) dst[k] = src[k];
    }
}


// ============================================================== dispatch
// UNR: FP lane-steps of loads kept in flight; 0 = runtime-width FP path.
template <uint32_t UNR>
// lz_row: this wave's LDS scratch (max(kAnsLdsWords, kSdBufAlloc) dwords):
// the LZ77 row, the ANS model and staging, the String-dictionary buffer or
// the RLE window slots.
ZF_DEV void run_unit(const LaunchArgs &A, uint32_t kind, uint32_t u, uint32_t *lz_row) {
    const Tile t = A.tiles[u];
    const ChunkDesc ck = A.chunks[t.chunk];
    switch (kind) {
    case K_PLAIN: unit_plain(A, t, ck); break;
    case K_FOR32: unit_fp<4, false, UNR>(A, t, ck); break;
    case K_F2I: unit_f2i<UNR>(A, t, ck); break;
    case K_FOR64: unit_fp<8, false, UNR>(A, t, ck); break;
    case K_DICT32: unit_fp<4, true, UNR>(A, t, ck); break;
    case K_DICT64: unit_fp<8, true, UNR>(A, t, ck); break;
    case K_DICT128: unit_fp<16, true, UNR>(A, t, ck); break;
    case K_RLE32:
        if (ck.codec == C_DSTRIDE_BP) unit_rle<uint32_t, true>(A, t, ck, lz_row);
        else if (ck.codec == C_DSTREE_STARTS) unit_tree_starts<uint32_t>(A, t, ck, lz_row);
        else unit_rle<uint32_t, false>(A, t, ck, lz_row);
        break;
    case K_RLE64:
        if (ck.codec == C_DSTRIDE_BP) unit_rle<uint64_t, true>(A, t, ck, lz_row);
        else if (ck.codec == C_DSTREE_STARTS) unit_tree_starts<uint64_t>(A, t, ck, lz_row);
        else unit_rle<uint64_t, false>(A, t, ck, lz_row);
        break;
    case K_TREE:
        if (ck.dtype == D_I32) unit_tree<uint32_t>(A, t, ck, lz_row);
        else unit_tree<uint64_t>(A, t, ck, lz_row);
        break;
    case K_LZ: unit_lz<4>(A, ck, lz_row); break;
    case K_SDICT: unit_sdict<false>(A, t, ck, lz_row); break;
    case K_ANS: unit_ans(A, ck, lz_row); break;
    }
}

// Workgroup b of n runs on XCD b mod 8 (workgroups are dealt to the eight
// XCDs in turn).  This maps it to a work index such that each XCD takes one
// contiguous eighth of the indices, in order: XCD x holds indices
// [x q + min(x, r), ...) with n = 8 q + r.
ZF_DEV uint32_t xcd_block(uint32_t b, uint32_t n) {
    constexpr uint32_t kXcds = 8;
    const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds, i = b / kXcds;
    return x * q + min(x, r) + i;
}

// One launch per kind: wave w of block b takes unit begin + b*waves + w.
// Only the routine of KIND is instantiated here.
template <uint32_t KIND>
__global__ __launch_bounds__(1024) void k_decode_kind(LaunchArgs A) {
    const uint32_t waves = blockDim.x / 64;
    // String-dictionary: the tiles of a chunk share its dictionary, so
    // neighbouring tiles go to the same XCD (and its L2)
    const uint32_t u = A.kind_begin[KIND] + blockIdx.x * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[KIND + 1]) return;
    const Tile t = A.tiles[u];
    const ChunkDesc ck = A.chunks[t.chunk];
    if constexpr (KIND == K_PLAIN) {
        unit_plain(A, t, ck);
    } else if constexpr (KIND == K_FOR32) {
        unit_fp<4, false, 8>(A, t, ck);
    } else if constexpr (KIND == K_FOR64) {
        unit_fp<8, false, 8>(A, t, ck);
    } else if constexpr (KIND == K_F2I) {
        unit_f2i<8>(A, t, ck);
    } else if constexpr (KIND == K_DICT32 || KIND == K_DICT64 || KIND == K_DICT128) {
        // each wave's dictionary copy, kDictLds bytes of dynamic shared memory
        extern __shared__ __attribute__((aligned(16))) uint8_t dict_lds[];
        uint8_t *lds = dict_lds + (threadIdx.x / 64) * kDictLds;
        if constexpr (KIND == K_DICT32) unit_fp<4, true, 8>(A, t, ck, lds);
        else if constexpr (KIND == K_DICT64) unit_fp<8, true, 8>(A, t, ck, lds);
        else unit_fp<16, true, 8>(A, t, ck, lds);
    } else if constexpr (KIND == K_RLE32) {
        __shared__ uint32_t rle_slots[16][256];
        if (ck.codec == C_DSTRIDE_BP) unit_rle<uint32_t, true>(A, t, ck, rle_slots[threadIdx.x / 64]);
        else if (ck.codec == C_DSTREE_STARTS) unit_tree_starts<uint32_t>(A, t, ck, rle_slots[threadIdx.x / 64]);
        else unit_rle<uint32_t, false>(A, t, ck, rle_slots[threadIdx.x / 64]);
    } else if constexpr (KIND == K_RLE64) {
        __shared__ uint32_t rle_slots[16][256];
        if (ck.codec == C_DSTRIDE_BP) unit_rle<uint64_t, true>(A, t, ck, rle_slots[threadIdx.x / 64]);
        else if (ck.codec == C_DSTREE_STARTS) unit_tree_starts<uint64_t>(A, t, ck, rle_slots[threadIdx.x / 64]);
        else unit_rle<uint64_t, false>(A, t, ck, rle_slots[threadIdx.x / 64]);
    } else if constexpr (KIND == K_TREE) {
        __shared__ uint32_t rle_slots[16][256];
        if (ck.dtype == D_I32) unit_tree<uint32_t>(A, t, ck, rle_slots[threadIdx.x / 64]);
        else unit_tree<uint64_t>(A, t, ck, rle_slots[threadIdx.x / 64]);
    }
}

void launch_sdict(const LaunchArgs &A, uint32_t waves, hipStream_t st);

// LZ77: one unit (chunk) per wave; each wave's LDS row is dynamic shared
// memory, 64 * BLK dwords.
template <uint32_t BLK>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_decode_lz(LaunchArgs A) {
    const uint32_t waves = blockDim.x / 64;
    const uint32_t u = A.kind_begin[K_LZ] + blockIdx.x * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[K_LZ + 1]) return;
    extern __shared__ uint32_t lz_smem[];
    unit_lz<BLK>(A, A.chunks[A.tiles[u].chunk], lz_smem + (threadIdx.x / 64) * 64 * BLK);
}
void launch_lz(const LaunchArgs &A, uint32_t waves, uint32_t blk, hipStream_t st);
hipError_t launch_decode(const LaunchArgs &A, uint32_t persistent_waves, const uint32_t *wpb,
                         uint32_t lz_blk, hipStream_t st, KindEvents *ev);

void launch_ans(const LaunchArgs &A, uint32_t waves, hipStream_t st);

// Host launchers, one per kind, each defined in its kind's translation unit.
#define ZF_KIND_LAUNCHERS(X)                                                                       \
    X(K_RLE64, launch_rle64) X(K_RLE32, launch_rle32) X(K_TREE, launch_tree)                       \
    X(K_DICT128, launch_dict128) X(K_DICT64, launch_dict64) X(K_DICT32, launch_dict32)              \
    X(K_FOR64, launch_for64) X(K_FOR32, launch_for32) X(K_F2I, launch_f2i) X(K_PLAIN, launch_plain)
#define ZF_DECLARE_LAUNCHER(KIND, NAME) void NAME(const LaunchArgs &A, uint32_t waves, hipStream_t st);
ZF_KIND_LAUNCHERS(ZF_DECLARE_LAUNCHER)

#define ZF_DEFINE_LAUNCHER(KIND, NAME)                                                             \
    void NAME(const LaunchArgs &A, uint32_t waves, hipStream_t st) {                               \
        const uint32_t n = A.kind_begin[KIND + 1] - A.kind_begin[KIND];                            \
        if (!n) return;                                                                            \
        const uint32_t lds = (KIND == K_DICT32 || KIND == K_DICT64 || KIND == K_DICT128) ? waves * kDictLds : 0; \
        hipLaunchKernelGGL(k_decode_kind<KIND>, dim3((n + waves - 1) / waves), dim3(64 * waves), lds, st, A); \
    }

}  // namespace zf
