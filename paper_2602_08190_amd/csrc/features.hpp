// Chunk statistics and the host copy of the cost model used by ZF_AUTO.
#pragma once
#include <string>
#include <vector>

#include "zf_internal.hpp"

namespace zf {

constexpr int kFeatures = 32;     // chunk statistics
constexpr int kChoices = 24;      // 6 codecs x 4 schedules
constexpr int kMlpParams = 7832;  // 32 -> 64 -> 64 -> 24

void chunk_features(const void *src, uint64_t n, uint32_t dtype, float *f);

// Codec of each group of 4 outputs: PLAIN, FOR_BP, DICT_BP, DELTA_BP,
// RLE_DELTA_BP, LZ77.
extern const uint8_t kChoiceCodec[6];
bool choice_allowed(uint32_t choice, uint32_t dtype, uint64_t chunk_bytes, bool have_dict);

// Trained network: feature standardisation (x - mean) * scale, then the
// 32-64-64-24 relu network.  File: "ZFMLP1\0\0", 32 means, 32 scales,
// 7832 parameters, all little-endian float32.
struct CostModel {
    std::vector<float> mean, scale, params;
    bool ok = false;
    bool load(const std::string &path);
    void predict(const float *x, float *y) const;
};

}  // namespace zf
