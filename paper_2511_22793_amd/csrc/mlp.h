// Internal constants and the argument block of the attribute-network kernels.
#pragma once
#include <stdint.h>

namespace gs {

constexpr int MLP_EMB = 32;      // embedding width
constexpr int MLP_BANDS = 8;     // Fourier bands of the transmitter encoding
constexpr int MLP_ENC = 3 + 6 * MLP_BANDS;  // 51
constexpr int MLP_ENC_PAD = 64;  // stride of the saved encodings
constexpr int MLP_IN = 96;       // padded input width (32 + 51 -> 96)
constexpr int MLP_HID = 64;      // hidden width
constexpr int MLP_F = 64;        // subcarriers (outputs = 2 * MLP_F)

struct MlpArgs {
    const uint16_t *W2, *W3, *W2T, *W3T, *W1eT;
    const float *b2, *b3;
    const float* Z1;
    const float* cb;
    const float* mean;
    int n;
    const float* tx;
    float r_near;
    const uint32_t* list;
    int64_t list_stride;
    const uint32_t* count;
    int count_stride;
    int64_t row_cap;
    float* attr;
    const float* d_attr;
    float* clear;  // d_attr again when consumed rows are to be zeroed
    int64_t attr_stride;
    uint16_t *save_h1, *save_h2, *save_do, *save_dz2, *save_dz1;
    float *db3, *db2, *dc, *dE;
};

}  // namespace gs
