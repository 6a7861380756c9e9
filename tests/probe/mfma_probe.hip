// Test-only probe of the BF16 matrix-core operand layout the attribute
// network kernels assume for v_mfma_f32_16x16x32_bf16 (lane l of a wave):
//   A (16 x 32): row l%16, k = 8*(l/16) .. +7
//   B (32 x 16): col l%16, k = 8*(l/16) .. +7
//   C (16 x 16): col l%16, rows 4*(l/16) .. +3
// probe_mfma_bf16 computes C = A B for one tile (A, B row-major bf16 bit
// patterns, C row-major FP32; device pointers) and synchronises.  Not part
// of the library.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void k_probe_mfma_bf16(const uint16_t* A, const uint16_t* B, float* C)
{
    const int l = threadIdx.x;
    uint16_t a[8], b[8];
    for (int j = 0; j < 8; ++j) {
        a[j] = A[(l % 16) * 32 + 8 * (l / 16) + j];
        b[j] = B[(8 * (l / 16) + j) * 16 + (l % 16)];
    }
    bf16x8 av, bv;
    __builtin_memcpy(&av, a, 16);
    __builtin_memcpy(&bv, b, 16);
    f32x4 c = {0, 0, 0, 0};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    for (int i = 0; i < 4; ++i) C[(4 * (l / 16) + i) * 16 + (l % 16)] = c[i];
}

extern "C" int probe_mfma_bf16(const uint16_t* A, const uint16_t* B, float* C)
{
    if (!A || !B || !C) return 1;
    hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(1), dim3(64), 0, 0, A, B, C);
    if (hipGetLastError() != hipSuccess) return 2;
    return hipDeviceSynchronize() == hipSuccess ? 0 : 2;
}
