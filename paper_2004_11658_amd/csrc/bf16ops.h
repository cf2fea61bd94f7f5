// BF16 MFMA operand helpers shared by the embedding and fitting kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace dp {

typedef float f4v __attribute__((ext_vector_type(4)));

// BF16 MFMA operands: 8 bf16 per lane for v_mfma_f32_16x16x32_bf16.  The k slot (lane
// group, element) is the same for the A and the B operand, so a product sums over any
// bijection of positions onto slots that both operands follow.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4v mfma_bf(bf8 a, bf8 b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// round 8 floats to bf16 (nearest even) and, for the split mode, the residuals
template <int PARTS>
__device__ __forceinline__ void split8(const float (&v)[8], bf8& hi, bf8& lo) {
#pragma unroll
  for (int j = 0; j < 8; j++) {
    __bf16 h = (__bf16)v[j];
    hi[j] = h;
    if (PARTS == 2) lo[j] = (__bf16)(v[j] - (float)h);
  }
}
// c += A B with A, B given as hi (+ lo): hi hi (+ hi lo + lo hi)
template <int PARTS>
__device__ __forceinline__ f4v mfma_split(bf8 ah, bf8 al, bf8 bh, bf8 bl, f4v c) {
  if (PARTS == 2) {
    c = mfma_bf(al, bh, c);
    c = mfma_bf(ah, bl, c);
  }
  return mfma_bf(ah, bh, c);
}

}  // namespace dp
