// Device helpers shared by the embedding kernels (full net and student net).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "bf16ops.h"
#include "devmath.h"
#include "kernels.h"

namespace dp {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <class T> struct Acc4;
template <> struct Acc4<double> { typedef d4v type; };
template <> struct Acc4<float> { typedef f4v type; };

__device__ __forceinline__ d4v mfma4(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class T>
__device__ __forceinline__ T tanh_t(T x) { return dp_tanh(x); }

// Accumulator row held by lane group g in register q of a 16x16 MFMA result:
// FP64 16x16x4 returns rows g + 4q, FP32 16x16x4 (and BF16 16x16x32) rows 4g + q.
__device__ __forceinline__ int lpos(double, int g, int q) { return g + 4 * q; }
__device__ __forceinline__ int lpos(float, int g, int q) { return 4 * g + q; }
#define LP(g, q) lpos(T(), g, q)

template <class T>
__device__ __forceinline__ T shfl_x(T v, int mask) {
  return __shfl_xor(v, mask);
}

// Cross-lane moves inside a 16-lane row with DPP (VALU, no LDS traffic).  The
// reduce-scatter over the 16 rows of a chunk pairs lanes by xor 8 (row_ror:8), xor 7
// (row_half_mirror), xor 2 and xor 1 (quad_perm); these partner offsets span the row.
enum { DPP_ROR8 = 0x128, DPP_HALF_MIRROR = 0x141, DPP_XOR2 = 0x4E, DPP_XOR1 = 0xB1 };
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  long long x = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// species of the rows starting at r0 (rows of one block never straddle species)
__device__ __forceinline__ int species_of(int r0, int ntypes, const int* __restrict__ type_row0) {
  for (int t = 0; t < ntypes; t++)
    if (r0 >= type_row0[t] && r0 < type_row0[t + 1]) return t;
  return -1;
}

template <class T>
__device__ __forceinline__ void stage_net(T* __restrict__ dst, const T* __restrict__ src) {
  for (int q = threadIdx.x; q < kNetElems; q += blockDim.x) dst[q] = src[q];
}

// copy nbytes (a multiple of 16, both pointers 16-byte aligned) into LDS
__device__ __forceinline__ void stage_bytes(void* __restrict__ dst, const void* __restrict__ src, int nbytes) {
  const uint4* s = (const uint4*)src;
  uint4* d = (uint4*)dst;
  for (int q = threadIdx.x; q < nbytes / 16; q += blockDim.x) d[q] = s[q];
}



// Environment row of one neighbour (Eq. 5) and its derivative with respect to d.
struct Env {
  double d[3], r, ir, s, ds, R[4];
};
__device__ __forceinline__ void env_row(const ModelC& m, const double* __restrict__ xe, int e,
                                        const double xi[3], Env& v) {
  v.d[0] = xe[3 * e] - xi[0];
  v.d[1] = xe[3 * e + 1] - xi[1];
  v.d[2] = xe[3 * e + 2] - xi[2];
  double r2 = v.d[0] * v.d[0] + v.d[1] * v.d[1] + v.d[2] * v.d[2];
  v.r = sqrt(r2);
  v.ir = 1.0 / v.r;
  smooth_fn_ir(m, v.r, v.ir, v.s, v.ds);
  double sr = v.s * v.ir;
  v.R[0] = v.s;
  v.R[1] = sr * v.d[0];
  v.R[2] = sr * v.d[1];
  v.R[3] = sr * v.d[2];
}

// one reduce-scatter step on an array of S values: the lane whose "up" bit is set
// keeps the upper half, its DPP partner (which has the bit clear) the lower half
template <class T, int S, int CTRL>
__device__ __forceinline__ void rs_step(T (&v)[64], bool up) {
#pragma unroll
  for (int k = 0; k < S / 2; k++) {
    T a = v[k], b = v[k + S / 2];
    T send = up ? a : b;
    T keep = up ? b : a;
    v[k] = keep + dpp_mov<CTRL>(send);
  }
}

// write T (row-major [M][4] per row) from the accumulators after contract_chunk: the lane
// holds tile mt = 4 b3 + 2 b2 + b1, register q = 2 b0 + j / 4, c = j % 4
template <class T>
__device__ __forceinline__ void write_T(T* __restrict__ Tout, const T (&acc)[8], int rb, int g, int s0,
                                        T scale) {
  const int mt = 4 * ((rb >> 3) & 1) + 2 * ((rb >> 2) & 1) + ((rb >> 1) & 1);
#pragma unroll
  for (int j = 0; j < 8; j++) {
    int q = 2 * (rb & 1) + (j >> 2), c = j & 3;
    int p = 16 * mt + LP(g, q);
    int f = (p % kP0) < s0 ? (p / kP0) * s0 + (p % kP0) : -1;
    if (f >= 0) Tout[f * 4 + c] = acc[j] * scale;
  }
}

}  // namespace dp
