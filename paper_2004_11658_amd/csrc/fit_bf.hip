// BF16 fitting net (Section 2, Eq. 1-4) and its adjoint in three kernels per 64-row tile.
//
// Rows are centres grouped by species (groups padded to 64 rows), so one workgroup takes
// one 64-row tile and one species' fitting net.  The MFMA runs with the weights as the
// A operand (16 outputs x 32 k) and the activations as the B operand (32 k x 16 rows): a
// lane of the result holds 4 consecutive outputs n = 16 ct + 4 g + q of one row 16 rt + rb
// (rb = lane % 16, g = lane / 16).  Wave w of the 8 owns the output tiles ct = w and
// w + 8 for all four row tiles rt; two waves share each SIMD, so one's epilogue and
// waits overlap the other's products.
//
// Weights are pre-packed as MFMA fragments (block (ct, ks, part) of 64 lanes x 8 bf16,
// lane l holding B[32 ks + 8 (l / 16) + j][16 ct + l % 16], B = W for the forward and
// B = W^T for the adjoint, hi and lo parts), so a wave fetches a fragment with one
// coalesced 1 KB load straight from L2, and every fragment is fetched by one wave only.
// Activations are staged in LDS in the same fragment order.
//
//   k_fit_l1_fwd   t1 = tanh(D W1 + b1) with D = T T<^T (Eq. 4) formed while staging
//   k_fit_tail     x_k = x_{k-1} + tanh(x_{k-1} W_k + b_k) for the square layers,
//                  E_i = x_L . w_o + b_o, then back to d1 = dE/dz1 = g1 (1 - t1^2), stored as
//                  MFMA operand fragments
//   k_fit_l1_bwd   dD = d1 W1^T and dE/dT = dD T< + [a < m2] dD^T T (Eq. 4's adjoint);
//                  dD never leaves the registers
#include <hip/hip_runtime.h>

#include "bf16ops.h"
#include "common.h"
#include "devmath.h"
#include "kernels.h"

namespace dp {

constexpr int FR = 64;    // rows per workgroup
constexpr int FW = 8;     // waves per workgroup
constexpr int FT = 64 * FW;
constexpr int kKS = 8;    // k steps of operands whose k dimension is a fitting width (<= 256, padded)

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

struct FitBfArgs {
  int M, N, nfit, ntypes, nrows;
  const int* type_row0;
  const int* row_atom;
  const float* T;                // [nrows][M][4]
  const void* const* Wf;         // [(species * nfit + k) * 2 + dir] fragment-packed weights
  const void* const* bias;       // [species * nfit + k] -> float [N]
  const void* const* wo;         // [species] -> float [N]
  const double* bo;              // [species]
  float* t1;                     // [nrows][N] first-layer tanh
  float* act;                    // [nfit][nrows][N] tanh of the square layers (per-tile lane order)
  __bf16* d1f;                   // per tile [kKS][4][PARTS][512] dE/dz1 fragments
  double* Ei;                    // [nrows]
  float* gT;                     // [nrows][M][4]
};

__device__ __forceinline__ int fitbf_species(const FitBfArgs& P, int r0) {
  for (int t = 0; t < P.ntypes; t++)
    if (r0 >= P.type_row0[t] && r0 < P.type_row0[t + 1]) return t;
  return -1;
}

// Loads through pointers read from the operand tables are generic (flat) unless told
// otherwise; flat loads also count against the LDS wait counter, so name them global.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gld(const void* p) {
  return *(const GAS T*)p;
}

// weight fragment (ct, ks) of a packed operand with KS k steps
template <int PARTS>
__device__ __forceinline__ void wfrag(const __bf16* __restrict__ W, int KS, int ct, int ks, int lane, bf8& h,
                                      bf8& l) {
  const __bf16* p = W + ((size_t)(ct * KS + ks) * PARTS) * 512 + lane * 8;
  h = gld<bf8>(p);
  l = PARTS == 2 ? gld<bf8>(p + 512) : h;
}

// the wave's two column tiles w and w + 8 at k step ks (operands padded to 16 tiles)
template <int PARTS>
__device__ __forceinline__ void load_wc(const __bf16* __restrict__ W, int KS, int ks, int w, int lane, bf8 (&wh)[2],
                                        bf8 (&wl)[2]) {
  wfrag<PARTS>(W, KS, w, ks, lane, wh[0], wl[0]);
  wfrag<PARTS>(W, KS, w + 8, ks, lane, wh[1], wl[1]);
}

// Activation fragments: the value of row 16 rt + rb at n = 16 ct + 4 g + q sits in
// fragment (ks = ct / 2, rt), lane rb + 16 (2 (ct % 2) + g / 2), element 4 (g % 2) + q.
__device__ __forceinline__ int xfrag_off(int ct, int rt, int part, int parts, int rb, int g) {
  const int ks = ct >> 1, lp = rb + 16 * (2 * (ct & 1) + (g >> 1));
  return (((ks * 4 + rt) * parts + part) * 64 + lp) * 8 + 4 * (g & 1);
}

template <int PARTS>
__device__ __forceinline__ void split4(f4v v, bf4& h, bf4& l) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const __bf16 hv = (__bf16)v[q];
    h[q] = hv;
    if (PARTS == 2) l[q] = (__bf16)(v[q] - (float)hv);
  }
}

template <int PARTS>
__device__ __forceinline__ void put4(__bf16* X, int ct, int rt, int rb, int g, f4v v) {
  bf4 h, l;
  split4<PARTS>(v, h, l);
  *(bf4*)(X + xfrag_off(ct, rt, 0, PARTS, rb, g)) = h;
  if (PARTS == 2) *(bf4*)(X + xfrag_off(ct, rt, 1, PARTS, rb, g)) = l;
}

// stage a [u][rt] register tile (C layout of the wave's column tiles) into LDS fragments
template <int PARTS>
__device__ __forceinline__ void stage_tile(__bf16* Xs, const f4v (&v)[2][4], int w, int NT, int rb, int g) {
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int ct = w + 8 * u;
    if (ct >= NT) continue;
#pragma unroll
    for (int rt = 0; rt < 4; rt++) put4<PARTS>(Xs, ct, rt, rb, g, v[u][rt]);
  }
}

// X fragments (all four row tiles) of k step ks from LDS
template <int PARTS>
__device__ __forceinline__ void load_x(const __bf16* Xs, int ks, int lane, bf8 (&xh)[4], bf8 (&xl)[4]) {
#pragma unroll
  for (int rt = 0; rt < 4; rt++) {
    const __bf16* p = Xs + ((size_t)(ks * 4 + rt) * PARTS) * 512 + lane * 8;
    xh[rt] = *(const bf8*)p;
    xl[rt] = PARTS == 2 ? *(const bf8*)(p + 512) : xh[rt];
  }
}

// acc[u][rt] += W(ct_u) X(rt) for one k step.  The split products go in three sweeps
// over the accumulators (lo hi, hi lo, then hi hi: the same order per accumulator as
// mfma_split), so that dependent products on one accumulator are never adjacent.
template <int PARTS, int U>
__device__ __forceinline__ void mma_sweeps(const bf8 (&wh)[U], const bf8 (&wl)[U], const bf8 (&xh)[4],
                                           const bf8 (&xl)[4], f4v (&acc)[U][4]) {
  if (PARTS == 2) {
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int rt = 0; rt < 4; rt++) acc[u][rt] = mfma_bf(wl[u], xh[rt], acc[u][rt]);
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int rt = 0; rt < 4; rt++) acc[u][rt] = mfma_bf(wh[u], xl[rt], acc[u][rt]);
  }
#pragma unroll
  for (int u = 0; u < U; u++)
#pragma unroll
    for (int rt = 0; rt < 4; rt++) acc[u][rt] = mfma_bf(wh[u], xh[rt], acc[u][rt]);
}

template <int PARTS>
__device__ __forceinline__ void mma_step(const bf8 (&wh)[2], const bf8 (&wl)[2], const __bf16* Xs, int ks, int lane,
                                         f4v (&acc)[2][4]) {
  bf8 xh[4], xl[4];
  load_x<PARTS>(Xs, ks, lane, xh, xl);
  mma_sweeps<PARTS, 2>(wh, wl, xh, xl, acc);
}

// acc += W X over the kKS steps of a square layer; weights and X fragments fetched one
// step ahead
template <int PARTS>
__device__ __forceinline__ void tile_mm(const __bf16* __restrict__ W, int w, int lane, const __bf16* Xs,
                                        f4v (&acc)[2][4]) {
  bf8 wh[2][2], wl[2][2], xh[2][4], xl[2][4];
  load_wc<PARTS>(W, kKS, 0, w, lane, wh[0], wl[0]);
  load_x<PARTS>(Xs, 0, lane, xh[0], xl[0]);
#pragma unroll
  for (int ks = 0; ks < kKS; ks++) {
    if (ks + 1 < kKS) {
      load_wc<PARTS>(W, kKS, ks + 1, w, lane, wh[(ks + 1) & 1], wl[(ks + 1) & 1]);
      load_x<PARTS>(Xs, ks + 1, lane, xh[(ks + 1) & 1], xl[(ks + 1) & 1]);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of this step's products
    mma_sweeps<PARTS, 2>(wh[ks & 1], wl[ks & 1], xh[ks & 1], xl[ks & 1], acc);
  }
}

template <int U>
__device__ __forceinline__ void zero_tile(f4v (&a)[U][4]) {
#pragma unroll
  for (int u = 0; u < U; u++)
#pragma unroll
    for (int rt = 0; rt < 4; rt++) a[u][rt] = f4v{0.f, 0.f, 0.f, 0.f};
}

// ------------------------------------------------------------------------------------
// first layer forward: t1 = tanh(D W1 + b1), K = 16 M consumed 32 at a time.  The D
// fragment slot of row 16 dr + rb (dr = w % 4) for a k step holds D[row][a][b] with
// a = 2 s + g / 2, b = 8 (g % 2) + j; wave w forms its half j = 4 (w / 4) .. + 3 from
// T[row][a] and T<[row][b] (in registers for the whole loop).  D slices are
// double-buffered in LDS with one barrier per step; the wave's weight fragments are
// fetched one step ahead.
// ------------------------------------------------------------------------------------
template <int PARTS>
__global__ __launch_bounds__(FT) void k_fit_l1_fwd(FitBfArgs P) {
  __shared__ __align__(16) __bf16 Ds[2][4 * PARTS * 512];
  const int r0 = blockIdx.x * FR;
  const int sp = fitbf_species(P, r0);
  if (sp < 0) return;
  const int M = P.M, KS = M / 2, N = P.N, NT = N / 16;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, rb = lane & 15,
            g = lane >> 4;
  const int dr = w & 3, dh = w >> 2;
  const int row = r0 + 16 * dr + rb;
  const bool real = P.row_atom[row] >= 0;
  const float* Tr = P.T + (size_t)row * M * 4;
  const f4v z4 = {0.f, 0.f, 0.f, 0.f};
  f4v tl[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    tl[j] = *(const f4v*)(Tr + 4 * (8 * (g & 1) + 4 * dh + j));   // pad rows: loaded, then zeroed
    if (!real) tl[j] = z4;
  }
  const __bf16* W = (const __bf16*)P.Wf[(sp * P.nfit) * 2];
  f4v acc[2][4];
  zero_tile(acc);
  bf8 ah[2], al[2], bh[2], bl[2];
  f4v ta;
  __bf16* dslot = &Ds[0][0] + (dr * PARTS) * 512 + lane * 8 + 4 * dh;
#define L1_LOAD_T(S_) ta = *(const f4v*)(Tr + 4 * (2 * (S_) + (g >> 1)))
#define L1_FORM_D(BUF_)                                                                           \
  do {                                                                                            \
    const f4v tv_ = real ? ta : z4;                                                               \
    f4v d_;                                                                                       \
    _Pragma("unroll") for (int j = 0; j < 4; j++) d_[j] =                                         \
        tv_[0] * tl[j][0] + tv_[1] * tl[j][1] + tv_[2] * tl[j][2] + tv_[3] * tl[j][3];            \
    bf4 h_, l_;                                                                                   \
    split4<PARTS>(d_, h_, l_);                                                                    \
    *(bf4*)(dslot + (BUF_) * 4 * PARTS * 512) = h_;                                               \
    if (PARTS == 2) *(bf4*)(dslot + (BUF_) * 4 * PARTS * 512 + 512) = l_;                         \
  } while (0)
  // KS is even; fetches past the last step are clamped to it (harmless repeats), so no
  // load sits behind a branch and the wait counts stay exact.  The prologue issues in
  // the loop's order (T of the next step, then the b fragments), so that the wait
  // counts at the loop head agree on both incoming paths.
  L1_LOAD_T(0);
  load_wc<PARTS>(W, KS, 0, w, lane, ah, al);
  L1_FORM_D(0);
  L1_LOAD_T(1);
  __builtin_amdgcn_sched_barrier(0);
  load_wc<PARTS>(W, KS, 1, w, lane, bh, bl);
  __syncthreads();
  for (int s = 0; s < KS; s += 2) {
    const int s2 = min(s + 2, KS - 1), s3 = min(s + 3, KS - 1);
    mma_step<PARTS>(ah, al, Ds[0], 0, lane, acc);
    __builtin_amdgcn_sched_barrier(0);
    load_wc<PARTS>(W, KS, s2, w, lane, ah, al);
    __builtin_amdgcn_sched_barrier(0);   // the fetch two steps ahead stays here
    L1_FORM_D(1);   // step s + 1
    L1_LOAD_T(s2);
    __syncthreads();
    mma_step<PARTS>(bh, bl, Ds[1], 0, lane, acc);
    __builtin_amdgcn_sched_barrier(0);
    load_wc<PARTS>(W, KS, s3, w, lane, bh, bl);
    __builtin_amdgcn_sched_barrier(0);
    L1_FORM_D(0);   // step s + 2 (unused after the last step)
    L1_LOAD_T(s3);
    __syncthreads();
  }
#undef L1_LOAD_T
#undef L1_FORM_D
  const float* bias = (const float*)P.bias[sp * P.nfit];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int ct = w + 8 * u;
    if (ct >= NT) continue;
    const f4v bv = gld<f4v>(bias + 16 * ct + 4 * g);
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
      f4v t;
#pragma unroll
      for (int q = 0; q < 4; q++) t[q] = dp_tanh(acc[u][rt][q] + bv[q]);
      *(f4v*)(P.t1 + (size_t)(r0 + 16 * rt + rb) * N + 16 * ct + 4 * g) = t;
    }
  }
}

// ------------------------------------------------------------------------------------
// square layers, output and the adjoint back to the first layer
// ------------------------------------------------------------------------------------
// LDS of the tail: the staged X fragments, the row sums of E_i and the tanh of the first
// square layer (the last one stays in registers; deeper nets keep the middle ones in the
// workspace)
size_t fit_tail_lds(int parts) {
  return (size_t)kKS * 4 * parts * 1024 + FW * 64 * 8 + (size_t)16 * 4 * 64 * 16;
}

template <int PARTS>
__global__ __launch_bounds__(FT) void k_fit_tail(FitBfArgs P) {
  extern __shared__ __align__(16) char smem[];
  const int N = P.N, NT = N / 16;
  __bf16* Xs = (__bf16*)smem;
  double* red = (double*)(smem + (size_t)kKS * 4 * PARTS * 1024);
  float* act1 = (float*)(smem + (size_t)kKS * 4 * PARTS * 1024 + FW * 64 * 8);   // [NT][4][64][4]
  const int r0 = blockIdx.x * FR;
  const int sp = fitbf_species(P, r0);
  if (sp < 0) return;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, rb = lane & 15,
            g = lane >> 4;
  // the k >= N tail of the last fragment step stays zero
  for (int q = tid; q < kKS * 4 * PARTS * 64; q += FT) ((u32x4v*)Xs)[q] = u32x4v{0u, 0u, 0u, 0u};
  const f4v z4 = {0.f, 0.f, 0.f, 0.f};
  f4v x[2][4];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int ct = w + 8 * u;
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
      x[u][rt] = ct < NT ? *(const f4v*)(P.t1 + (size_t)(r0 + 16 * rt + rb) * N + 16 * ct + 4 * g) : z4;
  }
  const size_t lstride = (size_t)P.nrows * N;
  // per-lane slot of a square layer's tanh: (ct, rt) tile, lane order
#define TAIL_ACT(BASE_, U_, RT_) (*(f4v*)((BASE_) + ((size_t)((w + 8 * (U_)) * 4 + (RT_)) * 64 + lane) * 4))
  f4v acc[2][4], tk[2][4];   // tk: tanh of the latest square layer
  for (int k = 1; k < P.nfit; k++) {
    __syncthreads();
    stage_tile<PARTS>(Xs, x, w, NT, rb, g);
    __syncthreads();
    zero_tile(acc);
    tile_mm<PARTS>((const __bf16*)P.Wf[(sp * P.nfit + k) * 2], w, lane, Xs, acc);
    const float* bias = (const float*)P.bias[sp * P.nfit + k];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      const int ct = w + 8 * u;
      const f4v bv = ct < NT ? gld<f4v>(bias + 16 * ct + 4 * g) : z4;
#pragma unroll
      for (int rt = 0; rt < 4; rt++) {
#pragma unroll
        for (int q = 0; q < 4; q++) tk[u][rt][q] = ct < NT ? dp_tanh(acc[u][rt][q] + bv[q]) : 0.f;
        x[u][rt] += tk[u][rt];
      }
    }
    if (k < P.nfit - 1) {   // kept for the adjoint: the first in LDS, deeper ones in the workspace
      float* dst = k == 1 ? act1 : P.act + k * lstride + (size_t)r0 * N;
#pragma unroll
      for (int u = 0; u < 2; u++)
        if (w + 8 * u < NT)
#pragma unroll
          for (int rt = 0; rt < 4; rt++) TAIL_ACT(dst, u, rt) = tk[u][rt];
    }
  }
  // E_i = x . w_o + b_o, FP64 sums
  const float* wo = (const float*)P.wo[sp];
  f4v wv[2];
#pragma unroll
  for (int u = 0; u < 2; u++) wv[u] = w + 8 * u < NT ? gld<f4v>(wo + 16 * (w + 8 * u) + 4 * g) : z4;
  double e[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 2; u++)
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
      for (int q = 0; q < 4; q++) e[rt] += (double)x[u][rt][q] * (double)wv[u][q];
#pragma unroll
  for (int rt = 0; rt < 4; rt++) {
    e[rt] += __shfl_xor(e[rt], 16);
    e[rt] += __shfl_xor(e[rt], 32);
  }
  if (g == 0)
#pragma unroll
    for (int rt = 0; rt < 4; rt++) red[w * 64 + 16 * rt + rb] = e[rt];
  __syncthreads();
  if (tid < 64) {
    const int row = r0 + tid;
    double s = 0.0;
    for (int v = 0; v < FW; v++) s += red[v * 64 + tid];
    P.Ei[row] = P.row_atom[row] >= 0 ? s + P.bo[sp] : 0.0;
  }
  // adjoint: g_L = w_o; g_{k-1} = g_k + (g_k (1 - t_k^2)) W_k^T
  f4v gr[2][4];
#pragma unroll
  for (int u = 0; u < 2; u++)
#pragma unroll
    for (int rt = 0; rt < 4; rt++) gr[u][rt] = wv[u];
  for (int k = P.nfit - 1; k >= 1; k--) {
    if (k < P.nfit - 1) {   // the last layer's tanh is still in tk
      const float* src = k == 1 ? act1 : P.act + k * lstride + (size_t)r0 * N;
#pragma unroll
      for (int u = 0; u < 2; u++)
#pragma unroll
        for (int rt = 0; rt < 4; rt++) tk[u][rt] = w + 8 * u < NT ? TAIL_ACT(src, u, rt) : z4;
    }
    f4v d[2][4];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int rt = 0; rt < 4; rt++) d[u][rt] = gr[u][rt] * (1.f - tk[u][rt] * tk[u][rt]);
    __syncthreads();
    stage_tile<PARTS>(Xs, d, w, NT, rb, g);
    __syncthreads();
    zero_tile(acc);
    tile_mm<PARTS>((const __bf16*)P.Wf[(sp * P.nfit + k) * 2 + 1], w, lane, Xs, acc);
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int rt = 0; rt < 4; rt++) gr[u][rt] += acc[u][rt];
  }
#undef TAIL_ACT
  // d1 = g1 (1 - t1^2) as fragments for the first layer's adjoint; pad rows and the
  // k >= N tail are zero (ct runs over all 2 kKS = 16 tiles)
  __bf16* out = P.d1f + (size_t)blockIdx.x * kKS * 4 * PARTS * 512;
  bool real[4];
#pragma unroll
  for (int rt = 0; rt < 4; rt++) real[rt] = P.row_atom[r0 + 16 * rt + rb] >= 0;
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int ct = w + 8 * u;
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
      f4v v = z4;
      if (ct < NT && real[rt]) {
        const f4v t = *(const f4v*)(P.t1 + (size_t)(r0 + 16 * rt + rb) * N + 16 * ct + 4 * g);
        v = gr[u][rt] * (1.f - t * t);
      }
      put4<PARTS>(out, ct, rt, rb, g, v);
    }
  }
}

// ------------------------------------------------------------------------------------
// first layer adjoint and the descriptor adjoint.  Output tile a of dD = d1 W1^T holds
// dD[row][a][b] for b < 16 in lane (rb = row, g) as b = 4 g + q, so
//   dE/dT[row][a][c]  = sum_b dD[row][a][b] T[row][b][c]     (sum over q in the lane, then
//                                                               a reduce-scatter over g)
//   dE/dT[row][b][c] += sum_a dD[row][a][b] T[row][a][c]     (b < 16; accumulated per lane
//                                                               over the wave's a, the
//                                                               waves' parts added in order)
// Wave w takes an even-sized a range, two a per pass; d1 fragments and T< sit in LDS, the
// wave's weight fragments are fetched one step ahead.
// ------------------------------------------------------------------------------------
// Reduce-scatter of four values over the four lane groups g (lanes rb + 16 g): returns
// in lane group g the sum over g' of v[g] held by group g'.  v_permlane32_swap trades
// the upper half of its first operand with the lower half of its second, so summing
// the swapped (v0, v2) pair leaves component 0 summed over g, g + 2 in lanes < 32 and
// component 2 in lanes >= 32 (likewise (v1, v3)); v_permlane16_swap then trades the odd
// rows of the first operand with the even rows of the second, finishing the sum.
__device__ __forceinline__ float rs4(f4v v) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]), __float_as_uint(v[2]), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[1]), __float_as_uint(v[3]), false, false);
  const float k0 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const float k1 = __uint_as_float(b[0]) + __uint_as_float(b[1]);
  const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(k0), __float_as_uint(k1), false, false);
  return __uint_as_float(c[0]) + __uint_as_float(c[1]);
}

constexpr int kTlStride = 68;   // floats per row of the staged T< (bank spread)
constexpr int kRowF = 68;        // floats per row of the [64][16][4] second-term and T1 tiles (bank spread)

size_t fit_l1_bwd_lds(int parts) {
  const size_t xs = (size_t)kKS * 4 * parts * 1024, p2 = (size_t)4 * 64 * kRowF * 4;
  return (xs > p2 ? xs : p2) + 64 * kRowF * 4 + 64 * kTlStride * 4;
}

// the weight fragments of the output tiles (a, a + 1) at k step ks
template <int PARTS>
__device__ __forceinline__ void load_w2(const __bf16* __restrict__ W, int a, int ks, int lane, bf8 (&wh)[2],
                                        bf8 (&wl)[2]) {
  wfrag<PARTS>(W, kKS, a, ks, lane, wh[0], wl[0]);
  wfrag<PARTS>(W, kKS, a + 1, ks, lane, wh[1], wl[1]);
}

template <int PARTS>
__global__ __launch_bounds__(FT) void k_fit_l1_bwd(FitBfArgs P) {
  extern __shared__ __align__(16) char smem[];
  const int M = P.M;
  const size_t xs_bytes = (size_t)kKS * 4 * PARTS * 1024, p2_bytes = (size_t)4 * 64 * kRowF * 4;
  __bf16* Xs = (__bf16*)smem;
  float* P2 = (float*)smem;                                                     // after the GEMMs: [4][64][kRowF]
  float* T1s = (float*)(smem + (xs_bytes > p2_bytes ? xs_bytes : p2_bytes));   // [64][kRowF]: [16][4] used
  float* Tls = T1s + 64 * kRowF;                                                // [64][kTlStride]: T<
  const int r0 = blockIdx.x * FR;
  const int sp = fitbf_species(P, r0);
  if (sp < 0) return;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, rb = lane & 15,
            g = lane >> 4;
  {
    const u32x4v* src = (const u32x4v*)(P.d1f + (size_t)blockIdx.x * kKS * 4 * PARTS * 512);
    for (int q = tid; q < kKS * 4 * PARTS * 64; q += FT) ((u32x4v*)Xs)[q] = src[q];
  }
  const f4v z4 = {0.f, 0.f, 0.f, 0.f};
  // T< of the tile's rows (pad rows zero)
  for (int q = tid; q < 64 * 16; q += FT) {
    const int rl = q >> 4, b = q & 15;
    f4v v = *(const f4v*)(P.T + ((size_t)(r0 + rl) * M + b) * 4);
    if (P.row_atom[r0 + rl] < 0) v = z4;
    *(f4v*)(Tls + rl * kTlStride + 4 * b) = v;
  }
  bool real[4];
  const float* Trow[4];
#pragma unroll
  for (int rt = 0; rt < 4; rt++) {
    const int row = r0 + 16 * rt + rb;
    real[rt] = P.row_atom[row] >= 0;
    Trow[rt] = P.T + (size_t)row * M * 4;
  }
  f4v p2[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int q = 0; q < 4; q++) p2[rt][q] = z4;
  const __bf16* W = (const __bf16*)P.Wf[(sp * P.nfit) * 2 + 1];
  // a range of this wave: whole pairs (M is even), two tiles per pass, the M / 2 pairs
  // dealt evenly over the waves (waves w and w + 4 share a SIMD's MFMA: with 100 a this
  // gives each SIMD 24 or 26 of them)
  const int np = M / 2, pw = np / FW, px = np % FW;
  const int p0 = w * pw + min(w, px);
  const int a0 = 2 * p0, a1 = 2 * (p0 + pw + (w < px ? 1 : 0));
  __syncthreads();
  bf8 wh[2][2], wl[2][2];   // [buffer][tile of the pair]
  bf8 xh[2][4], xl[2][4];   // [buffer][row tile]
  if (a0 < a1) load_w2<PARTS>(W, a0, 0, lane, wh[0], wl[0]);
  load_x<PARTS>(Xs, 0, lane, xh[0], xl[0]);
  for (int a = a0; a < a1; a += 2) {
    const int an = min(a + 2, a1 - 2);   // next pass (the last pass repeats itself)
    f4v acc[2][4], tav[2][4];
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
      for (int rt = 0; rt < 4; rt++) {
        acc[c][rt] = z4;
        tav[c][rt] = *(const f4v*)(Trow[rt] + (a + c) * 4);
      }
#pragma unroll
    for (int ks = 0; ks < kKS; ks++) {
      const int nb = (ks + 1) & 1;   // kKS is even: every pass starts at buffer 0
      if (ks + 1 < kKS) load_w2<PARTS>(W, a, ks + 1, lane, wh[nb], wl[nb]);
      else load_w2<PARTS>(W, an, 0, lane, wh[nb], wl[nb]);
      load_x<PARTS>(Xs, (ks + 1) % kKS, lane, xh[nb], xl[nb]);
      __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of this step's products
      mma_sweeps<PARTS, 2>(wh[ks & 1], wl[ks & 1], xh[ks & 1], xl[ks & 1], acc);
    }
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
      f4v tl[4];   // T[row_rt][4 g + q]
#pragma unroll
      for (int q = 0; q < 4; q++) tl[q] = *(const f4v*)(Tls + (16 * rt + rb) * kTlStride + 4 * (4 * g + q));
#pragma unroll
      for (int c = 0; c < 2; c++) {
        const f4v cv = acc[c][rt];
        // first term: sum over b = 4 g + q (in the lane, then over g by a reduce-scatter
        // that leaves component c = g in lane group g)
        const f4v pv = cv[0] * tl[0] + cv[1] * tl[1] + cv[2] * tl[2] + cv[3] * tl[3];
        const float kk = rs4(pv);
        if (a + c >= 16) P.gT[((size_t)(r0 + 16 * rt + rb) * M + a + c) * 4 + g] = kk;
        else T1s[(16 * rt + rb) * kRowF + (a + c) * 4 + g] = kk;
        // second term, accumulated over the wave's a
        const f4v tv = real[rt] ? tav[c][rt] : z4;
#pragma unroll
        for (int q = 0; q < 4; q++) p2[rt][q] += cv[q] * tv;
      }
    }
  }
  // second-term parts of the 8 waves, added in a fixed order: waves 4..7 hand theirs to
  // waves 0..3, which then hand the pair sums to the final pass
  float* mine = P2 + (size_t)(w & 3) * 64 * kRowF;
  __syncthreads();   // every read of the d1 fragments is done; P2 reuses that space
  if (w >= 4)
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
      for (int q = 0; q < 4; q++) *(f4v*)(mine + (16 * rt + rb) * kRowF + (4 * g + q) * 4) = p2[rt][q];
  __syncthreads();
  if (w < 4)
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        f4v* p = (f4v*)(mine + (16 * rt + rb) * kRowF + (4 * g + q) * 4);
        *p = p2[rt][q] + *p;
      }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += FT) {
    const int rl = e >> 6, b = (e >> 2) & 15, c = e & 3, x = rl * kRowF + 4 * b + c;
    constexpr int S = 64 * kRowF;
    const float v = T1s[x] + (((P2[x] + P2[S + x]) + P2[2 * S + x]) + P2[3 * S + x]);
    P.gT[((size_t)(r0 + rl) * M + b) * 4 + c] = v;
  }
}

bool fit_bf_supported(int M, int m2, int N) {
  return m2 == 16 && M >= 16 && M % 4 == 0 && N >= 16 && N % 16 == 0 && N <= 256;
}

void launch_fit_bf(const FitArgs& F, hipStream_t st) {
  const int parts = F.prec == PREC_BF16X3 ? 2 : 1;
  FitBfArgs P{};
  P.M = F.m.M;
  P.N = F.fw;
  P.nfit = F.nfit;
  P.ntypes = F.m.ntypes;
  P.nrows = F.nrows;
  P.type_row0 = F.type_row0;
  P.row_atom = F.row_atom;
  P.T = (const float*)F.T;
  P.Wf = F.Wf;
  P.bias = F.b;
  P.wo = F.wo;
  P.bo = F.bo;
  P.t1 = (float*)F.xs;
  P.act = (float*)F.act;
  P.d1f = (__bf16*)F.Dg;
  P.Ei = F.Ei;
  P.gT = (float*)F.gT;
  const dim3 grid((F.nrows + FR - 1) / FR), block(FT);
  const size_t sh_tail = fit_tail_lds(parts), sh_bwd = fit_l1_bwd_lds(parts);
  if (parts == 2) {
    (void)hipFuncSetAttribute((const void*)k_fit_tail<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_tail);
    (void)hipFuncSetAttribute((const void*)k_fit_l1_bwd<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_bwd);
    hipLaunchKernelGGL(k_fit_l1_fwd<2>, grid, block, 0, st, P);
    hipLaunchKernelGGL(k_fit_tail<2>, grid, block, sh_tail, st, P);
    hipLaunchKernelGGL(k_fit_l1_bwd<2>, grid, block, sh_bwd, st, P);
  } else {
    (void)hipFuncSetAttribute((const void*)k_fit_tail<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_tail);
    (void)hipFuncSetAttribute((const void*)k_fit_l1_bwd<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_bwd);
    hipLaunchKernelGGL(k_fit_l1_fwd<1>, grid, block, 0, st, P);
    hipLaunchKernelGGL(k_fit_tail<1>, grid, block, sh_tail, st, P);
    hipLaunchKernelGGL(k_fit_l1_bwd<1>, grid, block, sh_bwd, st, P);
  }
}

}  // namespace dp
