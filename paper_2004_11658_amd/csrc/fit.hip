// Descriptor and fitting net (paper Section 2, Eq. 1-4) with their adjoint.
//
// Rows are centre atoms grouped by species (row groups padded to 64, so a 64-row GEMM
// tile never mixes species and every tile uses one fitting net).  Per species:
//   D   = T T<^T flattened a * M< + b                       (Eq. 4)
//   x1  = tanh(D W1 + b1)                                    first layer, no skip
//   xk  = x_{k-1} + tanh(x_{k-1} Wk + bk)                    Eq. 3
//   E_i = x_last . w_o + b_o
// and back: g_last = w_o; g_{k-1} = g_k + (g_k * (1 - t_k^2)) Wk^T; dD = (g_1 (1 - t_1^2)) W1^T;
// dE/dT from dD.  GEMMs run on the 16x16x4 MFMA (FP64 or FP32 operands) or, in the BF16
// modes, on the 16x16x32 BF16 MFMA with FP32 accumulation (activations are rounded to
// BF16 while they are staged; the split mode adds the lo parts as hi lo + lo hi),
// 64x128 output tiles per workgroup, with the bias, tanh and skip fused into the
// epilogue and the 1 - tanh^2 factor fused into operand staging (the paper's fused
// TANH / TANHGrad, Section 3.2.3).
#include <hip/hip_runtime.h>

#include "bf16ops.h"
#include "common.h"
#include "embed_common.h"
#include "kernels.h"
#include "devmath.h"

namespace dp {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
template <class T> struct FAcc4;
template <> struct FAcc4<double> { typedef d4v type; };
template <> struct FAcc4<float> { typedef f4v type; };

__device__ __forceinline__ d4v fmfma4(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v fmfma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T>
__device__ __forceinline__ T ftanh(T x) { return dp_tanh(x); }

enum Epi { EPI_FWD1 = 0, EPI_FWDRES = 1, EPI_BWD = 2, EPI_BWD1 = 3 };

constexpr int BM = 64;    // output tile rows (one species per tile)
constexpr int BN = 128;   // output tile columns

// Output tile of this workgroup.  Workgroups are dealt to the 8 XCDs round robin
// (block b runs on XCD b % 8), each XCD with its own L2; the mapping gives every XCD a
// contiguous range of tiles, columns fastest, so the column tiles of one row tile
// (which read the same activation rows) run on one XCD and share its L2.
__device__ __forceinline__ void gemm_tile(int nct, int& r0, int& n0) {
  const int nb = gridDim.x, b = blockIdx.x, x = b & 7;
  const int q = nb >> 3, r = nb & 7;
  const int L = x * q + (x < r ? x : r) + (b >> 3);
  r0 = (L / nct) * BM;
  n0 = (L % nct) * BN;
}

struct GemmArgs {
  int nrows, K, N;
  const void* const* Wb; // BF16 modes: operand table (see FitArgs::Wb)

  const int* type_row0;
  int ntypes;
  const void* A;        // [nrows][K]
  const void* Aaux;     // BWD: t of this layer [nrows][K] (A staged as A * (1 - t^2))
  const void* const* W;  // per species weight pointer table (row major [K_w][N_w])
  int wsel;             // index offset into the table: species * wstride + wsel
  int wstride;
  const void* const* bias;
  const void* Xprev;    // FWDRES: x_{k-1} [nrows][N]; BWD: skip source g_k [nrows][N]
  void* out;            // [nrows][N]
  void* out2;           // FWD*: tanh part [nrows][N]
};

// 64 x 128 output tile per workgroup of 4 waves; wave w owns columns [32 w, 32 w + 32)
// as 4 x 2 MFMA tiles.  K is consumed in tiles of KT (16 doubles / 32 floats) staged
// in LDS; the next tile is prefetched into registers while the current one is used.
template <class T, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs G) {
  constexpr int KT = sizeof(T) == 8 ? 16 : 32;
  constexpr int APT = BM * KT / 256;     // A elements per thread per tile
  constexpr int BPT = KT * BN / 256;     // B elements per thread per tile
  __shared__ T As[BM][KT + 1];
  __shared__ T Bs[KT][BN + 1];
  int r0, n0;
  gemm_tile((G.N + BN - 1) / BN, r0, n0);
  int sp = -1;
  for (int t = 0; t < G.ntypes; t++)
    if (r0 >= G.type_row0[t] && r0 < G.type_row0[t + 1]) sp = t;
  if (sp < 0) return;
  const T* __restrict__ A = (const T*)G.A;
  const T* __restrict__ At = (const T*)G.Aaux;
  const T* __restrict__ W = (const T*)G.W[sp * G.wstride + G.wsel];
  constexpr bool transW = (EPI == EPI_BWD || EPI == EPI_BWD1);
  const int K = G.K, N = G.N;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, rb = lane & 15, g = lane >> 4;
  const int wc = wv * 32;
  typedef typename FAcc4<T>::type A4;
  A4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = A4{0, 0, 0, 0};
  T ra[APT], rbv[BPT];
  // A tile element e = tid + 256 j: row e / KT, k e % KT (consecutive threads along k)
  // B tile (not transposed) element e: k e / BN, col e % BN (consecutive along columns)
  // B tile (transposed W): element e: col e / KT, k e % KT (consecutive along k of W rows)
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < APT; j++) {
      int e = tid + 256 * j, r = e / KT, k = e % KT;
      int gk = k0 + k;
      T v = (T)0;
      if (gk < K) {
        size_t o = (size_t)(r0 + r) * K + gk;
        v = A[o];
        if (EPI == EPI_BWD || EPI == EPI_BWD1) {
          T t = At[o];
          v = v * ((T)1 - t * t);
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < BPT; j++) {
      int e = tid + 256 * j;
      int k, c;
      if (transW) { c = e / KT; k = e % KT; }
      else { k = e / BN; c = e % BN; }
      int gk = k0 + k, gc = n0 + c;
      T v = (T)0;
      if (gk < K && gc < N) v = transW ? W[(size_t)gc * K + gk] : W[(size_t)gk * N + gc];
      rbv[j] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int j = 0; j < APT; j++) {
      int e = tid + 256 * j;
      As[e / KT][e % KT] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < BPT; j++) {
      int e = tid + 256 * j;
      if (transW) Bs[e % KT][e / KT] = rbv[j];
      else Bs[e / BN][e % BN] = rbv[j];
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KT) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + KT < K) load(k0 + KT);
#pragma unroll
    for (int ks = 0; ks < KT; ks += 4) {
      T av[4], bv[2];
#pragma unroll
      for (int a = 0; a < 4; a++) av[a] = As[16 * a + rb][ks + g];
#pragma unroll
      for (int b = 0; b < 2; b++) bv[b] = Bs[ks + g][wc + 16 * b + rb];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = fmfma4(av[a], bv[b], acc[a][b]);
    }
  }
  // epilogue: lane holds column (wc + 16 b + rb) and four rows of each 16-row tile
  T* out = (T*)G.out;
  T* out2 = (T*)G.out2;
  const T* X = (const T*)G.Xprev;
  const T* bias = (EPI == EPI_FWD1 || EPI == EPI_FWDRES) ? (const T*)G.bias[sp * G.wstride + G.wsel] : nullptr;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      int col = n0 + wc + 16 * b + rb;
      if (col >= N) continue;
      T bc = bias ? bias[col] : (T)0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // FP64 16x16x4 results hold rows g + 4q, FP32 rows 4g + q
        int row = r0 + 16 * a + (sizeof(T) == 8 ? g + 4 * q : 4 * g + q);
        size_t o = (size_t)row * N + col;
        T v = acc[a][b][q];
        if (EPI == EPI_FWD1) {
          T t = ftanh(v + bc);
          out[o] = t;
          out2[o] = t;
        } else if (EPI == EPI_FWDRES) {
          T t = ftanh(v + bc);
          out[o] = X[o] + t;
          out2[o] = t;
        } else if (EPI == EPI_BWD) {
          out[o] = X[o] + v;
        } else {
          out[o] = v;
        }
      }
    }
}

typedef __bf16 fbf8 __attribute__((ext_vector_type(8)));
typedef __bf16 fbf4 __attribute__((ext_vector_type(4)));

// BF16 operands: the same 64 x 128 tile and wave split as k_gemm, K consumed in tiles
// of 64 (two MFMA k steps of 32).  Both operands sit in LDS k-contiguous, [row][k] for
// the activations and [column][k] for the weights (the forward reads W^T, the adjoint
// W, both pre-packed in BF16), so every lane reads its 8 k values with one 16-byte
// load.  K must be a multiple of 8 (checked when the model is loaded).
template <int PARTS, int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf(GemmArgs G) {
  constexpr int KT = 64, LDK = KT + 8;
  __shared__ __align__(16) __bf16 As[PARTS][BM][LDK];
  __shared__ __align__(16) __bf16 Bs[PARTS][BN][LDK];
  int r0, n0;
  gemm_tile((G.N + BN - 1) / BN, r0, n0);
  int sp = -1;
  for (int t = 0; t < G.ntypes; t++)
    if (r0 >= G.type_row0[t] && r0 < G.type_row0[t + 1]) sp = t;
  if (sp < 0) return;
  constexpr bool bwd = (EPI == EPI_BWD || EPI == EPI_BWD1);
  const float* __restrict__ A = (const float*)G.A;
  const float* __restrict__ At = (const float*)G.Aaux;
  const int wi = (sp * G.wstride + G.wsel) * 4 + (bwd ? 2 : 0);
  const __bf16* __restrict__ Wh = (const __bf16*)G.Wb[wi];
  const __bf16* __restrict__ Wl = (const __bf16*)G.Wb[wi + 1];
  const int K = G.K, N = G.N;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, rb = lane & 15, g = lane >> 4;
  const int wc = wv * 32;
  f4v acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = f4v{0, 0, 0, 0};
  // A tile: 64 rows x 64 k as 1024 float4, thread t takes t + 256 j: row e / 16, k 4 (e % 16)
  // B tile: 128 columns x 64 k as 1024 groups of 8, thread t takes t + 256 j: col e / 8, k 8 (e % 8)
  float4 ra[4];
  uint4 rbh[4], rbl[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int e = tid + 256 * j, r = e >> 4, k = k0 + 4 * (e & 15);
      float4 v = {0.f, 0.f, 0.f, 0.f};
      if (k < K) {
        size_t o = (size_t)(r0 + r) * K + k;
        v = *(const float4*)(A + o);
        if (bwd) {
          float4 t = *(const float4*)(At + o);
          v.x *= 1.f - t.x * t.x;
          v.y *= 1.f - t.y * t.y;
          v.z *= 1.f - t.z * t.z;
          v.w *= 1.f - t.w * t.w;
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int e = tid + 256 * j, c = n0 + (e >> 3), k = k0 + 8 * (e & 7);
      uint4 h = {0, 0, 0, 0}, l = {0, 0, 0, 0};
      if (k < K && c < N) {
        size_t o = (size_t)c * K + k;
        h = *(const uint4*)(Wh + o);
        if (PARTS == 2) l = *(const uint4*)(Wl + o);
      }
      rbh[j] = h;
      rbl[j] = l;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int e = tid + 256 * j, r = e >> 4, k = 4 * (e & 15);
      float x[4] = {ra[j].x, ra[j].y, ra[j].z, ra[j].w};
      fbf4 h, l;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        __bf16 hv = (__bf16)x[i];
        h[i] = hv;
        if (PARTS == 2) l[i] = (__bf16)(x[i] - (float)hv);
      }
      *(fbf4*)&As[0][r][k] = h;
      if (PARTS == 2) *(fbf4*)&As[1][r][k] = l;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int e = tid + 256 * j, c = e >> 3, k = 8 * (e & 7);
      *(uint4*)&Bs[0][c][k] = rbh[j];
      if (PARTS == 2) *(uint4*)&Bs[1][c][k] = rbl[j];
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KT) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + KT < K) load(k0 + KT);
#pragma unroll
    for (int ks = 0; ks < KT; ks += 32) {
      fbf8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < 4; a++) {
        ah[a] = *(const fbf8*)&As[0][16 * a + rb][ks + 8 * g];
        al[a] = PARTS == 2 ? *(const fbf8*)&As[1][16 * a + rb][ks + 8 * g] : ah[a];
      }
#pragma unroll
      for (int b = 0; b < 2; b++) {
        bh[b] = *(const fbf8*)&Bs[0][wc + 16 * b + rb][ks + 8 * g];
        bl[b] = PARTS == 2 ? *(const fbf8*)&Bs[1][wc + 16 * b + rb][ks + 8 * g] : bh[b];
      }
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
          if (PARTS == 2) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
  }
  float* out = (float*)G.out;
  float* out2 = (float*)G.out2;
  const float* X = (const float*)G.Xprev;
  const float* bias = (EPI == EPI_FWD1 || EPI == EPI_FWDRES) ? (const float*)G.bias[sp * G.wstride + G.wsel]
                                                           : nullptr;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      int col = n0 + wc + 16 * b + rb;
      if (col >= N) continue;
      float bc = bias ? bias[col] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int row = r0 + 16 * a + 4 * g + q;
        size_t o = (size_t)row * N + col;
        float v = acc[a][b][q];
        if (EPI == EPI_FWD1) {
          float t = ftanh(v + bc);
          out[o] = t;
          out2[o] = t;
        } else if (EPI == EPI_FWDRES) {
          float t = ftanh(v + bc);
          out[o] = X[o] + t;
          out2[o] = t;
        } else if (EPI == EPI_BWD) {
          out[o] = X[o] + v;
        } else {
          out[o] = v;
        }
      }
    }
}

// D[row][a m2 + b] = sum_c T[row][a][c] T[row][b][c]; pad rows get zeros
template <class T>
__global__ void k_desc(int nrows, int M, int m2, const int* __restrict__ row_atom,
                       const T* __restrict__ Tm, T* __restrict__ D) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)nrows * M * m2;
  if (q >= tot) return;
  int row = (int)(q / (M * m2));
  int ab = (int)(q % (M * m2));
  int a = ab / m2, b = ab % m2;
  T v = (T)0;
  if (row_atom[row] >= 0) {
    const T* t = Tm + (size_t)row * M * 4;
    v = t[a * 4] * t[b * 4] + t[a * 4 + 1] * t[b * 4 + 1] + t[a * 4 + 2] * t[b * 4 + 2] +
        t[a * 4 + 3] * t[b * 4 + 3];
  }
  D[q] = v;
}

// dE/dT[p][c] = sum_b dD[p][b] T[b][c] + [p < m2] sum_a dD[a][p] T[a][c]
// one workgroup per row: T and dD of the row staged in LDS
template <class T>
__global__ __launch_bounds__(256) void k_desc_bwd(int nrows, int M, int m2, const int* __restrict__ row_atom,
                                                 const T* __restrict__ Tm, const T* __restrict__ Dg,
                                                 T* __restrict__ gT) {
  extern __shared__ __align__(16) char sm[];
  T* st = (T*)sm;               // [M][4]
  T* sd = st + M * 4;           // [M][m2]
  const int row = blockIdx.x;
  T* o = gT + (size_t)row * M * 4;
  if (row_atom[row] < 0) {
    for (int q = threadIdx.x; q < M * 4; q += blockDim.x) o[q] = (T)0;
    return;
  }
  const T* t = Tm + (size_t)row * M * 4;
  const T* dg = Dg + (size_t)row * M * m2;
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) st[q] = t[q];
  for (int q = threadIdx.x; q < M * m2; q += blockDim.x) sd[q] = dg[q];
  __syncthreads();
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) {
    int p = q >> 2, c = q & 3;
    T v = (T)0;
    for (int b = 0; b < m2; b++) v += sd[p * m2 + b] * st[b * 4 + c];
    if (p < m2)
      for (int a = 0; a < M; a++) v += sd[a * m2 + p] * st[a * 4 + c];
    o[q] = v;
  }
}

// E_i = x . w_o + b_o (FP64 accumulation) and the backward seed g = w_o; one wave per row
template <class T>
__global__ void k_fit_out(int nrows, int N, int ntypes, const int* __restrict__ type_row0,
                          const int* __restrict__ row_atom, const T* __restrict__ X,
                          const void* const* __restrict__ wo, const double* __restrict__ bo,
                          double* __restrict__ Ei, T* __restrict__ gseed) {
  int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  int sp = -1;
  for (int t = 0; t < ntypes; t++)
    if (row >= type_row0[t] && row < type_row0[t + 1]) sp = t;
  if (sp < 0) return;
  const T* w = (const T*)wo[sp];
  double acc = 0.0;
  bool real = row_atom[row] >= 0;
  for (int c = lane; c < N; c += 64) {
    if (real) acc += (double)X[(size_t)row * N + c] * (double)w[c];
    gseed[(size_t)row * N + c] = w[c];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) Ei[row] = real ? acc + bo[sp] : 0.0;
}

template <class T, int EPI>
static void gemm(int prec, const GemmArgs& G, hipStream_t st) {
  dim3 grid(((G.nrows + BM - 1) / BM) * ((G.N + BN - 1) / BN));
  if (prec == PREC_BF16) hipLaunchKernelGGL((k_gemm_bf<1, EPI>), grid, dim3(256), 0, st, G);
  else if (prec == PREC_BF16X3) hipLaunchKernelGGL((k_gemm_bf<2, EPI>), grid, dim3(256), 0, st, G);
  else hipLaunchKernelGGL((k_gemm<T, EPI>), grid, dim3(256), 0, st, G);
}

template <class T>
static void fit_t(const FitArgs& F, hipStream_t st) {
  const int prec = F.prec;
  const int rows = F.nrows, M = F.m.M, m2 = F.m.m2, K1 = M * m2, fw = F.fw;
  // BF16 modes: the 64-row-tile kernels (descriptor fused into the first layer, no D or dD
  // in HBM) whenever the shapes allow
  const bool bf = prec == PREC_BF16 || prec == PREC_BF16X3;
  if (bf && fit_bf_supported(M, m2, fw)) {
    launch_fit_bf(F, st);
    return;
  }
  size_t tot = (size_t)rows * K1;
  hipLaunchKernelGGL(k_desc<T>, dim3((tot + 255) / 256), dim3(256), 0, st, rows, M, m2, F.row_atom,
                     (const T*)F.T, (T*)F.D);
  T* act = (T*)F.act;
  T* xs = (T*)F.xs;
  size_t L = (size_t)rows * fw;
  GemmArgs G{};
  G.nrows = rows;
  G.type_row0 = F.type_row0;
  G.ntypes = F.m.ntypes;
  G.W = F.W;
  G.Wb = F.Wb;
  G.bias = F.b;
  G.wstride = F.nfit;
  for (int k = 0; k < F.nfit; k++) {
    G.K = k == 0 ? K1 : fw;
    G.N = fw;
    G.wsel = k;
    G.A = k == 0 ? F.D : (const void*)(xs + (k - 1) * L);
    G.Xprev = k == 0 ? nullptr : (const void*)(xs + (k - 1) * L);
    G.out = xs + k * L;
    G.out2 = act + k * L;
    if (k == 0) {
      gemm<T, EPI_FWD1>(prec, G, st);
    } else {
      gemm<T, EPI_FWDRES>(prec, G, st);
    }
  }
  hipLaunchKernelGGL(k_fit_out<T>, dim3((rows + 3) / 4), dim3(256), 0, st, rows, fw, F.m.ntypes,
                     F.type_row0, F.row_atom, (const T*)(xs + (F.nfit - 1) * L), F.wo, F.bo, F.Ei,
                     (T*)F.g0);
  T* gcur = (T*)F.g0;
  T* gnext = (T*)F.g1;
  for (int k = F.nfit - 1; k >= 1; k--) {
    G.K = fw;
    G.N = fw;
    G.wsel = k;
    G.A = gcur;
    G.Aaux = act + k * L;
    G.Xprev = gcur;
    G.out = gnext;
    gemm<T, EPI_BWD>(prec, G, st);
    T* tmp = gcur;
    gcur = gnext;
    gnext = tmp;
  }
  G.K = fw;
  G.N = K1;
  G.wsel = 0;
  G.A = gcur;
  G.Aaux = act;
  G.Xprev = nullptr;
  G.out = F.Dg;
  gemm<T, EPI_BWD1>(prec, G, st);
  hipLaunchKernelGGL(k_desc_bwd<T>, dim3(rows), dim3(256), sizeof(T) * (M * 4 + M * m2), st, rows, M, m2,
                     F.row_atom, (const T*)F.T, (const T*)F.Dg, (T*)F.gT);
}

void launch_fit(const FitArgs& F, hipStream_t st) {
  if (F.prec == PREC_FP64) fit_t<double>(F, st);
  else fit_t<float>(F, st);
}

// ------------------------------------------------------------------------------------
// reductions and small helpers
// ------------------------------------------------------------------------------------
__global__ void k_zero(size_t n, double* __restrict__ p) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}
void launch_zero(double* p, size_t n, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, n, p);
}

// Per frame, fixed-order sums of E_i and the per-centre virials in two launches: block
// (c, f) sums the atoms [c * kRedChunk, (c + 1) * kRedChunk) of frame f (one per thread;
// wave sums by butterfly shuffles, then the four waves in order) into partial row (f, c);
// then one block per frame adds the partial rows in chunk order, so the result does not
// depend on block scheduling.  (A last-block-finishes scheme would need a device-wide
// fence per block, which writes back the L2 of every XCD.)
constexpr int kRedChunk = 256;

// sum of acc over the block (every thread of wave 0 gets it), the waves added in order
__device__ __forceinline__ void block_sum10(double (&acc)[10], double (*sh)[10]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int q = 0; q < 10; q++) acc[q] += __shfl_xor(acc[q], o);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 10; q++) sh[wv][q] = acc[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 10; q++) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < kRedChunk / 64; w++) a += sh[w][q];
    acc[q] = a;
  }
}

__global__ __launch_bounds__(kRedChunk) void k_frame_reduce(const Frame* __restrict__ frames,
                                                            const int* __restrict__ row_of,
                                                            const double* __restrict__ Ei,
                                                            const double* __restrict__ vir,
                                                            double* __restrict__ atom_energy,
                                                            double* __restrict__ part) {
  __shared__ double sh[kRedChunk / 64][10];
  const int f = blockIdx.y, nchunk = gridDim.x;
  const Frame& F = frames[f];
  const int i = F.atom0 + blockIdx.x * kRedChunk + threadIdx.x;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; q++) acc[q] = 0.0;
  if (i < F.atom0 + F.natoms) {
    const int r = row_of[i];
    const double e = Ei[r];
    acc[0] = e;
    if (atom_energy) atom_energy[i] = e;
    if (vir)
#pragma unroll
      for (int q = 0; q < 9; q++) acc[1 + q] = vir[(size_t)r * 9 + q];
  }
  block_sum10(acc, sh);
  if (threadIdx.x < 10) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < 10; q++) a = q == (int)threadIdx.x ? acc[q] : a;
    part[((size_t)f * nchunk + blockIdx.x) * 10 + threadIdx.x] = a;
  }
}

// the partial rows of frame blockIdx.x in a fixed order: thread t adds rows t,
// t + kRedChunk, ..., then the block sum as above
__global__ __launch_bounds__(kRedChunk) void k_frame_reduce_rows(int nchunk, const double* __restrict__ part,
                                                                 double* __restrict__ energies,
                                                                 double* __restrict__ virials, int with_vir) {
  __shared__ double sh[kRedChunk / 64][10];
  const int f = blockIdx.x;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; q++) acc[q] = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += kRedChunk)
#pragma unroll
    for (int q = 0; q < 10; q++) acc[q] += part[((size_t)f * nchunk + c) * 10 + q];
  block_sum10(acc, sh);
  const int q = threadIdx.x;
  if (q < 10) {
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 10; k++) a = k == q ? acc[k] : a;
    if (q == 0) energies[f] = a;
    else if (virials && with_vir) virials[f * 9 + q - 1] = a;
  }
}

int frame_reduce_chunks(int max_frame_atoms) { return (max_frame_atoms + kRedChunk - 1) / kRedChunk; }

void launch_frame_reduce(int nframes, int max_frame_atoms, const Frame* frames, const int* row_of,
                         const double* Ei, const double* vir_rows, double* energies, double* virials,
                         double* atom_energy, double* part, hipStream_t st) {
  const int nchunk = frame_reduce_chunks(max_frame_atoms);
  hipLaunchKernelGGL(k_frame_reduce, dim3(nchunk, nframes), dim3(kRedChunk), 0, st, frames, row_of, Ei, vir_rows,
                     atom_energy, part);
  hipLaunchKernelGGL(k_frame_reduce_rows, dim3(nframes), dim3(kRedChunk), 0, st, nchunk, part, energies, virials,
                     vir_rows ? 1 : 0);
}

template <class T>
__global__ void k_export_T(int n, int M, const int* __restrict__ row_of, const T* __restrict__ Tm,
                           const T* __restrict__ gT, double* __restrict__ To, double* __restrict__ gTo) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * M * 4) return;
  int i = (int)(q / (M * 4));
  size_t src = (size_t)row_of[i] * M * 4 + q % (M * 4);
  if (To) To[q] = (double)Tm[src];
  if (gTo) gTo[q] = (double)gT[src];
}

void launch_export_T(int prec, int n, int M, const int* row_of, const void* Tm, const void* gT,
                     double* To, double* gTo, hipStream_t st) {
  size_t tot = (size_t)n * M * 4;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(k_export_T<double>, dim3((tot + 255) / 256), dim3(256), 0, st, n, M, row_of,
                       (const double*)Tm, (const double*)gT, To, gTo);
  else
    hipLaunchKernelGGL(k_export_T<float>, dim3((tot + 255) / 256), dim3(256), 0, st, n, M, row_of,
                       (const float*)Tm, (const float*)gT, To, gTo);
}

__global__ void k_export_atom_virial(int n, const int* __restrict__ row_of, const double* __restrict__ vir_rows,
                                     double* __restrict__ out) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * 9) return;
  const int i = (int)(q / 9);
  out[q] = vir_rows[(size_t)row_of[i] * 9 + q % 9];
}

void launch_export_atom_virial(int n, const int* row_of, const double* vir_rows, double* out, hipStream_t st) {
  const size_t tot = (size_t)n * 9;
  if (tot) hipLaunchKernelGGL(k_export_atom_virial, dim3((tot + 255) / 256), dim3(256), 0, st, n, row_of, vir_rows, out);
}

}  // namespace dp
