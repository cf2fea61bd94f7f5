// Parameter gradient of an energy + force loss (training path of the DP-SE model).
//
// Given per-frame weights gE and per-atom weights gF, computes
//   g_theta = sum_f gE_f dE_f/dtheta + d<gF, F>/dtheta,     F = -dE/dr  (Eq. 10)
// exactly, by forward-over-reverse differentiation: every quantity of the energy
// evaluation carries a tangent along the coordinate direction r -> r + eps gF
// (d_ij -> d_ij + eps (gF_j - gF_i)), and the reverse pass over the network is run
// with the per-atom seed dE_i = (1, -gE_f(i)) in (value, tangent) form.  The tangent
// of the resulting parameter adjoint equals d_gF dE/dtheta - sum_f gE_f dE_f/dtheta,
// so g_theta = -(tangent part).
//
// The embedding nets run in two fused passes (pgrad_fused.hip): the forward with
// tangents straight into T, and after the fitting net the reverse chain, which recomputes
// the activations and writes per neighbour row only the operands of the weight gradients
// (layer inputs and pre-activation adjoints with their tangents), so that those become
// products over the rows (dW = X^T P).  The fitting net is per centre (row-major
// activations, GEMMs).  All arithmetic is FP64.  GEMMs run on the FP64 16x16x4 MFMA;
// long reductions over rows are split across workgroups and summed with FP64 atomics.
#include <hip/hip_runtime.h>

#include "common.h"
#include "devmath.h"
#include "kernels.h"

namespace dp {

typedef double d4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// generic FP64 GEMM: C[M][N] += op(A) op(B), op(A) is M x K, op(B) is K x N.
//   TA = 0: A stored [M][lda]; TA = 1: A stored [K][lda] (A^T)
//   TB = 0: B stored [K][ldb]; TB = 1: B stored [N][ldb] (B^T)
// gridDim.z splits K; with more than one split the partial tiles are added atomically.
// With `mode` 2 the tile is stored (C = op(A) op(B): one split), with 1 added atomically.
// ------------------------------------------------------------------------------------
constexpr int PG_T = 64, PG_KT = 16, PG_LD = PG_T * PG_KT / 256;

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_pg_gemm(int M, int N, int K, int kchunk, const double* __restrict__ A,
                                                 int lda, const double* __restrict__ B, int ldb,
                                                 double* __restrict__ C, int ldc, int mode) {
  __shared__ double As[PG_T][PG_KT + 1];
  __shared__ double Bs[PG_KT][PG_T + 1];
  const int m0 = blockIdx.x * PG_T, n0 = blockIdx.y * PG_T;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, rb = lane & 15, g = lane >> 4;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  d4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = d4v{0, 0, 0, 0};
  double ra[PG_LD], rbv[PG_LD];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < PG_LD; j++) {
      int e = tid + 256 * j;
      int m, k;
      if (TA) { k = e / PG_T; m = e % PG_T; } else { m = e / PG_KT; k = e % PG_KT; }
      int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < M && gk < kend) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < PG_LD; j++) {
      int e = tid + 256 * j;
      int n, k;
      if (TB) { n = e / PG_KT; k = e % PG_KT; } else { k = e / PG_T; n = e % PG_T; }
      int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < N && gk < kend) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
      rbv[j] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int j = 0; j < PG_LD; j++) {
      int e = tid + 256 * j;
      if (TA) As[e % PG_T][e / PG_T] = ra[j];
      else As[e / PG_KT][e % PG_KT] = ra[j];
      if (TB) Bs[e % PG_KT][e / PG_KT] = rbv[j];
      else Bs[e / PG_T][e % PG_T] = rbv[j];
    }
  };
  if (kbeg < kend) {
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += PG_KT) {
      __syncthreads();
      store();
      __syncthreads();
      if (k0 + PG_KT < kend) load(k0 + PG_KT);
#pragma unroll
      for (int ks = 0; ks < PG_KT; ks += 4) {
        double a0 = As[wr + rb][ks + g], a1 = As[wr + 16 + rb][ks + g];
        double b0 = Bs[ks + g][wc + rb], b1 = Bs[ks + g][wc + 16 + rb];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      int col = n0 + wc + 16 * b + rb;
      if (col >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int row = m0 + wr + 16 * a + g + 4 * q;  // FP64 16x16x4: rows g + 4q
        if (row >= M) continue;
        double* c = C + (size_t)row * ldc + col;
        if (mode == 1) unsafeAtomicAdd(c, acc[a][b][q]);
        else if (mode == 2) *c = acc[a][b][q];
        else *c += acc[a][b][q];
      }
    }
}

// C += op(A) op(B); with `store`, C = op(A) op(B) (C need not be cleared first).
void pg_gemm(int ta, int tb, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
             double* C, int ldc, hipStream_t st, bool store = false) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  int gm = (M + PG_T - 1) / PG_T, gn = (N + PG_T - 1) / PG_T;
  // split long K so that the grid has enough workgroups
  int splits = 1;
  while (!store && (long)gm * gn * splits < 1024 && K / (splits * 2) >= 256) splits *= 2;
  int kchunk = ((K + splits - 1) / splits + PG_KT - 1) / PG_KT * PG_KT;
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid(gm, gn, splits);
  const int mode = store ? 2 : (splits > 1 ? 1 : 0);
  if (!ta && !tb) hipLaunchKernelGGL((k_pg_gemm<0, 0>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, mode);
  else if (!ta && tb) hipLaunchKernelGGL((k_pg_gemm<0, 1>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, mode);
  else if (ta && !tb) hipLaunchKernelGGL((k_pg_gemm<1, 0>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, mode);
  else hipLaunchKernelGGL((k_pg_gemm<1, 1>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, mode);
}

// ------------------------------------------------------------------------------------
// weight gradient of one embedding layer over the pair rows of one species pair:
//   C[m][n] += sum_r A[r][m] Bd[r][n] + Ad[r][m] B[r][n]
// A, Ad: [K][mA] (layer inputs and their tangents), B, Bd: [K][nB] (pre-activation
// adjoints and their tangents), C: [mA][nB], all row-major.  The FP64 16x16x4 MFMA takes
// its A operand as lane (i + 16k) <- A^T[i][k] and its B operand as lane (j + 16k) <-
// B[k][j]; with the pair rows as the contracted index both are loads of 16 consecutive
// columns from 4 consecutive rows, so the operands go from memory straight into the
// products with no staging.
// One workgroup per slice of rows (about one per CU).  Its waves are G tile groups x R row
// waves: wave (g, r) accumulates the MT x NT output tiles of group g (a layer wider than
// one group reads its rows once from memory, the other groups hit the cache) over the r-th
// part of the slice.  The R row waves of a group are then summed in LDS in a fixed order
// and the workgroup adds each entry of C once, atomically: few atomics per address, since
// FP64 atomics on one address serialise.  Two groups of U K-steps are kept in flight; the
// loads of whole groups carry no masks, so that nothing makes the compiler wait on them.
// ------------------------------------------------------------------------------------
template <int MT, int NT, int U, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_pg_wgrad(int K, int rows_per_block, int rows_per_wave, int mA, int nB,
                                                   int ngn, int G, const double* __restrict__ A,
                                                   const double* __restrict__ Ad, const double* __restrict__ B,
                                                   const double* __restrict__ Bd, double* __restrict__ C) {
  extern __shared__ double red[];  // [G][MT][NT][4][64]
  constexpr int kGroup = MT * NT * 4 * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, i = lane & 15, k = lane >> 4;
  const int g = w % G, rw = w / G, R = (blockDim.x >> 6) / G;
  const int b0 = blockIdx.x * rows_per_block, b1 = min(K, b0 + rows_per_block);
  const int r0 = b0 + rw * rows_per_wave, r1 = min(b1, r0 + rows_per_wave);
  const int m0 = (g / ngn) * 16 * MT, n0 = (g % ngn) * 16 * NT;
  // columns past a width read the last column: they only feed result entries past the
  // widths, which are never written
  int ca[MT], cb[NT];
#pragma unroll
  for (int t = 0; t < MT; t++) ca[t] = min(m0 + 16 * t + i, mA - 1);
#pragma unroll
  for (int t = 0; t < NT; t++) cb[t] = min(n0 + 16 * t + i, nB - 1);
  d4v acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; a++)
#pragma unroll
    for (int b = 0; b < NT; b++) acc[a][b] = d4v{0, 0, 0, 0};
  struct Buf {
    double a[U][MT], ad[U][MT], b[U][NT], bd[U][NT];
  };
  // rows r .. r + 4U - 1; with `tail`, rows past the wave's part read row r0 and their A
  // side is zeroed (then they add nothing)
  auto load = [&](Buf& f, int r, bool tail) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int row = r + 4 * u + k;
      const bool vr = !tail || row < r1;
      const size_t rr = vr ? row : r0;
      const double* pa = A + rr * mA;
      const double* pad = Ad + rr * mA;
      const double* pb = B + rr * nB;
      const double* pbd = Bd + rr * nB;
#pragma unroll
      for (int t = 0; t < MT; t++) {
        f.a[u][t] = pa[ca[t]];
        f.ad[u][t] = pad[ca[t]];
        if (tail) {
          f.a[u][t] = vr ? f.a[u][t] : 0.0;
          f.ad[u][t] = vr ? f.ad[u][t] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < NT; t++) {
        f.b[u][t] = pb[cb[t]];
        f.bd[u][t] = pbd[cb[t]];
      }
    }
  };
  auto mma = [&](const Buf& f) {
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int a = 0; a < MT; a++)
#pragma unroll
        for (int b = 0; b < NT; b++)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[u][a], f.bd[u][b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < MT; a++)
#pragma unroll
        for (int b = 0; b < NT; b++)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.ad[u][a], f.b[u][b], acc[a][b], 0, 0, 0);
    }
  };
  if (r0 < r1) {
    // whole groups of 4U rows, two in flight; then the partial group, if any
    const int nfull = (r1 - r0) / (4 * U);
    Buf f0, f1;
    if (nfull > 0) {
      load(f0, r0, false);
      int gi = 0;
      for (; gi + 2 <= nfull; gi += 2) {
        load(f1, r0 + (gi + 1) * 4 * U, false);
        mma(f0);
        if (gi + 2 < nfull) load(f0, r0 + (gi + 2) * 4 * U, false);
        mma(f1);
      }
      if (gi < nfull) mma(f0);
    }
    const int rt = r0 + nfull * 4 * U;
    if (rt < r1) {
      load(f1, rt, true);
      mma(f1);
    }
  }
  // fixed-order sum of the row waves of each group: round j adds row wave j's tiles
  double* mine = red + (size_t)g * kGroup;
  for (int j = 0; j < R; j++) {
    if (rw == j) {
#pragma unroll
      for (int a = 0; a < MT; a++)
#pragma unroll
        for (int b = 0; b < NT; b++)
#pragma unroll
          for (int q = 0; q < 4; q++) {
            double* p = mine + ((a * NT + b) * 4 + q) * 64 + lane;
            *p = (j == 0 ? 0.0 : *p) + acc[a][b][q];
          }
    }
    __syncthreads();
  }
  // one atomic per entry of C and workgroup; result lane (i + 16k) of a tile holds rows
  // k + 4q, column i
  for (int e = threadIdx.x; e < G * kGroup; e += blockDim.x) {
    const int gg = e / kGroup, t = e % kGroup, l = t & 63, q = (t >> 6) & 3, ab = t >> 8;
    const int row = (gg / ngn) * 16 * MT + 16 * (ab / NT) + (l >> 4) + 4 * q;
    const int col = (gg % ngn) * 16 * NT + 16 * (ab % NT) + (l & 15);
    if (row < mA && col < nB) unsafeAtomicAdd(C + (size_t)row * nB + col, red[e]);
  }
}

// R row waves per tile group: the waves of one workgroup fill a CU at the kernel's
// occupancy (WAVES per CU), so one workgroup per CU and kWgradSlices workgroups.
constexpr int kWgradSlices = 256;

template <int MT, int NT, int U, int WAVES>
static void pg_wgrad_launch(int K, int mA, int nB, const double* A, const double* Ad, const double* B,
                            const double* Bd, double* C, hipStream_t st) {
  const int mt = (mA + 15) / 16, nt = (nB + 15) / 16;
  const int ngm = (mt + MT - 1) / MT, ngn = (nt + NT - 1) / NT, G = ngm * ngn;
  const int R = std::max(1, WAVES / G);
  int rpw = (K + kWgradSlices * R - 1) / (kWgradSlices * R);
  rpw = (rpw + 4 * U - 1) / (4 * U) * (4 * U);
  const int rpb = rpw * R;
  const size_t lds = sizeof(double) * (size_t)G * MT * NT * 4 * 64;
  (void)hipFuncSetAttribute((const void*)k_pg_wgrad<MT, NT, U, WAVES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL((k_pg_wgrad<MT, NT, U, WAVES>), dim3((K + rpb - 1) / rpb), dim3(64 * G * R), lds, st, K, rpb, rpw, mA,
                     nB, ngn, G, A, Ad, B, Bd, C);
}

// C [mA][nB] += A^T Bd + Ad^T B over K pair rows (see k_pg_wgrad).  Narrow layers take one
// tile group; wider ones groups of 64 x 64 tiles, at most 2 x 2 of them (128 KB of LDS) for
// the widths the model loader admits (s0 <= 32: layer 2 is at most 65 x 128).
void pg_wgrad(int K, int mA, int nB, const double* A, const double* Ad, const double* B, const double* Bd,
              double* C, hipStream_t st) {
  if (K <= 0 || mA <= 0 || nB <= 0) return;
  const int mt = (mA + 15) / 16, nt = (nB + 15) / 16;
  if (mt <= 1 && nt <= 2) pg_wgrad_launch<1, 2, 2, 16>(K, mA, nB, A, Ad, B, Bd, C, st);
  else if (mt <= 2 && nt <= 4) pg_wgrad_launch<2, 4, 2, 8>(K, mA, nB, A, Ad, B, Bd, C, st);
  else if (mt <= 4 && nt == 7) pg_wgrad_launch<2, 7, 1, 8>(K, mA, nB, A, Ad, B, Bd, C, st);
  else pg_wgrad_launch<4, 4, 1, 8>(K, mA, nB, A, Ad, B, Bd, C, st);
}

// ------------------------------------------------------------------------------------
// elementwise pieces
// ------------------------------------------------------------------------------------
// y = skip(x) + tanh(z + b) with tangents; z, zd hold x W and dx W on entry and
// receive t and dt.  skip: 0 none, 1 identity, 2 concat (x, x).  xo/xod may be null.
__global__ void k_pg_act(size_t rows, int nin, int nout, int skip, const double* __restrict__ bias,
                         const double* __restrict__ x, const double* __restrict__ xd,
                         double* __restrict__ z, double* __restrict__ zd, double* __restrict__ xo,
                         double* __restrict__ xod) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * nout) return;
  size_t r = q / nout;
  int j = (int)(q % nout);
  double t = dp_tanh(z[q] + bias[j]);
  double td = (1.0 - t * t) * zd[q];
  z[q] = t;
  zd[q] = td;
  if (xo) {
    double sv = 0.0, sd = 0.0;
    if (skip == 1) { sv = x[r * nin + j]; sd = xd[r * nin + j]; }
    else if (skip == 2) { sv = x[r * nin + j % nin]; sd = xd[r * nin + j % nin]; }
    xo[q] = sv + t;
    xod[q] = sd + td;
  }
}

// D = T T<^T (flattened a m2 + b) and its tangent
__global__ void k_pg_desc(int nrows, int M, int m2, const double* __restrict__ T, const double* __restrict__ Td,
                          double* __restrict__ D, double* __restrict__ Dd) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)nrows * M * m2) return;
  size_t row = q / (M * m2);
  int ab = (int)(q % (M * m2)), a = ab / m2, b = ab % m2;
  const double* t = T + row * M * 4;
  const double* td = Td + row * M * 4;
  double v = 0.0, vd = 0.0;
  for (int c = 0; c < 4; c++) {
    v += t[a * 4 + c] * t[b * 4 + c];
    vd += td[a * 4 + c] * t[b * 4 + c] + t[a * 4 + c] * td[b * 4 + c];
  }
  D[q] = v;
  Dd[q] = vd;
}

// output layer seeds: ebar_i = (1, -gE_f(i)) for real centres; xbar = ebar w_o;
// grad_wo (tangent) += ebar_t x + ebar_v dx; grad_bo (tangent) += ebar_t
__global__ void k_pg_out(int rows_begin, int rows_end, int N, const int* __restrict__ row_atom,
                         const int* __restrict__ frame_of, const double* __restrict__ gE,
                         const double* __restrict__ wo, const double* __restrict__ x,
                         const double* __restrict__ xd, double* __restrict__ xb, double* __restrict__ xbd,
                         double* __restrict__ gwo, double* __restrict__ gbo) {
  int j = blockIdx.y * blockDim.x + threadIdx.x;  // column
  if (j >= N) return;
  double acc = 0.0, accb = 0.0;
  for (int row = rows_begin + blockIdx.x; row < rows_end; row += gridDim.x) {
    int atom = row_atom[row];
    double ev = 0.0, et = 0.0;
    if (atom >= 0) {
      ev = 1.0;
      et = -gE[frame_of[atom]];
    }
    size_t o = (size_t)row * N + j;
    xb[o] = ev * wo[j];
    xbd[o] = et * wo[j];
    acc += et * x[o] + ev * xd[o];
    if (j == 0) accb += et;
  }
  unsafeAtomicAdd(&gwo[j], acc);
  if (j == 0) unsafeAtomicAdd(gbo, accb);
}

// adjoint of y = skip(x) + tanh(z): the skip part of dE/dx (identity, or the two
// concat halves summed) from the undamped dE/dy, written to sk / skd [rows][nin]
__global__ void k_pg_skip(size_t rows, int nout, int nin, int skip, const double* __restrict__ xb,
                          const double* __restrict__ xbd, double* __restrict__ sk, double* __restrict__ skd) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * nin) return;
  size_t r = q / nin;
  int j = (int)(q % nin);
  if (skip == 1) {
    sk[q] = xb[r * nout + j];
    skd[q] = xbd[r * nout + j];
  } else {
    sk[q] = xb[r * nout + j] + xb[r * nout + j + nin];
    skd[q] = xbd[r * nout + j] + xbd[r * nout + j + nin];
  }
}

// P = dE/dy (1 - t^2), dP = d(dE/dy) (1 - t^2) - 2 dE/dy t dt, in place
__global__ void k_pg_damp(size_t n, double* __restrict__ xb, double* __restrict__ xbd,
                          const double* __restrict__ t, const double* __restrict__ td) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double v = xb[q], vd = xbd[q], tt = t[q], ttd = td[q];
  double u = 1.0 - tt * tt;
  xb[q] = v * u;
  xbd[q] = vd * u - 2.0 * v * tt * ttd;
}

// column sums: out[j] += sum_r (a[r][j] * (wa ? wa[r*ws] : 1) + b[r][j] * (wb ? wb[r*ws] : 1))
// (b may be null).  Used for bias gradients and the first embedding layer's weights.
// Block (x, y) takes columns 64 y .. 64 y + 63 and a contiguous range of per_block rows;
// its four waves take every fourth row of the range with four independent partial sums
// each, then add in wave order; one atomic per column and block.
__global__ __launch_bounds__(256) void k_pg_colsum(size_t rows, size_t per_block, int N, const double* __restrict__ a,
                                                   const double* __restrict__ wa, const double* __restrict__ b,
                                                   const double* __restrict__ wb, int ws, double* __restrict__ out) {
  __shared__ double sh[4][64];
  const int c = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.y * 64 + c;
  const size_t r0 = (size_t)blockIdx.x * per_block, r1 = r0 + per_block < rows ? r0 + per_block : rows;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < N) {
    size_t r = r0 + wv;
    for (; r + 12 < r1; r += 16) {
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const size_t q = r + 4 * u;
        double v = a[q * N + j] * (wa ? wa[q * ws] : 1.0);
        if (b) v += b[q * N + j] * (wb ? wb[q * ws] : 1.0);
        acc[u] += v;
      }
    }
    for (; r < r1; r += 4) {
      double v = a[r * N + j] * (wa ? wa[r * ws] : 1.0);
      if (b) v += b[r * N + j] * (wb ? wb[r * ws] : 1.0);
      acc[0] += v;
    }
  }
  sh[wv][c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wv == 0 && j < N) unsafeAtomicAdd(&out[j], ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c]);
}

static void pg_colsum(size_t rows, int N, const double* a, const double* wa, const double* b,
                      const double* wb, int ws, double* out, hipStream_t st) {
  if (!rows || !N) return;
  const int by = (N + 63) / 64;
  // about 1024 blocks in all (a few rows each for short sums), rows in multiples of 16
  size_t per = (rows * by + 1023) / 1024;
  per = per < 16 ? 16 : (per + 15) / 16 * 16;
  const int bx = (int)((rows + per - 1) / per);
  hipLaunchKernelGGL(k_pg_colsum, dim3(bx, by), dim3(256), 0, st, rows, per, N, a, wa, b, wb, ws, out);
}

// dT from dD (Eq. 4 adjoint) with tangents, one block per centre row; the row's dD, its
// tangent, T and its tangent are staged in LDS first (coalesced), the strided reads of the
// second term then come from there
__global__ __launch_bounds__(256) void k_pg_desc_bwd(int M, int m2, const double* __restrict__ T,
                                                     const double* __restrict__ Td,
                                                     const double* __restrict__ Dg,
                                                     const double* __restrict__ Dgd,
                                                     double* __restrict__ gT, double* __restrict__ gTd) {
  extern __shared__ double sm[];
  const int K1 = M * m2;
  double* sdg = sm;           // [M][m2]
  double* sdgd = sdg + K1;
  double* st = sdgd + K1;     // [M][4]
  double* std4 = st + M * 4;
  const size_t row = blockIdx.x;
  for (int q = threadIdx.x; q < K1; q += blockDim.x) {
    sdg[q] = Dg[row * K1 + q];
    sdgd[q] = Dgd[row * K1 + q];
  }
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) {
    st[q] = T[row * M * 4 + q];
    std4[q] = Td[row * M * 4 + q];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) {
    int p = q >> 2, c = q & 3;
    double v = 0.0, vd = 0.0;
    for (int b = 0; b < m2; b++) {
      v += sdg[p * m2 + b] * st[b * 4 + c];
      vd += sdgd[p * m2 + b] * st[b * 4 + c] + sdg[p * m2 + b] * std4[b * 4 + c];
    }
    if (p < m2)
      for (int a = 0; a < M; a++) {
        v += sdg[a * m2 + p] * st[a * 4 + c];
        vd += sdgd[a * m2 + p] * st[a * 4 + c] + sdg[a * m2 + p] * std4[a * 4 + c];
      }
    gT[row * M * 4 + q] = v;
    gTd[row * M * 4 + q] = vd;
  }
}

// ------------------------------------------------------------------------------------
// orchestration
// ------------------------------------------------------------------------------------
static size_t pgal(size_t x) { return (x + 255) & ~(size_t)255; }

size_t param_grad_scratch_bytes(int nrows, long np_max, int M, int m2, int s0, int fw, int nfit) {
  int s1 = 2 * s0;
  // per pair: X0, X0d (s0 + 1), P0, P0d (s0), X1, X1d (s1 + 1), P1, P1d (s1), P2, P2d (M),
  // S, Sd (2)
  size_t per_pair = 4 * (size_t)s0 + 4 * (size_t)s1 + 2 * (size_t)M + 8;
  size_t per_row = 8 * M + 4 * M * m2 + (size_t)nfit * 6 * fw + 4 * fw;
  return 12 * pgal(0) + pgal(sizeof(double) * per_pair * np_max) + 12 * 256 +
         pgal(sizeof(double) * per_row * nrows) + 65536;
}

int launch_param_grad(const PGradArgs& G, hipStream_t st) {
  const ModelC& m = G.m;
  const int nt = m.ntypes, M = m.M, m2 = m.m2, s0 = m.s0, s1 = 2 * s0, K1 = M * m2, fw = G.fw;
  const int nrows = G.nrows, np = G.np;
  const double* th = G.theta;
  double* gt = G.gtheta_tan;
  char* w = (char*)G.scratch;
  auto take = [&](size_t bytes) { char* p = w; w += pgal(bytes); return p; };
  PgfArgs F{};
  F.m = m;
  F.nrows = nrows;
  F.type_row0 = G.type_row0;
  F.row_atom = G.row_atom;
  F.nnei = G.nnei;
  F.nlist = G.nlist;
  F.eown = G.eown;
  F.xe = G.xe;
  F.vdir = G.vdir;
  F.nets = G.nets;
  for (int b = 0; b < kMaxTypes; b++) {
    F.base[b] = G.base[b];
    F.boff[b] = G.boff[b];
  }
  F.X0 = (double*)take(sizeof(double) * (s0 + 1) * (size_t)np);
  F.X0d = (double*)take(sizeof(double) * (s0 + 1) * (size_t)np);
  F.P0 = (double*)take(sizeof(double) * s0 * (size_t)np);
  F.P0d = (double*)take(sizeof(double) * s0 * (size_t)np);
  F.X1 = (double*)take(sizeof(double) * (s1 + 1) * (size_t)np);
  F.X1d = (double*)take(sizeof(double) * (s1 + 1) * (size_t)np);
  F.P1 = (double*)take(sizeof(double) * s1 * (size_t)np);
  F.P1d = (double*)take(sizeof(double) * s1 * (size_t)np);
  F.P2 = (double*)take(sizeof(double) * M * (size_t)np);
  F.P2d = (double*)take(sizeof(double) * M * (size_t)np);
  F.S = (double*)take(sizeof(double) * 2 * (size_t)np);
  F.Sd = (double*)take(sizeof(double) * 2 * (size_t)np);
  size_t rs = nrows;
  double* Tm = (double*)take(sizeof(double) * rs * M * 4);
  double* Tmd = (double*)take(sizeof(double) * rs * M * 4);
  double* gTm = (double*)take(sizeof(double) * rs * M * 4);
  double* gTmd = (double*)take(sizeof(double) * rs * M * 4);
  double* D = (double*)take(sizeof(double) * rs * K1);
  double* Dd = (double*)take(sizeof(double) * rs * K1);
  double* Dg = (double*)take(sizeof(double) * rs * K1);
  double* Dgd = (double*)take(sizeof(double) * rs * K1);
  double* ft = (double*)take(sizeof(double) * rs * fw * G.nfit);   // tanh parts
  double* ftd = (double*)take(sizeof(double) * rs * fw * G.nfit);
  double* fx = (double*)take(sizeof(double) * rs * fw * G.nfit);   // layer outputs
  double* fxd = (double*)take(sizeof(double) * rs * fw * G.nfit);
  double* xb = (double*)take(sizeof(double) * rs * fw);
  double* xbd = (double*)take(sizeof(double) * rs * fw);
  double* xb2 = (double*)take(sizeof(double) * rs * fw);
  double* xb2d = (double*)take(sizeof(double) * rs * fw);
  if ((size_t)(w - (char*)G.scratch) > G.scratch_bytes) return -1;

  // 1-3. T and its tangent per centre (fused embedding forward), then D = T T<^T
  F.Tm = Tm;
  F.Tmd = Tmd;
  launch_pgf_fwd(F, st);
  hipLaunchKernelGGL(k_pg_desc, dim3(((size_t)nrows * K1 + 255) / 256), dim3(256), 0, st, nrows, M, m2, Tm, Tmd, D, Dd);
  // 4. fitting net per species: forward with tangents, reverse with dual seeds
  const int nf = G.nfit;
  for (int a = 0; a < nt; a++) {
    int r0 = G.type_row0_h[a], r1 = G.type_row0_h[a + 1], nr = r1 - r0;
    if (nr <= 0) continue;
    size_t L = (size_t)rs * fw;
    for (int k = 0; k < nf; k++) {
      const double* Wk = th + G.fW[a * (nf + 1) + k];
      const double* bk = th + G.fB[a * (nf + 1) + k];
      int kin = k == 0 ? K1 : fw;
      const double* xin = k == 0 ? D + (size_t)r0 * K1 : fx + (k - 1) * L + (size_t)r0 * fw;
      const double* xind = k == 0 ? Dd + (size_t)r0 * K1 : fxd + (k - 1) * L + (size_t)r0 * fw;
      double* tk = ft + k * L + (size_t)r0 * fw;
      double* tkd = ftd + k * L + (size_t)r0 * fw;
      pg_gemm(0, 0, nr, fw, kin, xin, kin, Wk, fw, tk, fw, st, true);
      pg_gemm(0, 0, nr, fw, kin, xind, kin, Wk, fw, tkd, fw, st, true);
      int skip = (kin == fw) ? 1 : 0;
      hipLaunchKernelGGL(k_pg_act, dim3(((size_t)nr * fw + 255) / 256), dim3(256), 0, st, (size_t)nr, kin, fw, skip, bk,
                         xin, xind, tk, tkd, fx + k * L + (size_t)r0 * fw, fxd + k * L + (size_t)r0 * fw);
    }
    // output layer and seeds
    const double* wo = th + G.fW[a * (nf + 1) + nf];
    double* gwo = gt + G.fW[a * (nf + 1) + nf];
    double* gbo = gt + G.fB[a * (nf + 1) + nf];
    {
      dim3 grid(std::min(nr, 512), (fw + 63) / 64);
      hipLaunchKernelGGL(k_pg_out, grid, dim3(64), 0, st, r0, r1, fw, G.row_atom, G.frame_of, G.gE, wo,
                         fx + (nf - 1) * L, fxd + (nf - 1) * L, xb, xbd, gwo, gbo);
    }
    // hidden layers, last to first; xb holds dE/dx_k (rows r0..r1, stored from row 0 of xb)
    double* cur = xb;
    double* curd = xbd;
    double* nxt = xb2;
    double* nxtd = xb2d;
    // xb was written at absolute rows by k_pg_out: use absolute offsets
    for (int k = nf - 1; k >= 0; k--) {
      const double* Wk = th + G.fW[a * (nf + 1) + k];
      double* gWk = gt + G.fW[a * (nf + 1) + k];
      double* gbk = gt + G.fB[a * (nf + 1) + k];
      int kin = k == 0 ? K1 : fw;
      double* c = cur + (size_t)r0 * fw;
      double* cd = curd + (size_t)r0 * fw;
      double* tk = ft + k * L + (size_t)r0 * fw;
      double* tkd = ftd + k * L + (size_t)r0 * fw;
      const double* xin = k == 0 ? D + (size_t)r0 * K1 : fx + (k - 1) * L + (size_t)r0 * fw;
      const double* xind = k == 0 ? Dd + (size_t)r0 * K1 : fxd + (k - 1) * L + (size_t)r0 * fw;
      double* dst = k == 0 ? Dg + (size_t)r0 * K1 : nxt + (size_t)r0 * fw;
      double* dstd = k == 0 ? Dgd + (size_t)r0 * K1 : nxtd + (size_t)r0 * fw;
      int skip = (kin == fw) ? 1 : 0;
      if (skip) {
        hipLaunchKernelGGL(k_pg_skip, dim3(((size_t)nr * kin + 255) / 256), dim3(256), 0, st, (size_t)nr, fw, kin, 1,
                           c, cd, dst, dstd);
      }
      hipLaunchKernelGGL(k_pg_damp, dim3(((size_t)nr * fw + 255) / 256), dim3(256), 0, st, (size_t)nr * fw, c, cd, tk, tkd);
      // weight gradient (tangent): x^T dP + dx^T P; bias: sum dP
      pg_gemm(1, 0, kin, fw, nr, xin, kin, cd, fw, gWk, fw, st);
      pg_gemm(1, 0, kin, fw, nr, xind, kin, c, fw, gWk, fw, st);
      pg_colsum((size_t)nr, fw, cd, nullptr, nullptr, nullptr, 0, gbk, st);
      // input adjoint += P W^T (value and tangent; stored where there is no skip term)
      pg_gemm(0, 1, nr, kin, fw, c, fw, Wk, fw, dst, kin, st, !skip);
      pg_gemm(0, 1, nr, kin, fw, cd, fw, Wk, fw, dstd, kin, st, !skip);
      double* t1 = cur; cur = nxt; nxt = t1;
      double* t2 = curd; curd = nxtd; nxtd = t2;
    }
  }
  // 5. dE/dT with tangents
  {
    const size_t sh = sizeof(double) * (2 * (size_t)K1 + 8 * (size_t)M);
    (void)hipFuncSetAttribute((const void*)k_pg_desc_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL(k_pg_desc_bwd, dim3(nrows), dim3(256), sh, st, M, m2, Tm, Tmd, Dg, Dgd, gTm, gTmd);
  }
  // 6. embedding reverse (fused: the per-pair operands of the weight gradients), then the
  // weight gradients as products over the pair rows of each species pair
  F.gTm = gTm;
  F.gTmd = gTmd;
  launch_pgf_bwd(F, st);
  for (int a = 0; a < nt; a++)
    for (int b = 0; b < nt; b++) {
      int g0 = G.group[(a * nt + b) * 2], ng = G.group[(a * nt + b) * 2 + 1];
      if (ng <= 0) continue;
      int net = a * nt + b;
      // (theta keeps each embedding layer's bias right after its weights: eB = eW + n_in n_out)
      double* gW0 = gt + G.eW[net * 3 + 0];
      double* gW1 = gt + G.eW[net * 3 + 1];
      double* gW2 = gt + G.eW[net * 3 + 2];
      size_t o0 = (size_t)g0 * s0, o1 = (size_t)g0 * s1, o2 = (size_t)g0 * M;
      // the biases follow the weights in theta: the trailing column of the inputs (ones in
      // the value, zeros in the tangent) turns row n_in of each product into the bias sum
      // layer 2: [gW2; gB2] += [X1 1]^T dP2 + [dX1 0]^T P2
      pg_wgrad(ng, s1 + 1, M, F.X1 + (size_t)g0 * (s1 + 1), F.X1d + (size_t)g0 * (s1 + 1), F.P2 + o2, F.P2d + o2,
               gW2, st);
      // layer 1: [gW1; gB1] += [X0 1]^T dP1 + [dX0 0]^T P1
      pg_wgrad(ng, s0 + 1, s1, F.X0 + (size_t)g0 * (s0 + 1), F.X0d + (size_t)g0 * (s0 + 1), F.P1 + o1, F.P1d + o1,
               gW1, st);
      // layer 0: [gW0; gB0] += [s 1]^T dP0 + [ds 0]^T P0
      pg_wgrad(ng, 2, s0, F.S + 2 * (size_t)g0, F.Sd + 2 * (size_t)g0, F.P0 + o0, F.P0d + o0, gW0, st);
    }
  return 0;
}

}  // namespace dp
