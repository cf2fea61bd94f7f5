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
// Unlike the force path, this path stores the per-neighbour activations of the
// embedding nets (grouped by species pair) so that the weight gradients become GEMMs
// over the neighbour rows (dW = X^T P).  All arithmetic is FP64.  GEMMs run on the
// FP64 16x16x4 MFMA; long reductions over rows are split across workgroups and summed
// with FP64 atomics.
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
// ------------------------------------------------------------------------------------
constexpr int PG_T = 64, PG_KT = 16;

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_pg_gemm(int M, int N, int K, int kchunk, const double* __restrict__ A,
                                                 int lda, const double* __restrict__ B, int ldb,
                                                 double* __restrict__ C, int ldc, int atomic) {
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
  double ra[4], rbv[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int e = tid + 256 * j;
      int m, k;
      if (TA) { k = e / PG_T; m = e % PG_T; } else { m = e / PG_KT; k = e % PG_KT; }
      int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < M && gk < kend) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
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
    for (int j = 0; j < 4; j++) {
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
        if (atomic) unsafeAtomicAdd(c, acc[a][b][q]);
        else *c += acc[a][b][q];
      }
    }
}

void pg_gemm(int ta, int tb, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
             double* C, int ldc, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  int gm = (M + PG_T - 1) / PG_T, gn = (N + PG_T - 1) / PG_T;
  // split long K so that the grid has enough workgroups
  int splits = 1;
  while ((long)gm * gn * splits < 1024 && K / (splits * 2) >= 256) splits *= 2;
  int kchunk = ((K + splits - 1) / splits + PG_KT - 1) / PG_KT * PG_KT;
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid(gm, gn, splits);
  int atomic = splits > 1;
  if (!ta && !tb) hipLaunchKernelGGL((k_pg_gemm<0, 0>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, atomic);
  else if (!ta && tb) hipLaunchKernelGGL((k_pg_gemm<0, 1>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, atomic);
  else if (ta && !tb) hipLaunchKernelGGL((k_pg_gemm<1, 0>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, atomic);
  else hipLaunchKernelGGL((k_pg_gemm<1, 1>), grid, dim3(256), 0, st, M, N, K, kchunk, A, lda, B, ldb, C, ldc, atomic);
}

// ------------------------------------------------------------------------------------
// elementwise pieces
// ------------------------------------------------------------------------------------
__global__ void k_pg_zero(size_t n, double* __restrict__ p) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}
static void pg_zero(double* p, size_t n, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_pg_zero, dim3((n + 255) / 256), dim3(256), 0, st, n, p);
}

// pair rows of each centre: for species block beta, rows [base[row], base[row] + nnei)
__global__ void k_pg_pairs(int nrows, int ntypes, int nm, int beta, int sel_off,
                           const int* __restrict__ row_atom, const int* __restrict__ nnei,
                           const int* __restrict__ nlist, const int* __restrict__ base, int off,
                           int* __restrict__ p_row, int* __restrict__ p_e) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  int atom = row_atom[row];
  if (atom < 0) return;
  int nn = nnei[atom * ntypes + beta];
  int b = off + base[row];
  for (int k = 0; k < nn; k++) {
    p_row[b + k] = row;
    p_e[b + k] = nlist[(size_t)atom * nm + sel_off + k];
  }
}

// environment rows with tangents: R, dR = (dR/dd) (v_j - v_i); S = R[0]
__global__ void k_pg_env(int np, ModelC m, const int* __restrict__ p_row, const int* __restrict__ p_e,
                         const int* __restrict__ row_atom, const int* __restrict__ eown,
                         const double* __restrict__ xe, const double* __restrict__ vdir,
                         double* __restrict__ R, double* __restrict__ Rd) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  int i = row_atom[p_row[p]], e = p_e[p];
  double d[3], dd[3];
  int own = eown[e];
  for (int c = 0; c < 3; c++) {
    d[c] = xe[3 * e + c] - xe[3 * i + c];
    dd[c] = vdir[3 * own + c] - vdir[3 * i + c];
  }
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double s, ds;
  smooth_fn(m, r, s, ds);
  double ir = 1.0 / r, sr = s * ir;
  double dot = (d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2]) * ir;  // dr along the tangent
  double qf = (ds * ir - s * ir * ir);                               // d(s/r)/dr
  R[4 * p] = s;
  Rd[4 * p] = ds * dot;
  for (int c = 0; c < 3; c++) {
    R[4 * p + 1 + c] = sr * d[c];
    Rd[4 * p + 1 + c] = qf * dot * d[c] + sr * dd[c];
  }
}

// first embedding layer: X0 = tanh(s W0 + b0), dX0 = (1 - X0^2) ds W0
__global__ void k_pg_l0(int np, int s0, const double* __restrict__ R, const double* __restrict__ Rd,
                        const double* __restrict__ W0, const double* __restrict__ b0,
                        double* __restrict__ X0, double* __restrict__ X0d) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)np * s0) return;
  size_t p = q / s0;
  int j = (int)(q % s0);
  double s = R[4 * p], sd = Rd[4 * p];
  double t = dp_tanh(s * W0[j] + b0[j]);
  X0[q] = t;
  X0d[q] = (1.0 - t * t) * sd * W0[j];
}

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

// T = sum over a centre's pair rows of G R / N_m (and tangent), G = (X1, X1) + T2
__global__ __launch_bounds__(256) void k_pg_contract(int nrows, int ntypes, int M, double inv_norm,
                                                     const int* __restrict__ row_atom,
                                                     const int* __restrict__ nnei,
                                                     const int* const* __restrict__ base,
                                                     const int* __restrict__ boff,
                                                     const double* __restrict__ X1,
                                                     const double* __restrict__ X1d,
                                                     const double* __restrict__ T2,
                                                     const double* __restrict__ T2d,
                                                     const double* __restrict__ R,
                                                     const double* __restrict__ Rd,
                                                     double* __restrict__ T, double* __restrict__ Td) {
  const int row = blockIdx.x;
  const int atom = row_atom[row];
  const int s1 = M / 2;
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) {
    int a = q >> 2, c = q & 3;
    double v = 0.0, vd = 0.0;
    if (atom >= 0)
      for (int beta = 0; beta < ntypes; beta++) {
        int nn = nnei[atom * ntypes + beta];
        size_t p0 = (size_t)boff[beta] + base[beta][row];
        for (int k = 0; k < nn; k++) {
          size_t p = p0 + k;
          double G = X1[p * s1 + a % s1] + T2[p * M + a];
          double Gd = X1d[p * s1 + a % s1] + T2d[p * M + a];
          v += G * R[4 * p + c];
          vd += Gd * R[4 * p + c] + G * Rd[4 * p + c];
        }
      }
    T[(size_t)row * M * 4 + q] = v * inv_norm;
    Td[(size_t)row * M * 4 + q] = vd * inv_norm;
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
__global__ void k_pg_colsum(size_t rows, int N, const double* __restrict__ a, const double* __restrict__ wa,
                            const double* __restrict__ b, const double* __restrict__ wb, int ws,
                            double* __restrict__ out) {
  int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double acc = 0.0;
  for (size_t r = blockIdx.x; r < rows; r += gridDim.x) {
    double v = a[r * N + j] * (wa ? wa[r * ws] : 1.0);
    if (b) v += b[r * N + j] * (wb ? wb[r * ws] : 1.0);
    acc += v;
  }
  unsafeAtomicAdd(&out[j], acc);
}

static void pg_colsum(size_t rows, int N, const double* a, const double* wa, const double* b,
                      const double* wb, int ws, double* out, hipStream_t st) {
  if (!rows || !N) return;
  int by = (N + 63) / 64;
  int bx = (int)std::min<size_t>(rows, 1024);
  hipLaunchKernelGGL(k_pg_colsum, dim3(bx, by), dim3(64), 0, st, rows, N, a, wa, b, wb, ws, out);
}

// dT from dD (Eq. 4 adjoint) with tangents, one block per centre row
__global__ __launch_bounds__(256) void k_pg_desc_bwd(int M, int m2, const double* __restrict__ T,
                                                     const double* __restrict__ Td,
                                                     const double* __restrict__ Dg,
                                                     const double* __restrict__ Dgd,
                                                     double* __restrict__ gT, double* __restrict__ gTd) {
  const size_t row = blockIdx.x;
  const double* t = T + row * M * 4;
  const double* td = Td + row * M * 4;
  const double* dg = Dg + row * M * m2;
  const double* dgd = Dgd + row * M * m2;
  for (int q = threadIdx.x; q < M * 4; q += blockDim.x) {
    int p = q >> 2, c = q & 3;
    double v = 0.0, vd = 0.0;
    for (int b = 0; b < m2; b++) {
      v += dg[p * m2 + b] * t[b * 4 + c];
      vd += dgd[p * m2 + b] * t[b * 4 + c] + dg[p * m2 + b] * td[b * 4 + c];
    }
    if (p < m2)
      for (int a = 0; a < M; a++) {
        v += dg[a * m2 + p] * t[a * 4 + c];
        vd += dgd[a * m2 + p] * t[a * 4 + c] + dg[a * m2 + p] * td[a * 4 + c];
      }
    gT[row * M * 4 + q] = v;
    gTd[row * M * 4 + q] = vd;
  }
}

// per pair row: dE/dG = dT R / N_m (with tangent); writes the concat-skip part of
// dE/dX1 (G = (X1, X1) + T2) and P2 = dE/dG (1 - T2^2) with its tangent
__global__ void k_pg_gbar(size_t np, int M, double inv_norm, const int* __restrict__ p_row,
                          const double* __restrict__ gT, const double* __restrict__ gTd,
                          const double* __restrict__ R, const double* __restrict__ Rd,
                          const double* __restrict__ T2, const double* __restrict__ T2d,
                          double* __restrict__ P2, double* __restrict__ P2d, double* __restrict__ X1b,
                          double* __restrict__ X1bd) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int s1 = M / 2;
  if (q >= np * s1) return;
  size_t p = q / s1;
  int a = (int)(q % s1);
  size_t row = p_row[p];
  const double* r = R + 4 * p;
  const double* rd = Rd + 4 * p;
  double sk = 0.0, skd = 0.0;
  for (int h = 0; h < 2; h++) {
    int f = a + h * s1;
    const double* g = gT + row * M * 4 + f * 4;
    const double* gd = gTd + row * M * 4 + f * 4;
    double v = 0.0, vd = 0.0;
    for (int c = 0; c < 4; c++) {
      v += g[c] * r[c];
      vd += gd[c] * r[c] + g[c] * rd[c];
    }
    v *= inv_norm;
    vd *= inv_norm;
    sk += v;
    skd += vd;
    double t = T2[p * M + f], td = T2d[p * M + f];
    double u = 1.0 - t * t;
    P2[p * M + f] = v * u;
    P2d[p * M + f] = vd * u - 2.0 * v * t * td;
  }
  X1b[p * s1 + a] = sk;
  X1bd[p * s1 + a] = skd;
}

// first-layer weight gradient (tangent): gW0[j] += sum_r (S dP0 + dS P0); S = R[0]
// handled by k_pg_colsum with weights taken from R (stride 4)

// ------------------------------------------------------------------------------------
// orchestration
// ------------------------------------------------------------------------------------
static size_t pgal(size_t x) { return (x + 255) & ~(size_t)255; }

size_t param_grad_scratch_bytes(int nrows, long np_max, int M, int m2, int s0, int fw, int nfit) {
  int s1 = 2 * s0;
  size_t per_pair = 8 + 8 + 2 * s0 + 2 * s0 + 2 * s1 + 2 * s1 + 2 * M + 2 * M + 2 * s1 + 2 * s0;
  size_t per_row = 8 * M + 4 * M * m2 + (size_t)nfit * 6 * fw + 4 * fw + 8 * M;
  return pgal(sizeof(int) * 2 * np_max) + pgal(sizeof(double) * per_pair * np_max) +
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
  int* p_row = (int*)take(sizeof(int) * np);
  int* p_e = (int*)take(sizeof(int) * np);
  double* R = (double*)take(sizeof(double) * 4 * np);
  double* Rd = (double*)take(sizeof(double) * 4 * np);
  double* X0 = (double*)take(sizeof(double) * s0 * np);
  double* X0d = (double*)take(sizeof(double) * s0 * np);
  double* T1 = (double*)take(sizeof(double) * s1 * np);
  double* T1d = (double*)take(sizeof(double) * s1 * np);
  double* X1 = (double*)take(sizeof(double) * s1 * np);
  double* X1d = (double*)take(sizeof(double) * s1 * np);
  double* T2 = (double*)take(sizeof(double) * M * np);
  double* T2d = (double*)take(sizeof(double) * M * np);
  double* P2 = (double*)take(sizeof(double) * M * np);
  double* P2d = (double*)take(sizeof(double) * M * np);
  double* X1b = (double*)take(sizeof(double) * s1 * np);
  double* X1bd = (double*)take(sizeof(double) * s1 * np);
  double* X0b = (double*)take(sizeof(double) * s0 * np);
  double* X0bd = (double*)take(sizeof(double) * s0 * np);
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

  // 1. pair rows, grouped by neighbour species beta, then by centre species (row order)
  for (int beta = 0; beta < nt; beta++)
    hipLaunchKernelGGL(k_pg_pairs, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, nt, m.nm, beta,
                       m.sel_off[beta], G.row_atom, G.nnei, G.nlist, G.base[beta], G.boff[beta], p_row, p_e);
  hipLaunchKernelGGL(k_pg_env, dim3((np + 255) / 256), dim3(256), 0, st, np, m, p_row, p_e, G.row_atom,
                     G.eown, G.xe, G.vdir, R, Rd);
  // 2. embedding forward with tangents, per species pair group
  for (int a = 0; a < nt; a++)
    for (int b = 0; b < nt; b++) {
      int g0 = G.group[(a * nt + b) * 2], ng = G.group[(a * nt + b) * 2 + 1];
      if (ng <= 0) continue;
      const double* W0 = th + G.eW[(a * nt + b) * 3 + 0];
      const double* B0 = th + G.eB[(a * nt + b) * 3 + 0];
      const double* W1 = th + G.eW[(a * nt + b) * 3 + 1];
      const double* B1 = th + G.eB[(a * nt + b) * 3 + 1];
      const double* W2 = th + G.eW[(a * nt + b) * 3 + 2];
      const double* B2 = th + G.eB[(a * nt + b) * 3 + 2];
      size_t o0 = (size_t)g0 * s0, o1 = (size_t)g0 * s1, o2 = (size_t)g0 * M;
      hipLaunchKernelGGL(k_pg_l0, dim3(((size_t)ng * s0 + 255) / 256), dim3(256), 0, st, ng, s0, R + 4 * (size_t)g0,
                         Rd + 4 * (size_t)g0, W0, B0, X0 + o0, X0d + o0);
      pg_zero(T1 + o1, (size_t)ng * s1, st);
      pg_zero(T1d + o1, (size_t)ng * s1, st);
      pg_gemm(0, 0, ng, s1, s0, X0 + o0, s0, W1, s1, T1 + o1, s1, st);
      pg_gemm(0, 0, ng, s1, s0, X0d + o0, s0, W1, s1, T1d + o1, s1, st);
      hipLaunchKernelGGL(k_pg_act, dim3(((size_t)ng * s1 + 255) / 256), dim3(256), 0, st, (size_t)ng, s0, s1, 2, B1,
                         X0 + o0, X0d + o0, T1 + o1, T1d + o1, X1 + o1, X1d + o1);
      pg_zero(T2 + o2, (size_t)ng * M, st);
      pg_zero(T2d + o2, (size_t)ng * M, st);
      pg_gemm(0, 0, ng, M, s1, X1 + o1, s1, W2, M, T2 + o2, M, st);
      pg_gemm(0, 0, ng, M, s1, X1d + o1, s1, W2, M, T2d + o2, M, st);
      hipLaunchKernelGGL(k_pg_act, dim3(((size_t)ng * M + 255) / 256), dim3(256), 0, st, (size_t)ng, s1, M, 2, B2,
                         (const double*)nullptr, (const double*)nullptr, T2 + o2, T2d + o2, (double*)nullptr,
                         (double*)nullptr);
    }
  // 3. contraction and descriptor (with tangents)
  hipLaunchKernelGGL(k_pg_contract, dim3(nrows), dim3(256), 0, st, nrows, nt, M, m.inv_norm, G.row_atom, G.nnei,
                     G.base_dev, G.boff_dev, X1, X1d, T2, T2d, R, Rd, Tm, Tmd);
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
      pg_zero(tk, (size_t)nr * fw, st);
      pg_zero(tkd, (size_t)nr * fw, st);
      pg_gemm(0, 0, nr, fw, kin, xin, kin, Wk, fw, tk, fw, st);
      pg_gemm(0, 0, nr, fw, kin, xind, kin, Wk, fw, tkd, fw, st);
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
      } else {
        pg_zero(dst, (size_t)nr * kin, st);
        pg_zero(dstd, (size_t)nr * kin, st);
      }
      hipLaunchKernelGGL(k_pg_damp, dim3(((size_t)nr * fw + 255) / 256), dim3(256), 0, st, (size_t)nr * fw, c, cd, tk, tkd);
      // weight gradient (tangent): x^T dP + dx^T P; bias: sum dP
      pg_gemm(1, 0, kin, fw, nr, xin, kin, cd, fw, gWk, fw, st);
      pg_gemm(1, 0, kin, fw, nr, xind, kin, c, fw, gWk, fw, st);
      pg_colsum((size_t)nr, fw, cd, nullptr, nullptr, nullptr, 0, gbk, st);
      // input adjoint += P W^T (value and tangent)
      pg_gemm(0, 1, nr, kin, fw, c, fw, Wk, fw, dst, kin, st);
      pg_gemm(0, 1, nr, kin, fw, cd, fw, Wk, fw, dstd, kin, st);
      double* t1 = cur; cur = nxt; nxt = t1;
      double* t2 = curd; curd = nxtd; nxtd = t2;
    }
  }
  // 5. dE/dT with tangents
  hipLaunchKernelGGL(k_pg_desc_bwd, dim3(nrows), dim3(256), 0, st, M, m2, Tm, Tmd, Dg, Dgd, gTm, gTmd);
  // 6. embedding reverse per species pair group
  hipLaunchKernelGGL(k_pg_gbar, dim3(((size_t)np * s1 + 255) / 256), dim3(256), 0, st, (size_t)np, M, m.inv_norm,
                     p_row, gTm, gTmd, R, Rd, T2, T2d, P2, P2d, X1b, X1bd);
  for (int a = 0; a < nt; a++)
    for (int b = 0; b < nt; b++) {
      int g0 = G.group[(a * nt + b) * 2], ng = G.group[(a * nt + b) * 2 + 1];
      if (ng <= 0) continue;
      int net = a * nt + b;
      const double* W1 = th + G.eW[net * 3 + 1];
      const double* W2 = th + G.eW[net * 3 + 2];
      double* gW0 = gt + G.eW[net * 3 + 0];
      double* gB0 = gt + G.eB[net * 3 + 0];
      double* gW1 = gt + G.eW[net * 3 + 1];
      double* gB1 = gt + G.eB[net * 3 + 1];
      double* gW2 = gt + G.eW[net * 3 + 2];
      double* gB2 = gt + G.eB[net * 3 + 2];
      size_t o0 = (size_t)g0 * s0, o1 = (size_t)g0 * s1, o2 = (size_t)g0 * M;
      // layer 2: gW2 += X1^T dP2 + dX1^T P2; gB2 += sum dP2; X1b += P2 W2^T
      pg_gemm(1, 0, s1, M, ng, X1 + o1, s1, P2d + o2, M, gW2, M, st);
      pg_gemm(1, 0, s1, M, ng, X1d + o1, s1, P2 + o2, M, gW2, M, st);
      pg_colsum((size_t)ng, M, P2d + o2, nullptr, nullptr, nullptr, 0, gB2, st);
      pg_gemm(0, 1, ng, s1, M, P2 + o2, M, W2, M, X1b + o1, s1, st);
      pg_gemm(0, 1, ng, s1, M, P2d + o2, M, W2, M, X1bd + o1, s1, st);
      // layer 1: skip to X0b, damp, gradients, X0b += P1 W1^T
      hipLaunchKernelGGL(k_pg_skip, dim3(((size_t)ng * s0 + 255) / 256), dim3(256), 0, st, (size_t)ng, s1, s0, 2,
                         X1b + o1, X1bd + o1, X0b + o0, X0bd + o0);
      hipLaunchKernelGGL(k_pg_damp, dim3(((size_t)ng * s1 + 255) / 256), dim3(256), 0, st, (size_t)ng * s1, X1b + o1,
                         X1bd + o1, T1 + o1, T1d + o1);
      pg_gemm(1, 0, s0, s1, ng, X0 + o0, s0, X1bd + o1, s1, gW1, s1, st);
      pg_gemm(1, 0, s0, s1, ng, X0d + o0, s0, X1b + o1, s1, gW1, s1, st);
      pg_colsum((size_t)ng, s1, X1bd + o1, nullptr, nullptr, nullptr, 0, gB1, st);
      pg_gemm(0, 1, ng, s0, s1, X1b + o1, s1, W1, s1, X0b + o0, s0, st);
      pg_gemm(0, 1, ng, s0, s1, X1bd + o1, s1, W1, s1, X0bd + o0, s0, st);
      // layer 0: P0 = X0b (1 - X0^2); gW0 += sum (s dP0 + ds P0); gB0 += sum dP0
      hipLaunchKernelGGL(k_pg_damp, dim3(((size_t)ng * s0 + 255) / 256), dim3(256), 0, st, (size_t)ng * s0, X0b + o0,
                         X0bd + o0, X0 + o0, X0d + o0);
      pg_colsum((size_t)ng, s0, X0bd + o0, R + 4 * (size_t)g0, X0b + o0, Rd + 4 * (size_t)g0, 4, gW0, st);
      pg_colsum((size_t)ng, s0, X0bd + o0, nullptr, nullptr, nullptr, 0, gB0, st);
    }
  return 0;
}

}  // namespace dp
