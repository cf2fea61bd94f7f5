// Student embedding net: training-side kernels.
//
// The student replaces the embedding net G^{a,b}(s) (Section 2, Eq. 6-9) inside the
// range of s it was trained on by a narrower net  G_s(s) = tanh(s W1 + b1) W2 + b2
// (1 -> H tanh -> M affine).  Training data are (s, G(s)) pairs: s values of real
// neighbours in frames of the full model's own MD trajectory, and G evaluated by the
// full net in FP64.  This file holds
//   * the sample gather (s of every real neighbour slot of one species pair, kept with
//     a given probability using caller-supplied uniform numbers, compacted in slot order),
//   * the full net evaluated at given s (FP64, position-padded net block),
//   * the student's MSE loss and its gradient (FP64 GEMMs),
//   * an Adam update.
#include <hip/hip_runtime.h>

#include "common.h"
#include "devmath.h"
#include "kernels.h"

namespace dp {

void pg_gemm(int ta, int tb, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
             double* C, int ldc, hipStream_t st, bool store);

// keep flag of each (atom, slot) of the species pair (alpha, beta)
__global__ void k_st_flag(int n, int nm, int ntypes, int alpha, int beta, int sel_off, int sel,
                          const int* __restrict__ types, const int* __restrict__ nnei,
                          const float* __restrict__ u, float keep, int* __restrict__ flag) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * nm) return;
  int i = (int)(q / nm), k = (int)(q % nm);
  int f = 0;
  if (types[i] == alpha && k >= sel_off && k < sel_off + sel && (k - sel_off) < nnei[i * ntypes + beta] &&
      u[q] < keep)
    f = 1;
  flag[q] = f;
}

__global__ void k_st_write(int n, int nm, const double* __restrict__ xe, const int* __restrict__ nlist,
                           const int* __restrict__ flag, const int* __restrict__ pos, ModelC m,
                           long cap, double* __restrict__ out) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * nm || !flag[q]) return;
  long p = pos[q];
  if (p >= cap) return;
  int i = (int)(q / nm);
  int e = nlist[q];
  double d0 = xe[3 * e] - xe[3 * i], d1 = xe[3 * e + 1] - xe[3 * i + 1], d2 = xe[3 * e + 2] - xe[3 * i + 2];
  double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double s, ds;
  smooth_fn(m, r, s, ds);
  out[p] = s;
}

void launch_scan_int(int n, const int* in, int* out, int* sums, int* total, hipStream_t st);

// s of every real (alpha, beta) neighbour slot kept with probability keep, compacted in
// slot order: out [min(count, cap)], total[0] = count
void launch_student_gather(int n, const ModelC& m, int alpha, int beta, const int* types, const int* nnei,
                           const int* nlist, const double* xe, const float* u, float keep, int* flag,
                           int* pos, int* sums, int* total, long cap, double* out, hipStream_t st) {
  size_t tot = (size_t)n * m.nm;
  hipLaunchKernelGGL(k_st_flag, dim3((tot + 255) / 256), dim3(256), 0, st, n, m.nm, m.ntypes, alpha, beta,
                     m.sel_off[beta], m.sel[beta], types, nnei, u, keep, flag);
  launch_scan_int((int)tot, flag, pos, sums, total, st);
  hipLaunchKernelGGL(k_st_write, dim3((tot + 255) / 256), dim3(256), 0, st, n, m.nm, xe, nlist, flag, pos, m, cap,
                     out);
}

// full embedding net (alpha, beta) at given s: G [n][M], FP64, one thread per (sample, feature)
// using the flat parameter vector (row-major [in][out] layers)
__global__ void k_st_full_eval(long n, int s0, const double* __restrict__ W0, const double* __restrict__ b0,
                               const double* __restrict__ W1, const double* __restrict__ b1,
                               const double* __restrict__ W2, const double* __restrict__ b2,
                               const double* __restrict__ s, double* __restrict__ G) {
  // one thread per sample: three small layers in registers
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s1 = 2 * s0, M = 4 * s0;
  double h0[32], h1[64];
  double sv = s[i];
  for (int a = 0; a < s0; a++) h0[a] = dp_tanh(sv * W0[a] + b0[a]);
  for (int o = 0; o < s1; o++) {
    double z = b1[o];
    for (int a = 0; a < s0; a++) z += h0[a] * W1[a * s1 + o];
    h1[o] = h0[o % s0] + dp_tanh(z);
  }
  for (int o = 0; o < M; o++) {
    double z = b2[o];
    for (int a = 0; a < s1; a++) z += h1[a] * W2[a * M + o];
    G[i * M + o] = h1[o % s1] + dp_tanh(z);
  }
}

// student forward, layer 1: H = tanh(s W1 + b1)
__global__ void k_st_hidden(long n, int H, const double* __restrict__ s, const double* __restrict__ W1,
                            const double* __restrict__ b1, double* __restrict__ Hm) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * H) return;
  size_t i = q / H;
  int j = (int)(q % H);
  Hm[q] = dp_tanh(s[i] * W1[j] + b1[j]);
}

// Y = H W2 (from the GEMM) + b2; dY = 2 (Y - G) / (n M); the loss summed per block (a
// grid-stride loop over a bounded grid, so the loss takes one atomic per block rather
// than one per wave)
constexpr int kResidBlocks = 2048;
__global__ __launch_bounds__(256) void k_st_resid(long n, int M, const double* __restrict__ b2,
                                                  const double* __restrict__ G, double* __restrict__ Y,
                                                  double* __restrict__ loss) {
  __shared__ double part[4];
  const size_t tot = (size_t)n * M;
  const double inv = 1.0 / ((double)n * M);
  double l = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(q % M);
    const double r = Y[q] + b2[j] - G[q];
    Y[q] = 2.0 * r * inv;
    l += r * r * inv;
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = (part[0] + part[1]) + (part[2] + part[3]);
    if (b != 0.0) unsafeAtomicAdd(loss, b);
  }
}

// dP = dH (1 - H^2) in place
__global__ void k_st_damp(size_t n, const double* __restrict__ Hm, double* __restrict__ dH) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dH[q] *= (1.0 - Hm[q] * Hm[q]);
}

// out[j] += sum_i a[i][j] * (w ? w[i] : 1)
__global__ void k_st_colsum(long n, int N, const double* __restrict__ a, const double* __restrict__ w,
                            double* __restrict__ out) {
  int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double acc = 0.0;
  for (long i = blockIdx.x; i < n; i += gridDim.x) acc += a[i * N + j] * (w ? w[i] : 1.0);
  unsafeAtomicAdd(&out[j], acc);
}

__global__ void k_st_zero(size_t n, double* __restrict__ p) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = 0.0;
}

// design matrix A = [tanh(s W1 + b1), 1]  [n][H + 1]
__global__ void k_st_design(long n, int H, const double* __restrict__ s, const double* __restrict__ W1,
                            const double* __restrict__ b1, double* __restrict__ A) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * (H + 1)) return;
  size_t i = q / (H + 1);
  int j = (int)(q % (H + 1));
  A[q] = j < H ? dp_tanh(s[i] * W1[j] + b1[j]) : 1.0;
}

// Least squares for the output layer: (A^T A + ridge max_diag I) X = A^T G by Cholesky in
// one workgroup (K = H + 1 <= 33 unknowns, M right-hand sides); writes W2 = X[0:H],
// b2 = X[H] into theta.
__global__ __launch_bounds__(128) void k_st_cholsolve(int K, int M, double ridge, double* __restrict__ C,
                                                      double* __restrict__ R, double* __restrict__ W2,
                                                      double* __restrict__ b2) {
  __shared__ double L[33][34];
  __shared__ double dmax;
  const int tid = threadIdx.x;
  for (int q = tid; q < K * K; q += blockDim.x) L[q / K][q % K] = C[q];
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < K; i++) m = fmax(m, L[i][i]);
    dmax = m;
  }
  __syncthreads();
  if (tid < K) L[tid][tid] += ridge * dmax;
  __syncthreads();
  for (int k = 0; k < K; k++) {
    if (tid == 0) L[k][k] = sqrt(L[k][k]);
    __syncthreads();
    if (tid > k && tid < K) L[tid][k] /= L[k][k];
    __syncthreads();
    for (int q = tid; q < K * K; q += blockDim.x) {
      int i = q / K, j = q % K;
      if (i > k && j > k && j <= i) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  for (int c = tid; c < M; c += blockDim.x) {
    double y[33];
    for (int i = 0; i < K; i++) {
      double v = R[i * M + c];
      for (int j = 0; j < i; j++) v -= L[i][j] * y[j];
      y[i] = v / L[i][i];
    }
    for (int i = K - 1; i >= 0; i--) {
      double v = y[i];
      for (int j = i + 1; j < K; j++) v -= L[j][i] * y[j];
      y[i] = v / L[i][i];
    }
    for (int i = 0; i < K - 1; i++) W2[i * M + c] = y[i];
    b2[c] = y[K - 1];
  }
}

size_t student_lsq_scratch_bytes(long n, int H, int M) {
  return sizeof(double) * ((size_t)n * (H + 1) + (size_t)(H + 1) * (H + 1) + (size_t)(H + 1) * M) + 1024;
}

void launch_student_lsq(long n, int H, int M, const double* s, const double* G, double* th, double ridge,
                        void* scratch, hipStream_t st) {
  const int K = H + 1;
  double* A = (double*)scratch;
  double* C = A + (size_t)n * K;
  double* R = C + (size_t)K * K;
  hipLaunchKernelGGL(k_st_design, dim3(((size_t)n * K + 255) / 256), dim3(256), 0, st, n, H, s, th, th + H, A);
  hipLaunchKernelGGL(k_st_zero, dim3((K * K + K * M + 255) / 256), dim3(256), 0, st, (size_t)(K * K + K * M), C);
  pg_gemm(1, 0, K, K, (int)n, A, K, A, K, C, K, st, false);
  pg_gemm(1, 0, K, M, (int)n, A, K, G, M, R, M, st, false);
  hipLaunchKernelGGL(k_st_cholsolve, dim3(1), dim3(128), 0, st, K, M, ridge, C, R, th + 2 * H, th + 2 * H + H * M);
}

// Adam (Kingma & Ba 2015) with bias correction, step t >= 1
__global__ void k_adam(size_t n, double* __restrict__ th, double* __restrict__ m, double* __restrict__ v,
                       const double* __restrict__ g, double lr, double b1, double b2, double eps, double c1,
                       double c2) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double gq = g[q];
  double mq = b1 * m[q] + (1.0 - b1) * gq;
  double vq = b2 * v[q] + (1.0 - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  th[q] -= lr * (mq / c1) / (sqrt(vq / c2) + eps);
}

static void colsum(long n, int N, const double* a, const double* w, double* out, hipStream_t st) {
  dim3 grid((unsigned)std::min<long>(n, 1024), (N + 63) / 64);
  hipLaunchKernelGGL(k_st_colsum, grid, dim3(64), 0, st, n, N, a, w, out);
}

size_t student_scratch_bytes(long n, int H, int M) {
  return sizeof(double) * ((size_t)n * (2 * H + M)) + 1024;
}

// loss (accumulated into loss[0]) and gradient (overwritten) of the student MSE
void launch_student_loss_grad(long n, int H, int M, const double* s, const double* G, const double* th,
                              double* loss, double* grad, void* scratch, hipStream_t st) {
  const double* W1 = th;
  const double* b1 = th + H;
  const double* W2 = th + 2 * H;
  const double* b2 = th + 2 * H + H * M;
  double* gW1 = grad;
  double* gb1 = grad + H;
  double* gW2 = grad + 2 * H;
  double* gb2 = grad + 2 * H + H * M;
  size_t size = 2 * H + (size_t)H * M + M;
  double* Hm = (double*)scratch;
  double* Y = Hm + (size_t)n * H;
  double* dH = Y + (size_t)n * M;
  hipLaunchKernelGGL(k_st_zero, dim3((size + 255) / 256), dim3(256), 0, st, size, grad);
  hipLaunchKernelGGL(k_st_zero, dim3(((size_t)n * M + 255) / 256), dim3(256), 0, st, (size_t)n * M, Y);
  hipLaunchKernelGGL(k_st_zero, dim3(((size_t)n * H + 255) / 256), dim3(256), 0, st, (size_t)n * H, dH);
  hipLaunchKernelGGL(k_st_hidden, dim3(((size_t)n * H + 255) / 256), dim3(256), 0, st, n, H, s, W1, b1, Hm);
  pg_gemm(0, 0, (int)n, M, H, Hm, H, W2, M, Y, M, st, false);
  const size_t rb = ((size_t)n * M + 255) / 256;
  hipLaunchKernelGGL(k_st_resid, dim3(rb < (size_t)kResidBlocks ? (rb ? rb : 1) : kResidBlocks), dim3(256), 0, st, n,
                     M, b2, G, Y, loss);
  // Y now holds dL/dY
  pg_gemm(1, 0, H, M, (int)n, Hm, H, Y, M, gW2, M, st, false);
  colsum(n, M, Y, nullptr, gb2, st);
  pg_gemm(0, 1, (int)n, H, M, Y, M, W2, M, dH, H, st, false);
  hipLaunchKernelGGL(k_st_damp, dim3(((size_t)n * H + 255) / 256), dim3(256), 0, st, (size_t)n * H, Hm, dH);
  colsum(n, H, dH, s, gW1, st);
  colsum(n, H, dH, nullptr, gb1, st);
}

void launch_full_eval(long n, int s0, const double* th_net[6], const double* s, double* G, hipStream_t st) {
  hipLaunchKernelGGL(k_st_full_eval, dim3((n + 127) / 128), dim3(128), 0, st, n, s0, th_net[0], th_net[1],
                     th_net[2], th_net[3], th_net[4], th_net[5], s, G);
}

void launch_adam(size_t n, double* th, double* m, double* v, const double* g, double lr, double b1, double b2,
                 double eps, int t, hipStream_t st) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, n, th, m, v, g, lr, b1, b2, eps, c1, c2);
}

}  // namespace dp
