// Student embedding net at inference: forward contraction and adjoint.
//
// Same work layout and transposed MFMA formulation as the full embedding kernels, but
// the per-neighbour net is the student G_s(s) = tanh(s W1 + b1) W2 + b2 (1 -> H <= 32
// -> M): per 16-neighbour chunk 8 tanh and 64 MFMA instead of 56 tanh and 160 MFMA.
// Its outputs use the same position layout as the full net's G, so the contraction
// and everything downstream are unchanged.
//
// A neighbour whose s lies outside the student's trained range [s_lo, s_hi] of its
// species pair is left out of these kernels and appended to a fallback list; the full
// net handles those rows afterwards (k_fb_fwd / k_fb_bwd, FP64, one wave per row).
#include <hip/hip_runtime.h>

#include "embed_common.h"

namespace dp {

template <class T>
__device__ __forceinline__ void stage_student(T* __restrict__ dst, const T* __restrict__ src) {
  for (int q = threadIdx.x; q < kStuElems; q += blockDim.x) dst[q] = src[q];
}

template <class T>
__device__ __forceinline__ void student_fwd(const T* __restrict__ sn, T s, int g, int rb, T (&h)[2][4],
                                            T (&G)[8][4]) {
  typedef typename Acc4<T>::type A4;
#pragma unroll
  for (int n = 0; n < 2; n++)
#pragma unroll
    for (int q = 0; q < 4; q++) {
      int p = 16 * n + LP(g, q);
      h[n][q] = tanh_t(s * sn[kSW1 + p] + sn[kSB1 + p]);
    }
#pragma unroll
  for (int mt = 0; mt < 8; mt++) {
    A4 c = {0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < 2; n++)
#pragma unroll
      for (int q = 0; q < 4; q++) c = mfma4(sn[kSW2 + (16 * n + LP(g, q)) * kSW2Stride + 16 * mt + rb], h[n][q], c);
#pragma unroll
    for (int q = 0; q < 4; q++) G[mt][q] = c[q] + sn[kSB2 + 16 * mt + LP(g, q)];
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ bool out_of_range(const EmbedArgs& A, int pair, double s) {
  return s < A.st_lo[pair] || s > A.st_hi[pair];
}

template <class T, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_student_fwd(EmbedArgs A) {
  extern __shared__ __align__(16) char smem_raw[];
  T* sn = (T*)smem_raw;
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * WPB;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  double xi[3] = {0, 0, 0};
  if (atom >= 0) {
    xi[0] = A.xe[3 * atom];
    xi[1] = A.xe[3 * atom + 1];
    xi[2] = A.xe[3 * atom + 2];
  }
  T acc[8];
#pragma unroll
  for (int j = 0; j < 8; j++) acc[j] = (T)0;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_student<T>(sn, (const T*)A.snets + (size_t)pair * kStuElems);
    __syncthreads();
    if (atom < 0) continue;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int k = c0 + rb;
      Env v;
      T s = (T)0;
      T R[4] = {(T)0, (T)0, (T)0, (T)0};
      if (k < nn) {
        int e = nl[k];
        env_row(m, A.xe, e, xi, v);
        if (out_of_range(A, pair, v.s)) {
          if (g == 0) {
            int p = atomicAdd(A.fb_count, 1);
            if (p < A.fb_cap) A.fb_list[p] = make_int2(row, e);
          }
        } else {
          s = (T)v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
        }
      }
      T h[2][4], G[8][4];
      student_fwd<T>(sn, s, g, rb, h, G);
      const bool b3 = rb & 8, b2 = rb & 4, b1 = rb & 2, b0 = rb & 1;
      T vv[64];
#pragma unroll
      for (int kk = 0; kk < 64; kk++) {
        int mt = kk >> 4, q = (kk >> 2) & 3, c = kk & 3;
        T a = G[mt][q] * R[c];
        T b = G[mt + 4][q] * R[c];
        T send = b3 ? a : b;
        T keep = b3 ? b : a;
        vv[kk] = keep + dpp_mov<DPP_ROR8>(send);
        if ((kk & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
      rs_step<T, 64, DPP_HALF_MIRROR>(vv, b2);
      rs_step<T, 32, DPP_XOR2>(vv, b1);
      rs_step<T, 16, DPP_XOR1>(vv, b0);
#pragma unroll
      for (int j = 0; j < 8; j++) acc[j] += vv[j];
    }
  }
  if (atom < 0) return;
  write_T<T>((T*)A.T + (size_t)row * m.M * 4, acc, rb, g, m.s0, (T)m.inv_norm);
}

template <class T, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_student_bwd(EmbedArgs A) {
  extern __shared__ __align__(16) char smem_raw[];
  T* sn = (T*)smem_raw;
  T* gts = sn + kStuElems + 64;
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * WPB;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  T* gt = gts + wv * kP2 * 4;
  double xi[3] = {0, 0, 0};
  if (atom >= 0) {
    xi[0] = A.xe[3 * atom];
    xi[1] = A.xe[3 * atom + 1];
    xi[2] = A.xe[3 * atom + 2];
    const T* src = (const T*)A.gT + (size_t)row * m.M * 4;
    for (int q = lane; q < kP2 * 4; q += 64) {
      int p = q >> 2, c = q & 3;
      int f = (p % kP0) < m.s0 ? (p / kP0) * m.s0 + (p % kP0) : -1;
      gt[q] = f >= 0 ? src[f * 4 + c] : (T)0;
    }
  }
  double fi[3] = {0, 0, 0};
  double vir[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const T inorm = (T)m.inv_norm;
  typedef typename Acc4<T>::type A4;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_student<T>(sn, (const T*)A.snets + (size_t)pair * kStuElems);
    __syncthreads();
    if (atom < 0) continue;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int k = c0 + rb;
      bool valid = k < nn;
      Env v;
      int e = -1;
      T s = (T)0;
      T R[4] = {(T)0, (T)0, (T)0, (T)0};
      if (valid) {
        e = nl[k];
        env_row(m, A.xe, e, xi, v);
        if (out_of_range(A, pair, v.s)) {
          valid = false;  // handled by the fallback kernel
        } else {
          s = (T)v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
        }
      }
      T h[2][4], G[8][4];
      student_fwd<T>(sn, s, g, rb, h, G);
      T gR[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
      for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const T* gp = gt + (16 * mt + LP(g, q)) * 4;
#pragma unroll
          for (int c = 0; c < 4; c++) gR[c] += G[mt][q] * gp[c];
          G[mt][q] = (gp[0] * R[0] + gp[1] * R[1] + gp[2] * R[2] + gp[3] * R[3]) * inorm;  // now dE/dG
        }
      // dE/dh = W2 . dE/dG, then through tanh and W1 to dE/ds
      T dsl = (T)0;
#pragma unroll
      for (int nt = 0; nt < 2; nt++) {
        A4 c = {0, 0, 0, 0};
#pragma unroll
        for (int mt = 0; mt < 8; mt++)
#pragma unroll
          for (int q = 0; q < 4; q++)
            c = mfma4(sn[kSW2 + (16 * nt + rb) * kSW2Stride + 16 * mt + LP(g, q)], G[mt][q], c);
#pragma unroll
        for (int q = 0; q < 4; q++)
          dsl += c[q] * ((T)1 - h[nt][q] * h[nt][q]) * sn[kSW1 + 16 * nt + LP(g, q)];
        __builtin_amdgcn_sched_barrier(0);
      }
      dsl += shfl_x(dsl, 16);
      dsl += shfl_x(dsl, 32);
#pragma unroll
      for (int c = 0; c < 4; c++) {
        gR[c] += shfl_x(gR[c], 16);
        gR[c] += shfl_x(gR[c], 32);
      }
      if (valid && g == 0) {
        double gRd[4] = {(double)gR[0] * m.inv_norm + (double)dsl, (double)gR[1] * m.inv_norm,
                         (double)gR[2] * m.inv_norm, (double)gR[3] * m.inv_norm};
        double ir = 1.0 / v.r;
        double sr = v.s * ir;
        double qf = (v.ds * ir - v.s * ir * ir) * ir;
        double dot = gRd[1] * v.d[0] + gRd[2] * v.d[1] + gRd[3] * v.d[2];
        double gv[3];
#pragma unroll
        for (int b = 0; b < 3; b++) gv[b] = gRd[0] * v.ds * v.d[b] * ir + qf * dot * v.d[b] + sr * gRd[1 + b];
        int own = A.eown[e];
#pragma unroll
        for (int b = 0; b < 3; b++) {
          fi[b] += gv[b];
          unsafeAtomicAdd(&A.forces[3 * own + b], -gv[b]);
        }
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) vir[3 * a + b] -= v.d[a] * gv[b];
      }
    }
  }
  if (atom < 0) return;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int b = 0; b < 3; b++) fi[b] += __shfl_xor(fi[b], o);
#pragma unroll
    for (int q = 0; q < 9; q++) vir[q] += __shfl_xor(vir[q], o);
  }
  if (lane == 0) {
#pragma unroll
    for (int b = 0; b < 3; b++) unsafeAtomicAdd(&A.forces[3 * atom + b], fi[b]);
  }
  if (lane < 9) {
    double val = 0;
#pragma unroll
    for (int q = 0; q < 9; q++) val = (lane == q) ? vir[q] : val;
    A.vir_part[(size_t)row * 9 + lane] = val;
  }
}

// ------------------------------------------------------------------------------------
// fallback rows: the full net in FP64 from the flat parameters
// ------------------------------------------------------------------------------------
struct FbNet {
  const double *W0, *b0, *W1, *b1, *W2, *b2;
};

__device__ __forceinline__ FbNet fb_net(const EmbedArgs& A, int pair) {
  const int64_t* o = A.net_off + pair * 6;
  FbNet n;
  n.W0 = A.theta + o[0];
  n.b0 = A.theta + o[1];
  n.W1 = A.theta + o[2];
  n.b1 = A.theta + o[3];
  n.W2 = A.theta + o[4];
  n.b2 = A.theta + o[5];
  return n;
}

// one wave (64 lanes) per fallback row; features spread over the lanes
template <class T>
__global__ __launch_bounds__(64) void k_fb_fwd(EmbedArgs A) {
  __shared__ double h0[32], h1[64], env[8];
  const ModelC& m = A.m;
  const int lane = threadIdx.x;
  const int cnt = min(*A.fb_count, A.fb_cap);
  const int s0 = m.s0, s1 = 2 * s0, M = m.M;
  for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
    const int2 it = A.fb_list[idx];
    const int row = it.x, e = it.y;
    const int atom = A.row_atom[row];
    const FbNet nt = fb_net(A, A.etype[atom] * m.ntypes + A.etype[e]);
    if (lane == 0) {
      double xi[3] = {A.xe[3 * atom], A.xe[3 * atom + 1], A.xe[3 * atom + 2]};
      Env v;
      env_row(m, A.xe, e, xi, v);
      env[0] = v.s;
      for (int c = 0; c < 4; c++) env[1 + c] = v.R[c];
    }
    __syncthreads();
    const double s = env[0];
    if (lane < s0) h0[lane] = dp_tanh(s * nt.W0[lane] + nt.b0[lane]);
    __syncthreads();
    if (lane < s1) {
      double z = nt.b1[lane];
      for (int a = 0; a < s0; a++) z += h0[a] * nt.W1[a * s1 + lane];
      h1[lane] = h0[lane % s0] + dp_tanh(z);
    }
    __syncthreads();
    T* Tr = (T*)A.T + (size_t)row * M * 4;
    for (int o = lane; o < M; o += 64) {
      double z = nt.b2[o];
      for (int a = 0; a < s1; a++) z += h1[a] * nt.W2[a * M + o];
      double G = h1[o % s1] + dp_tanh(z);
      for (int c = 0; c < 4; c++) unsafeAtomicAdd(&Tr[o * 4 + c], (T)(G * env[1 + c] * m.inv_norm));
    }
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(64) void k_fb_bwd(EmbedArgs A) {
  __shared__ double t0[32], t1[64], h1[64], gg[128], d2[128], gh1[64], d1[64], envs[16];
  const ModelC& m = A.m;
  const int lane = threadIdx.x;
  const int cnt = min(*A.fb_count, A.fb_cap);
  const int s0 = m.s0, s1 = 2 * s0, M = m.M;
  for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
    const int2 it = A.fb_list[idx];
    const int row = it.x, e = it.y;
    const int atom = A.row_atom[row];
    const FbNet nt = fb_net(A, A.etype[atom] * m.ntypes + A.etype[e]);
    if (lane == 0) {
      double xi[3] = {A.xe[3 * atom], A.xe[3 * atom + 1], A.xe[3 * atom + 2]};
      Env v;
      env_row(m, A.xe, e, xi, v);
      envs[0] = v.s; envs[1] = v.ds; envs[2] = v.r;
      for (int c = 0; c < 3; c++) envs[3 + c] = v.d[c];
      for (int c = 0; c < 4; c++) envs[6 + c] = v.R[c];
    }
    __syncthreads();
    const double s = envs[0];
    if (lane < s0) t0[lane] = dp_tanh(s * nt.W0[lane] + nt.b0[lane]);
    __syncthreads();
    if (lane < s1) {
      double z = nt.b1[lane];
      for (int a = 0; a < s0; a++) z += t0[a] * nt.W1[a * s1 + lane];
      t1[lane] = dp_tanh(z);
      h1[lane] = t0[lane % s0] + t1[lane];
    }
    __syncthreads();
    const T* gT = (const T*)A.gT + (size_t)row * M * 4;
    double gR[4] = {0, 0, 0, 0};
    for (int o = lane; o < M; o += 64) {
      double z = nt.b2[o];
      for (int a = 0; a < s1; a++) z += h1[a] * nt.W2[a * M + o];
      double t2 = dp_tanh(z);
      double G = h1[o % s1] + t2;
      double g = 0.0;
      for (int c = 0; c < 4; c++) {
        double gt = (double)gT[o * 4 + c];
        gR[c] += G * gt;
        g += gt * envs[6 + c];
      }
      g *= m.inv_norm;
      gg[o] = g;
      d2[o] = g * (1.0 - t2 * t2);
    }
    __syncthreads();
    if (lane < s1) {
      double v = gg[lane] + gg[lane + s1];   // concat skip of the last layer
      for (int o = 0; o < M; o++) v += d2[o] * nt.W2[lane * M + o];
      gh1[lane] = v;
      d1[lane] = v * (1.0 - t1[lane] * t1[lane]);
    }
    __syncthreads();
    double ds = 0.0;
    if (lane < s0) {
      double v = gh1[lane] + gh1[lane + s0];   // concat skip of the middle layer
      for (int o = 0; o < s1; o++) v += d1[o] * nt.W1[lane * s1 + o];
      ds = v * (1.0 - t0[lane] * t0[lane]) * nt.W0[lane];
    }
    for (int o = 32; o > 0; o >>= 1) {
      ds += __shfl_xor(ds, o);
      for (int c = 0; c < 4; c++) gR[c] += __shfl_xor(gR[c], o);
    }
    if (lane == 0) {
      const double vs = envs[0], vds = envs[1], vr = envs[2];
      const double d[3] = {envs[3], envs[4], envs[5]};
      double gRd[4] = {gR[0] * m.inv_norm + ds, gR[1] * m.inv_norm, gR[2] * m.inv_norm, gR[3] * m.inv_norm};
      double ir = 1.0 / vr, sr = vs * ir, qf = (vds * ir - vs * ir * ir) * ir;
      double dot = gRd[1] * d[0] + gRd[2] * d[1] + gRd[3] * d[2];
      double gv[3];
      for (int b = 0; b < 3; b++) gv[b] = gRd[0] * vds * d[b] * ir + qf * dot * d[b] + sr * gRd[1 + b];
      int own = A.eown[e];
      for (int b = 0; b < 3; b++) {
        unsafeAtomicAdd(&A.forces[3 * atom + b], gv[b]);
        unsafeAtomicAdd(&A.forces[3 * own + b], -gv[b]);
      }
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) unsafeAtomicAdd(&A.vir_part[(size_t)row * 9 + 3 * a + b], -d[a] * gv[b]);
    }
    __syncthreads();
  }
}

constexpr int kStuWaves = 8;

void launch_student_fwd(const EmbedArgs& a, hipStream_t st) {
  int grid = (a.nrows + kStuWaves - 1) / kStuWaves;
  if (a.prec == PREC_FP64) {
    hipLaunchKernelGGL((k_student_fwd<double, kStuWaves>), dim3(grid), dim3(64 * kStuWaves),
                       sizeof(double) * kStuElems, st, a);
  } else {
    hipLaunchKernelGGL((k_student_fwd<float, kStuWaves>), dim3(grid), dim3(64 * kStuWaves),
                       sizeof(float) * kStuElems, st, a);
  }
}

void launch_fallback_fwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) hipLaunchKernelGGL(k_fb_fwd<double>, dim3(1024), dim3(64), 0, st, a);
  else hipLaunchKernelGGL(k_fb_fwd<float>, dim3(1024), dim3(64), 0, st, a);
}

void launch_fallback_bwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) hipLaunchKernelGGL(k_fb_bwd<double>, dim3(1024), dim3(64), 0, st, a);
  else hipLaunchKernelGGL(k_fb_bwd<float>, dim3(1024), dim3(64), 0, st, a);
}

void launch_student_bwd(const EmbedArgs& a, hipStream_t st) {
  int grid = (a.nrows + kStuWaves - 1) / kStuWaves;
  if (a.prec == PREC_FP64) {
    size_t sh = sizeof(double) * (kStuElems + 64 + kStuWaves * kP2 * 4);
    (void)hipFuncSetAttribute((const void*)k_student_bwd<double, kStuWaves>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_student_bwd<double, kStuWaves>), dim3(grid), dim3(64 * kStuWaves), sh, st, a);
  } else {
    size_t sh = sizeof(float) * (kStuElems + 64 + kStuWaves * kP2 * 4);
    hipLaunchKernelGGL((k_student_bwd<float, kStuWaves>), dim3(grid), dim3(64 * kStuWaves), sh, st, a);
  }
}

}  // namespace dp
