// Fallback rows of the student embedding nets at inference.
//
// The student kernels (student_embed.hip) leave out every neighbour whose s lies
// outside the student's trained range
// [s_lo, s_hi] of its species pair and append it to a fallback list; these kernels
// evaluate the full net for those rows afterwards in FP64 (one wave per row) and add
// their contribution to T, and in the adjoint to the forces and the virial.
#include <hip/hip_runtime.h>

#include "embed_common.h"

namespace dp {

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
  if (blockIdx.x == 0 && lane == 0 && A.fb_note) *A.fb_note = cnt;
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
#pragma unroll 8
      for (int a = 0; a < s0; a++) z += h0[a] * nt.W1[a * s1 + lane];
      h1[lane] = h0[lane % s0] + dp_tanh(z);
    }
    __syncthreads();
    T* Tr = (T*)A.T + (size_t)row * M * 4;
    for (int o = lane; o < M; o += 64) {
      double z = nt.b2[o];
#pragma unroll 8
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
  if (blockIdx.x == 0 && lane == 0 && A.fb_note) *A.fb_note = cnt;
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
#pragma unroll 8
      for (int a = 0; a < s0; a++) z += t0[a] * nt.W1[a * s1 + lane];
      t1[lane] = dp_tanh(z);
      h1[lane] = t0[lane % s0] + t1[lane];
    }
    __syncthreads();
    const T* gT = (const T*)A.gT + (size_t)row * M * 4;
    double gR[4] = {0, 0, 0, 0};
    for (int o = lane; o < M; o += 64) {
      double z = nt.b2[o];
#pragma unroll 8
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
#pragma unroll 8
      for (int o = 0; o < M; o++) v += d2[o] * nt.W2[lane * M + o];
      gh1[lane] = v;
      d1[lane] = v * (1.0 - t1[lane] * t1[lane]);
    }
    __syncthreads();
    double ds = 0.0;
    if (lane < s0) {
      double v = gh1[lane] + gh1[lane + s0];   // concat skip of the middle layer
#pragma unroll 8
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

// The row count lives on the device, so the grid is fixed: 16 one-wave blocks per CU, so
// that a few thousand rows run about one per wave (each row is a chain of dependent
// loads and products, latency-bound); surplus blocks exit at once.
constexpr int kFbBlocks = 4096;

void launch_fallback_fwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) hipLaunchKernelGGL(k_fb_fwd<double>, dim3(kFbBlocks), dim3(64), 0, st, a);
  else hipLaunchKernelGGL(k_fb_fwd<float>, dim3(kFbBlocks), dim3(64), 0, st, a);
}

void launch_fallback_bwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) hipLaunchKernelGGL(k_fb_bwd<double>, dim3(kFbBlocks), dim3(64), 0, st, a);
  else hipLaunchKernelGGL(k_fb_bwd<float>, dim3(kFbBlocks), dim3(64), 0, st, a);
}


}  // namespace dp
