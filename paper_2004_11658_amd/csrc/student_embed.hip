// Student embedding nets at inference: the forward contraction T and its adjoint.
//
// A student net replaces the embedding net G of a species pair (Section 2, Eq. 6-9)
// inside the range of s it was trained on: G(s) = W2^T h(s) + b2, h(s) = tanh(W1 s + b1),
// with H <= 32 hidden units.  Because G is affine in h, the sums over neighbours j of
// the contraction (Eq. 4, Remark 1) and of its adjoint factor through small per-centre
// products:
//   forward   T = (1/N_m) (W2^T S + b2 rbar^T),   S = sum_j h_j R~_j^T (H x 4),
//                                                  rbar = sum_j R~_j
//   adjoint   with V = W2 dE/dT (H x 4) and u = b2^T dE/dT (4), per neighbour
//             sum_p G_j[p] dE/dT[p][c] = h_j . V[:, c] + u[c]
//             dE/ds_j (through G) = (1/N_m) sum_k (V R~_j)[k] (1 - h_j[k]^2) W1[k]
// so a neighbour costs its environment row, H tanh and 3 x 4 H multiply-adds; no
// per-neighbour matrix product remains.  Neighbours outside the trained range are
// left to the full net (the fallback rows of student_infer.hip).
//
// One wave per centre; lane (rb, g) (rb = lane % 16, g = lane / 16) takes neighbour rb of
// each chunk of 16 and the hidden units k = 16 n + 4 g + q (n < 2, q < 4).
#include <hip/hip_runtime.h>

#include "embed_common.h"

namespace dp {

constexpr int kStuWaves = 8;
constexpr int kStuS = 33 * 4;   // per wave: S (or V) rows k < 32, then rbar (or u)

// sum over the 16 lanes of a row (all lanes get the sum): DPP row rotations by 8, 4, 2, 1
template <int CTRL>
__device__ __forceinline__ float row_rot(float v) { return dpp_mov<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double row_rot(double v) { return dpp_mov<CTRL>(v); }
template <class T>
__device__ __forceinline__ T row_sum16(T v) {
  v += row_rot<0x128>(v);
  v += row_rot<0x124>(v);
  v += row_rot<0x122>(v);
  v += row_rot<0x121>(v);
  return v;
}

// sum over the four rows (lane groups g) of the wave, every lane gets the sum:
// v_permlane32_swap(v, v) pairs each lane with lane +- 32, v_permlane16_swap(v, v)
// each row with its neighbour row
__device__ __forceinline__ float sum_g(float v) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double sum_g(double v) {
  unsigned lo = (unsigned)__double_as_longlong(v), hi = (unsigned)(__double_as_longlong(v) >> 32);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  v = __longlong_as_double((long long)(((unsigned long long)b[0] << 32) | a[0])) +
      __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | a[1]));
  lo = (unsigned)__double_as_longlong(v);
  hi = (unsigned)(__double_as_longlong(v) >> 32);
  const auto c = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto d = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __longlong_as_double((long long)(((unsigned long long)d[0] << 32) | c[0])) +
         __longlong_as_double((long long)(((unsigned long long)d[1] << 32) | c[1]));
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool stu_out_of_range(const EmbedArgs& A, int pair, double s) {
  return s < A.st_lo[pair] || s > A.st_hi[pair];
}

// Environment row of one neighbour (Eq. 5) in the student's storage type: FP64 as
// everywhere else, or FP32 (displacement from the FP64 coordinates, then r, 1/r, the
// switch and R~ in FP32 with the hardware square root and reciprocal, about 1e-7
// relative) for the FP32 student.
template <class T>
struct StuEnv {
  T d[3], ir, s, ds, R[4];
};
__device__ __forceinline__ void stu_env(const ModelC& m, const double xj[3], const double xi[3], StuEnv<double>& v) {
  Env e;
  e.d[0] = xj[0] - xi[0];
  e.d[1] = xj[1] - xi[1];
  e.d[2] = xj[2] - xi[2];
  const double r2 = e.d[0] * e.d[0] + e.d[1] * e.d[1] + e.d[2] * e.d[2];
  e.r = sqrt(r2);
  e.ir = 1.0 / e.r;
  smooth_fn_ir(m, e.r, e.ir, e.s, e.ds);
  const double sr = e.s * e.ir;
  for (int c = 0; c < 3; c++) v.d[c] = e.d[c];
  v.ir = e.ir;
  v.s = e.s;
  v.ds = e.ds;
  v.R[0] = e.s;
  v.R[1] = sr * e.d[0];
  v.R[2] = sr * e.d[1];
  v.R[3] = sr * e.d[2];
}
__device__ __forceinline__ void stu_env(const ModelC& m, const double xj[3], const double xi[3], StuEnv<float>& v) {
  v.d[0] = (float)(xj[0] - xi[0]);
  v.d[1] = (float)(xj[1] - xi[1]);
  v.d[2] = (float)(xj[2] - xi[2]);
  const float r2 = v.d[0] * v.d[0] + v.d[1] * v.d[1] + v.d[2] * v.d[2];
  const float r = __builtin_amdgcn_sqrtf(r2);
  v.ir = __builtin_amdgcn_rcpf(r);
  float w = 0.f, dw = 0.f;
  const float rcs = (float)m.rcs, rc = (float)m.rc, ih = (float)m.inv_h;
  if (r < rcs) {
    w = 1.f;
  } else if (r < rc) {
    // 1 - u = (rc - r) / (rc - rcs) without cancellation, and the quintic in the
    // factored form w = (1 - u)^3 (6 u^2 + 3 u + 1), which keeps its relative precision
    // as w -> 0 at the cutoff (1 + u^3 (-6 u^2 + 15 u - 10) would cancel there in FP32)
    const float om = (rc - r) * ih, u = 1.f - om;
    if (m.switch_kind == 1) {
      float sp, cp;
      __sincosf(3.14159265358979f * om, &sp, &cp);   // cos(pi u) = -cos(pi (1 - u))
      w = 0.5f - 0.5f * cp;
      dw = -0.5f * 3.14159265358979f * sp * ih;      // sin(pi u) = sin(pi (1 - u))
    } else {
      w = om * om * om * (6.f * u * u + 3.f * u + 1.f);
      dw = -30.f * u * u * om * om * ih;
    }
  }
  v.s = w * v.ir;
  v.ds = (dw - w * v.ir) * v.ir;
  const float sr = v.s * v.ir;
  v.R[0] = v.s;
  v.R[1] = sr * v.d[0];
  v.R[2] = sr * v.d[1];
  v.R[3] = sr * v.d[2];
}

// neighbour k of the chunk (its extended index and coordinates), -1 past the end
__device__ __forceinline__ int stu_fetch(const double* __restrict__ xe, const int* __restrict__ nl, int k, int nn,
                                         double (&x)[3]) {
  const int e = k < nn ? nl[k] : -1;
  if (e >= 0) {
    x[0] = xe[3 * e];
    x[1] = xe[3 * e + 1];
    x[2] = xe[3 * e + 2];
  }
  return e;
}

// feature of output position p (positions (f / s0) * 32 + f % s0), or -1
__device__ __forceinline__ int pos_feat(int p, int s0) { return (p % kP0) < s0 ? (p / kP0) * s0 + (p % kP0) : -1; }

size_t stu_lds_bytes(int elem, bool bwd) {
  return (size_t)elem * (kStuElems + kStuWaves * kStuS + (bwd ? kStuWaves * kP2 * 4 : 0));
}

// ------------------------------------------------------------------------------------
// forward: T of each centre
// ------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(64 * kStuWaves) void k_stu_fwd(EmbedArgs A) {
  extern __shared__ __align__(16) char smem[];
  T* sn = (T*)smem;                                    // the pair's student block
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  T* Sw = sn + kStuElems + wv * kStuS;                 // this wave's S and rbar
  const int r0 = blockIdx.x * kStuWaves;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;   // uniform over the block
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  double xi[3] = {0, 0, 0};
  if (atom >= 0) {
    xi[0] = A.xe[3 * atom];
    xi[1] = A.xe[3 * atom + 1];
    xi[2] = A.xe[3 * atom + 2];
  }
  T tacc[2][4];   // T at positions lane and lane + 64 (unscaled)
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int c = 0; c < 4; c++) tacc[i][c] = (T)0;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_bytes(sn, (const T*)A.snets + (size_t)pair * kStuElems, (int)sizeof(T) * kStuElems);
    __syncthreads();
    if (atom < 0) continue;
    T w1[8], b1[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int k = 16 * (j >> 2) + 4 * g + (j & 3);
      w1[j] = sn[kSW1 + k];
      b1[j] = sn[kSB1 + k];
    }
    T S[8][4], rs[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int j = 0; j < 8; j++)
#pragma unroll
      for (int c = 0; c < 4; c++) S[j][c] = (T)0;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    double xn[3] = {0, 0, 0};
    int en = stu_fetch(A.xe, nl, rb, nn, xn);   // the next chunk's neighbour, fetched a chunk ahead
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int e = en;
      const double xj[3] = {xn[0], xn[1], xn[2]};
      en = stu_fetch(A.xe, nl, c0 + 16 + rb, nn, xn);
      T s = (T)0, R[4] = {(T)0, (T)0, (T)0, (T)0};
      if (e >= 0) {
        StuEnv<T> v;
        stu_env(m, xj, xi, v);
        if (stu_out_of_range(A, pair, (double)v.s)) {
          // left to the full net (fallback list); contributes nothing here
          if (g == 0) {
            const int p = atomicAdd(A.fb_count, 1);
            if (p < A.fb_cap) A.fb_list[p] = make_int2(row, e);
          }
        } else {
          s = v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) R[c] = v.R[c];
        }
      }
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const T h = tanh_t(s * w1[j] + b1[j]);
#pragma unroll
        for (int c = 0; c < 4; c++) S[j][c] += h * R[c];
      }
#pragma unroll
      for (int c = 0; c < 4; c++) rs[c] += R[c];
    }
    // sums over the 16 neighbour lanes (each lane group holds all rows for its k)
#pragma unroll
    for (int j = 0; j < 8; j++)
#pragma unroll
      for (int c = 0; c < 4; c++) S[j][c] = row_sum16(S[j][c]);
#pragma unroll
    for (int c = 0; c < 4; c++) rs[c] = row_sum16(rs[c]);
    if (rb == 0) {
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int kk = 16 * (j >> 2) + 4 * g + (j & 3);
#pragma unroll
        for (int c = 0; c < 4; c++) Sw[kk * 4 + c] = S[j][c];
      }
      if (g == 0)
#pragma unroll
        for (int c = 0; c < 4; c++) Sw[32 * 4 + c] = rs[c];
    }
    wave_sync_lds();
    // T += W2^T S + b2 rbar^T at this lane's two positions
    for (int kk = 0; kk < 32; kk++) {
      T s4[4];
#pragma unroll
      for (int c = 0; c < 4; c++) s4[c] = Sw[kk * 4 + c];
      const T wa = sn[kSW2 + kk * kSW2Stride + lane], wb = sn[kSW2 + kk * kSW2Stride + lane + 64];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        tacc[0][c] += wa * s4[c];
        tacc[1][c] += wb * s4[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
      tacc[0][c] += sn[kSB2 + lane] * Sw[32 * 4 + c];
      tacc[1][c] += sn[kSB2 + lane + 64] * Sw[32 * 4 + c];
    }
    wave_sync_lds();   // Sw is rewritten by the next pair
  }
  if (atom < 0) return;
  T* Tout = (T*)A.T + (size_t)row * m.M * 4;
  const T scale = (T)m.inv_norm;
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int f = pos_feat(lane + 64 * i, m.s0);
    if (f >= 0 && f < m.M)
#pragma unroll
      for (int c = 0; c < 4; c++) Tout[f * 4 + c] = tacc[i][c] * scale;
  }
}

// ------------------------------------------------------------------------------------
// adjoint: forces (scattered with atomics to the neighbours' owners) and per-centre virial
// ------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(64 * kStuWaves) void k_stu_bwd(EmbedArgs A) {
  extern __shared__ __align__(16) char smem[];
  T* sn = (T*)smem;
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  T* Vw = sn + kStuElems + wv * kStuS;                                   // V rows, then u
  T* gt = sn + kStuElems + kStuWaves * kStuS + wv * kP2 * 4;            // dE/dT at positions
  const int r0 = blockIdx.x * kStuWaves;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  double xi[3] = {0, 0, 0};
  if (atom >= 0) {
    xi[0] = A.xe[3 * atom];
    xi[1] = A.xe[3 * atom + 1];
    xi[2] = A.xe[3 * atom + 2];
    const T* src = (const T*)A.gT + (size_t)row * m.M * 4;
    for (int q = lane; q < kP2 * 4; q += 64) {
      const int f = pos_feat(q >> 2, m.s0);
      gt[q] = (f >= 0 && f < m.M) ? src[f * 4 + (q & 3)] : (T)0;
    }
  }
  T fi = (T)0;                    // force component g on the centre (lane groups 0..2)
  T vir[3] = {(T)0, (T)0, (T)0};  // virial column g: W[a][g]
  const T inorm = (T)m.inv_norm;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_bytes(sn, (const T*)A.snets + (size_t)pair * kStuElems, (int)sizeof(T) * kStuElems);
    __syncthreads();
    if (atom < 0) continue;
    // V[k][c] = sum_p W2[k][p] gt[p][c]: the lane pair (2 k, 2 k + 1) takes hidden unit k,
    // each lane every other position, and the pair adds its halves (DPP quad_perm 1,0,3,2)
    {
      const int kk = lane >> 1, ph = lane & 1;
      T v4[4] = {(T)0, (T)0, (T)0, (T)0};
      const T* w = sn + kSW2 + kk * kSW2Stride;
      for (int p = ph; p < kP2; p += 2) {
        const T wp = w[p];
#pragma unroll
        for (int c = 0; c < 4; c++) v4[c] += wp * gt[p * 4 + c];
      }
#pragma unroll
      for (int c = 0; c < 4; c++) v4[c] += dpp_mov<DPP_XOR1>(v4[c]);
      if (ph == 0)
#pragma unroll
        for (int c = 0; c < 4; c++) Vw[kk * 4 + c] = v4[c];
      // u[c] = sum_p b2[p] gt[p][c]
      T u[4];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        u[c] = sn[kSB2 + lane] * gt[lane * 4 + c] + sn[kSB2 + lane + 64] * gt[(lane + 64) * 4 + c];
        u[c] = sum_g(row_sum16(u[c]));
      }
      if (lane == 0)
#pragma unroll
        for (int c = 0; c < 4; c++) Vw[32 * 4 + c] = u[c];
    }
    wave_sync_lds();
    T w1[8], b1[8], vk[8][4], uu[4];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int kk = 16 * (j >> 2) + 4 * g + (j & 3);
      w1[j] = sn[kSW1 + kk];
      b1[j] = sn[kSB1 + kk];
#pragma unroll
      for (int c = 0; c < 4; c++) vk[j][c] = Vw[kk * 4 + c];
    }
#pragma unroll
    for (int c = 0; c < 4; c++) uu[c] = Vw[32 * 4 + c];
    wave_sync_lds();   // Vw is rewritten by the next pair
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    double xn[3] = {0, 0, 0};
    int en = stu_fetch(A.xe, nl, rb, nn, xn);   // the next chunk's neighbour, fetched a chunk ahead
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int e = en;
      const double xj[3] = {xn[0], xn[1], xn[2]};
      en = stu_fetch(A.xe, nl, c0 + 16 + rb, nn, xn);
      bool valid = e >= 0;
      StuEnv<T> v;
      T s = (T)0, R[4] = {(T)0, (T)0, (T)0, (T)0};
      if (valid) {
        stu_env(m, xj, xi, v);
        if (stu_out_of_range(A, pair, (double)v.s)) {
          valid = false;   // handled by the fallback kernel
        } else {
          s = v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) R[c] = v.R[c];
        }
      }
      // gR[c] = sum_p G[p] gt[p][c] = h . V[:, c] + u[c];  dsl = dE/ds through G
      T gR[4] = {(T)0, (T)0, (T)0, (T)0}, dsp = (T)0;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const T h = tanh_t(s * w1[j] + b1[j]);
        T dh = (T)0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
          gR[c] += h * vk[j][c];
          dh += vk[j][c] * R[c];
        }
        dsp += dh * ((T)1 - h * h) * w1[j];
      }
#pragma unroll
      for (int c = 0; c < 4; c++) gR[c] = sum_g(gR[c]) + uu[c];
      const T dsl = sum_g(dsp) * inorm;
      // g_ij = dR^T dE/dR (Eq. 5 differentiated): lane group g < 3 computes component g
      if (valid && g < 3) {
        const T gRd[4] = {gR[0] * inorm + dsl, gR[1] * inorm, gR[2] * inorm, gR[3] * inorm};
        const T ir = v.ir;
        const T sr = v.s * ir;
        const T qf = (v.ds * ir - v.s * ir * ir) * ir;
        const T dot = gRd[1] * v.d[0] + gRd[2] * v.d[1] + gRd[3] * v.d[2];
        const T db = g == 0 ? v.d[0] : g == 1 ? v.d[1] : v.d[2];
        const T gRb = g == 0 ? gRd[1] : g == 1 ? gRd[2] : gRd[3];
        const T gv = gRd[0] * v.ds * db * ir + qf * dot * db + sr * gRb;
        fi += gv;
        unsafeAtomicAdd(&A.forces[3 * A.eown[e] + g], -(double)gv);
#pragma unroll
        for (int a = 0; a < 3; a++) vir[a] -= v.d[a] * gv;   // W[a][g]
      }
    }
  }
  if (atom < 0) return;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    fi += __shfl_xor(fi, o);
#pragma unroll
    for (int a = 0; a < 3; a++) vir[a] += __shfl_xor(vir[a], o);
  }
  if (rb == 0 && g < 3) {
    unsafeAtomicAdd(&A.forces[3 * atom + g], (double)fi);
#pragma unroll
    for (int a = 0; a < 3; a++) A.vir_part[(size_t)row * 9 + 3 * a + g] = (double)vir[a];
  }
}

template <class T>
static void stu_fwd_t(const EmbedArgs& a, hipStream_t st) {
  const size_t sh = stu_lds_bytes(sizeof(T), false);
  (void)hipFuncSetAttribute((const void*)k_stu_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_stu_fwd<T>, dim3((a.nrows + kStuWaves - 1) / kStuWaves), dim3(64 * kStuWaves), sh, st, a);
}

template <class T>
static void stu_bwd_t(const EmbedArgs& a, hipStream_t st) {
  const size_t sh = stu_lds_bytes(sizeof(T), true);
  (void)hipFuncSetAttribute((const void*)k_stu_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL(k_stu_bwd<T>, dim3((a.nrows + kStuWaves - 1) / kStuWaves), dim3(64 * kStuWaves), sh, st, a);
}

// The student blocks are FP64 in the FP64 mode and FP32 otherwise: with no per-neighbour
// matrix product left, the operand-precision modes do not apply to the student path.
void launch_student_fwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) stu_fwd_t<double>(a, st);
  else stu_fwd_t<float>(a, st);
}

void launch_student_bwd(const EmbedArgs& a, hipStream_t st) {
  if (a.prec == PREC_FP64) stu_bwd_t<double>(a, st);
  else stu_bwd_t<float>(a, st);
}

}  // namespace dp
