// Embedding net, descriptor contraction and its adjoint (paper Section 2, Eq. 4-10;
// Section 3.2.3 for the fused bias / tanh / tanh-gradient epilogues).
//
// Work layout.  Rows (centre atoms) are grouped by species and padded (kRowPad); a
// workgroup of WPB waves handles WPB centres of one species alpha, one wave per centre.
// For each neighbour species beta the workgroup stages the position-padded net
// (alpha, beta) in LDS and every wave walks its centre's real neighbours of species
// beta in chunks of 16 (padded slots hold no atom and are skipped: their R rows are 0).
//
// Transposed MFMA chain.  A layer y = x W + b is evaluated as y^T = W^T x^T on the
// 16x16x4 MFMA: the weights are the A operand (read from LDS), the activations the B
// operand, so the 16 neighbour rows run along lane % 16 and the features along
// (lane / 16, accumulator register).  Layer outputs come out in exactly the layout the
// next layer needs as its B operand (the k order of each MFMA step is permuted to
// match), so activations never leave registers.  Features are placed at "positions":
// feature f of a width-s0 block sits at position (f / s0) * 32 + f % s0; with this
// placement the concatenation skip (x, x) of Eq. 9 adds values held by the same lane
// and register, and the pads (position % 32 >= s0) carry zero weights and stay zero.
//
// The contraction T = G^T R / N_m (Eq. 4) reduces over the 16 rows of a chunk with a
// lane reduce-scatter (16 lanes -> 8 values per lane), accumulated over chunks.
//
// The adjoint recomputes G (no per-neighbour activations are stored) and runs the
// chain backwards with the transposed weight access, fusing 1 - tanh^2 into the MFMA
// operand preparation; g_ij = dR^T dE/dR, F_i += g, F_j -= g (FP64 atomics), and the
// per-centre virial -d (x) g.
//
// Operand precision is a policy of the kernels: NetNative<T> runs the layers on the
// 16x16x4 MFMA in T (FP64 or FP32); NetBF16<PARTS> rounds the layer inputs to BF16 and
// runs v_mfma_f32_16x16x32_bf16 with FP32 accumulation, one k chunk of 32 positions per
// instruction, against weights pre-packed per lane (PARTS = 2 splits both operands
// into hi + lo BF16 and sums hi hi + hi lo + lo hi).  Everything outside the layer
// products (s, L0, biases, tanh, the skips, the contraction) stays in FP32.
#include <hip/hip_runtime.h>

#include "common.h"
#include "embed_common.h"

namespace dp {

// forward chain of one 16-row chunk: t0 (L0 = tanh), t1, t2 (tanh parts of L1, L2)
template <class T>
__device__ __forceinline__ void chain_fwd(const T* __restrict__ net, T s, int g, int rb,
                                          T (&t0)[2][4], T (&t1)[4][4], T (&t2)[8][4]) {
  typedef typename Acc4<T>::type A4;
#pragma unroll
  for (int n = 0; n < 2; n++)
#pragma unroll
    for (int q = 0; q < 4; q++) {
      int p = 16 * n + LP(g, q);
      t0[n][q] = tanh_t(s * net[kOffW0 + p] + net[kOffB0 + p]);
    }
#pragma unroll
  for (int mt = 0; mt < 4; mt++) {
    A4 c = {0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < 2; n++)
#pragma unroll
      for (int q = 0; q < 4; q++)
        c = mfma4(net[kOffW1 + (16 * n + LP(g, q)) * kW1Stride + 16 * mt + rb], t0[n][q], c);
#pragma unroll
    for (int q = 0; q < 4; q++) t1[mt][q] = tanh_t(c[q] + net[kOffB1 + 16 * mt + LP(g, q)]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // h1 = (h0, h0) + t1, h0 = t0
  T h1[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; mt++)
#pragma unroll
    for (int q = 0; q < 4; q++) h1[mt][q] = t0[mt & 1][q] + t1[mt][q];
#pragma unroll
  for (int mt = 0; mt < 8; mt++) {
    A4 c = {0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < 4; n++)
#pragma unroll
      for (int q = 0; q < 4; q++)
        c = mfma4(net[kOffW2 + (16 * n + LP(g, q)) * kW2Stride + 16 * mt + rb], h1[n][q], c);
#pragma unroll
    for (int q = 0; q < 4; q++) t2[mt][q] = tanh_t(c[q] + net[kOffB2 + 16 * mt + LP(g, q)]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// G = (h1, h1) + t2 with h1 = (t0, t0) + t1, at position 16 mt + lpos(g, q)
template <class T>
__device__ __forceinline__ T g_at(const T (&t0)[2][4], const T (&t1)[4][4], const T (&t2)[8][4],
                                  int mt, int q) {
  return t0[mt & 1][q] + t1[mt & 3][q] + t2[mt][q];
}


// ------------------------------------------------------------------------------------
// operand policies
// ------------------------------------------------------------------------------------
template <class T>
struct NetNative {
  typedef T Tv;
  static constexpr int kFwdBytes = sizeof(T) * kNetElems;   // staged by the forward kernel
  static constexpr int kBwdBytes = sizeof(T) * kNetElems;   // staged by the adjoint kernel
  static constexpr int kBlockBytes = sizeof(T) * kNetElems; // stride of the net blocks
  __device__ static const T* fpart(const char* sm) { return (const T*)sm; }
  __device__ static void fwd(const char* sm, T s, int g, int rb, int lane, T (&t0)[2][4], T (&t1)[4][4],
                             T (&t2)[8][4]) {
    chain_fwd<T>((const T*)sm, s, g, rb, t0, t1, t2);
  }
  // out[nt] = (W2 d2)[nt] at layer-1 output positions 16 nt + lpos(g, q)
  __device__ static void adj2(const char* sm, const T (&d2)[8][4], int g, int rb, int lane, T (&out)[4][4]) {
    typedef typename Acc4<T>::type A4;
    const T* net = (const T*)sm;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      A4 c = {0, 0, 0, 0};
#pragma unroll
      for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int q = 0; q < 4; q++)
          c = mfma4(net[kOffW2 + (16 * nt + rb) * kW2Stride + 16 * mt + LP(g, q)], d2[mt][q], c);
#pragma unroll
      for (int q = 0; q < 4; q++) out[nt][q] = c[q];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // out[nt] = (W1 d1)[nt] at layer-0 output positions 16 nt + lpos(g, q)
  __device__ static void adj1(const char* sm, const T (&d1)[4][4], int g, int rb, int lane, T (&out)[2][4]) {
    typedef typename Acc4<T>::type A4;
    const T* net = (const T*)sm;
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
      A4 c = {0, 0, 0, 0};
#pragma unroll
      for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int q = 0; q < 4; q++)
          c = mfma4(net[kOffW1 + (16 * nt + rb) * kW1Stride + 16 * mt + LP(g, q)], d1[mt][q], c);
#pragma unroll
      for (int q = 0; q < 4; q++) out[nt][q] = c[q];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
};

// BF16 operands.  In the packed tiles, lane (g, rb) element j of k chunk kc stands for
// the position 16 (2 kc + j / 4) + 4 g + j % 4 of the layer input: exactly the value the
// lane holds in register j % 4 of tile 2 kc + j / 4, so a chunk of the B operand is two
// accumulator tiles rounded to BF16 in place.
template <int PARTS>
struct NetBF16 {
  typedef float Tv;
  static constexpr int kFloatBytes = 4 * kBFloat;
  static constexpr int kFwdBytes = kFloatBytes + PARTS * 2 * kBFwd;
  static constexpr int kBwdBytes = kFwdBytes + PARTS * 2 * kBBwd;
  static constexpr int kBlockBytes = 2 * bnet_u16(PARTS);
  __device__ static const float* fpart(const char* sm) { return (const float*)sm; }
  // tile t of a packed group starting at byte offset off, part (0 hi, 1 lo), group size gs (u16)
  __device__ static bf8 tile(const char* sm, int off, int part, int gs, int t, int lane) {
    return ((const bf8*)(sm + off + part * 2 * gs))[t * 64 + lane];
  }
  template <int NT>
  __device__ static void pack(const float (&v)[NT][4], int kc, bf8& hi, bf8& lo) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = v[2 * kc + j / 4][j % 4];
    split8<PARTS>(x, hi, lo);
  }
  __device__ static void fwd(const char* sm, float s, int g, int rb, int lane, float (&t0)[2][4],
                             float (&t1)[4][4], float (&t2)[8][4]) {
    const float* fn = (const float*)sm;
    const int oF = kFloatBytes;
#pragma unroll
    for (int n = 0; n < 2; n++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int p = 16 * n + 4 * g + q;
        t0[n][q] = tanh_t(s * fn[kOffW0 + p] + fn[kOffB0 + p]);
      }
    bf8 xh, xl;
    pack<2>(t0, 0, xh, xl);
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
      f4v c = {0, 0, 0, 0};
      bf8 wh = tile(sm, oF, 0, kBFwd, mt, lane);
      bf8 wl = PARTS == 2 ? tile(sm, oF, 1, kBFwd, mt, lane) : wh;
      c = mfma_split<PARTS>(wh, wl, xh, xl, c);
#pragma unroll
      for (int q = 0; q < 4; q++) t1[mt][q] = tanh_t(c[q] + fn[kOffB1 + 16 * mt + 4 * g + q]);
    }
    __builtin_amdgcn_sched_barrier(0);
    float h1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
      for (int q = 0; q < 4; q++) h1[mt][q] = t0[mt & 1][q] + t1[mt][q];
    bf8 hh[2], hl[2];
    pack<4>(h1, 0, hh[0], hl[0]);
    pack<4>(h1, 1, hh[1], hl[1]);
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 2; kc++) {
        bf8 wh = tile(sm, oF + 2 * kBW1F, 0, kBFwd, 2 * mt + kc, lane);
        bf8 wl = PARTS == 2 ? tile(sm, oF + 2 * kBW1F, 1, kBFwd, 2 * mt + kc, lane) : wh;
        c = mfma_split<PARTS>(wh, wl, hh[kc], hl[kc], c);
      }
#pragma unroll
      for (int q = 0; q < 4; q++) t2[mt][q] = tanh_t(c[q] + fn[kOffB2 + 16 * mt + 4 * g + q]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __device__ static void adj2(const char* sm, const float (&d2)[8][4], int g, int rb, int lane,
                              float (&out)[4][4]) {
    const int oB = kFwdBytes + 2 * kBW1B;
    bf8 xh[4], xl[4];
#pragma unroll
    for (int kc = 0; kc < 4; kc++) pack<8>(d2, kc, xh[kc], xl[kc]);
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 4; kc++) {
        bf8 wh = tile(sm, oB, 0, kBBwd, 4 * nt + kc, lane);
        bf8 wl = PARTS == 2 ? tile(sm, oB, 1, kBBwd, 4 * nt + kc, lane) : wh;
        c = mfma_split<PARTS>(wh, wl, xh[kc], xl[kc], c);
      }
#pragma unroll
      for (int q = 0; q < 4; q++) out[nt][q] = c[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ static void adj1(const char* sm, const float (&d1)[4][4], int g, int rb, int lane,
                              float (&out)[2][4]) {
    const int oB = kFwdBytes;
    bf8 xh[2], xl[2];
#pragma unroll
    for (int kc = 0; kc < 2; kc++) pack<4>(d1, kc, xh[kc], xl[kc]);
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 2; kc++) {
        bf8 wh = tile(sm, oB, 0, kBBwd, 2 * nt + kc, lane);
        bf8 wl = PARTS == 2 ? tile(sm, oB, 1, kBBwd, 2 * nt + kc, lane) : wh;
        c = mfma_split<PARTS>(wh, wl, xh[kc], xl[kc], c);
      }
#pragma unroll
      for (int q = 0; q < 4; q++) out[nt][q] = c[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
};

// ------------------------------------------------------------------------------------
// forward: T_i = (1/N_m) sum_j G_j^T R_j
// ------------------------------------------------------------------------------------
template <class NP, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_embed_fwd(EmbedArgs A) {
  typedef typename NP::Tv T;
  extern __shared__ __align__(16) char smem_raw[];
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * WPB;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;  // uniform over the block
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
    __syncthreads();
    stage_bytes(smem_raw, (const char*)A.nets + (size_t)(alpha * m.ntypes + beta) * NP::kBlockBytes,
                NP::kFwdBytes);
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
        env_row(m, A.xe, nl[k], xi, v);
        s = (T)v.s;
#pragma unroll
        for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
      }
      T t0[2][4], t1[4][4], t2[8][4];
      NP::fwd(smem_raw, s, g, rb, lane, t0, t1, t2);
      // reduce-scatter of the 128 products G[mt][q] R[c] over the 16 rows
      const bool b3 = rb & 8, b2 = rb & 4, b1 = rb & 2, b0 = rb & 1;
      T vv[64];
#pragma unroll
      for (int kk = 0; kk < 64; kk++) {
        int mt = kk >> 4, q = (kk >> 2) & 3, c = kk & 3;
        T a = g_at(t0, t1, t2, mt, q) * R[c];
        T b = g_at(t0, t1, t2, mt + 4, q) * R[c];
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
  // lane holds tile mt = 4 b3 + 2 b2 + b1, register q = 2 b0 + j / 4, c = j % 4
  const int mt = 4 * ((rb >> 3) & 1) + 2 * ((rb >> 2) & 1) + ((rb >> 1) & 1);
  T* Tout = (T*)A.T + (size_t)row * m.M * 4;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    int q = 2 * (rb & 1) + (j >> 2), c = j & 3;
    int p = 16 * mt + LP(g, q);
    int f = (p % kP0) < m.s0 ? (p / kP0) * m.s0 + (p % kP0) : -1;
    if (f >= 0) Tout[f * 4 + c] = acc[j] * (T)m.inv_norm;
  }
}

// ------------------------------------------------------------------------------------
// adjoint: forces and per-centre virial
// ------------------------------------------------------------------------------------
template <class NP, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_embed_bwd(EmbedArgs A) {
  typedef typename NP::Tv T;
  extern __shared__ __align__(16) char smem_raw[];
  T* gts = (T*)(smem_raw + NP::kBwdBytes + 256);   // per wave: dE/dT at positions [kP2][4]
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
  for (int beta = 0; beta < m.ntypes; beta++) {
    __syncthreads();
    stage_bytes(smem_raw, (const char*)A.nets + (size_t)(alpha * m.ntypes + beta) * NP::kBlockBytes,
                NP::kBwdBytes);
    __syncthreads();
    if (atom < 0) continue;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int k = c0 + rb;
      const bool valid = k < nn;
      Env v;
      int e = -1;
      T s = (T)0;
      T R[4] = {(T)0, (T)0, (T)0, (T)0};
      if (valid) {
        e = nl[k];
        env_row(m, A.xe, e, xi, v);
        s = (T)v.s;
#pragma unroll
        for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
      }
      T t0[2][4], t1[4][4], t2[8][4];
      NP::fwd(smem_raw, s, g, rb, lane, t0, t1, t2);
      // dE/dG (Eq. 4 adjoint) and the G.dE/dT part of dE/dR
      T gR[4] = {(T)0, (T)0, (T)0, (T)0};
      T res1[4][4];   // dE/dG[p] + dE/dG[p + 64]: the concat skip of the last layer
#pragma unroll
      for (int mt = 0; mt < 8; mt++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const T* gp = gt + (16 * mt + LP(g, q)) * 4;
          T G = g_at(t0, t1, t2, mt, q);
          T gG = (gp[0] * R[0] + gp[1] * R[1] + gp[2] * R[2] + gp[3] * R[3]) * inorm;
#pragma unroll
          for (int c = 0; c < 4; c++) gR[c] += G * gp[c];
          if (mt < 4) res1[mt][q] = gG;
          else res1[mt - 4][q] += gG;
          t2[mt][q] = gG * ((T)1 - t2[mt][q] * t2[mt][q]);  // becomes d(pre-activation)
        }
      // layer 2 adjoint: dh1 = res1 + W2 . d2; the concat skip of layer 1 passes the
      // undamped dh1 on (dh1[p] + dh1[p + 32]); then dh1 is damped by 1 - t1^2
      T dh1[4][4];
      NP::adj2(smem_raw, t2, g, rb, lane, dh1);
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int q = 0; q < 4; q++) dh1[nt][q] += res1[nt][q];
      T dh0[2][4];
#pragma unroll
      for (int nt = 0; nt < 2; nt++)
#pragma unroll
        for (int q = 0; q < 4; q++) dh0[nt][q] = dh1[nt][q] + dh1[nt + 2][q];
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int q = 0; q < 4; q++) dh1[nt][q] *= ((T)1 - t1[nt][q] * t1[nt][q]);
      // layer 1 adjoint: dh0 += W1 . d1
      {
        T w1d[2][4];
        NP::adj1(smem_raw, dh1, g, rb, lane, w1d);
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
#pragma unroll
          for (int q = 0; q < 4; q++) dh0[nt][q] += w1d[nt][q];
      }
      // layer 0: ds = sum_p dh0 (1 - t0^2) W0
      T dsl = (T)0;
#pragma unroll
      for (int nt = 0; nt < 2; nt++)
#pragma unroll
        for (int q = 0; q < 4; q++)
          dsl += dh0[nt][q] * ((T)1 - t0[nt][q] * t0[nt][q]) * NP::fpart(smem_raw)[kOffW0 + 16 * nt + LP(g, q)];
      // sum over the 4 lane groups holding the same row
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
        // g_b = sum_c dE/dR_c dR_c/dd_b (Eq. 5 differentiated)
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
  // reduce over the 16 rows (lanes 0..15 hold the sums; other lane groups hold zeros)
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

constexpr int kEmbWaves = 8;

static int embed_grid(int nrows) { return (nrows + kEmbWaves - 1) / kEmbWaves; }
int embed_bwd_blocks(int nrows) { return embed_grid(nrows); }

template <class NP>
static void embed_fwd_t(const EmbedArgs& a, hipStream_t st) {
  const size_t sh = NP::kFwdBytes;
  (void)hipFuncSetAttribute((const void*)k_embed_fwd<NP, kEmbWaves>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sh);
  hipLaunchKernelGGL((k_embed_fwd<NP, kEmbWaves>), dim3(embed_grid(a.nrows)), dim3(64 * kEmbWaves), sh, st, a);
}

template <class NP>
static void embed_bwd_t(const EmbedArgs& a, hipStream_t st) {
  const size_t sh = NP::kBwdBytes + 256 + sizeof(typename NP::Tv) * kEmbWaves * kP2 * 4;
  (void)hipFuncSetAttribute((const void*)k_embed_bwd<NP, kEmbWaves>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sh);
  hipLaunchKernelGGL((k_embed_bwd<NP, kEmbWaves>), dim3(embed_grid(a.nrows)), dim3(64 * kEmbWaves), sh, st, a);
}

void launch_embed_fwd(const EmbedArgs& a, hipStream_t st) {
  switch (a.prec) {
    case PREC_FP64: embed_fwd_t<NetNative<double>>(a, st); break;
    case PREC_FP32: embed_fwd_t<NetNative<float>>(a, st); break;
    case PREC_BF16: embed_fwd_t<NetBF16<1>>(a, st); break;
    default: embed_fwd_t<NetBF16<2>>(a, st); break;
  }
}

void launch_embed_bwd(const EmbedArgs& a, hipStream_t st) {
  switch (a.prec) {
    case PREC_FP64: embed_bwd_t<NetNative<double>>(a, st); break;
    case PREC_FP32: embed_bwd_t<NetNative<float>>(a, st); break;
    case PREC_BF16: embed_bwd_t<NetBF16<1>>(a, st); break;
    default: embed_bwd_t<NetBF16<2>>(a, st); break;
  }
}

}  // namespace dp
