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
// The operand precision is a policy of the kernels: native operands (NetNative: 16x16x4
// MFMA in T, FP64 or FP32) or BF16 operands (NetBF16: layer inputs rounded to BF16 on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, one k chunk of 32 positions per
// instruction, against weights pre-packed per lane; PARTS = 2 splits both operands into
// hi + lo BF16 and sums hi hi + hi lo + lo hi).  Everything outside the layer products
// (s, layer 0, biases, tanh, the skips, the contraction) stays in FP32 or FP64.  Student
// nets have kernels of their own (student_embed.hip).
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


template <class NP, class T>
__device__ __forceinline__ T chain_back(const char* sm, typename NP::State& st, T (&res1)[4][4], const T* fn,
                                        int g, int rb, int lane);

// The full chain receives dE/dG element by element: the concat skip of the last layer
// sums dE/dG[p] + dE/dG[p + 64] (res1), and t2 is overwritten by dE/dG (1 - t2^2), the
// gradient of layer 2's pre-activation.
template <class T>
__device__ __forceinline__ void chain_take_dG(T (&t2)[8][4], T (&res1)[4][4], int mt, int q, T gG) {
  if (mt < 4) res1[mt][q] = gG;
  else res1[mt - 4][q] += gG;
  t2[mt][q] = gG * ((T)1 - t2[mt][q] * t2[mt][q]);
}

// ------------------------------------------------------------------------------------
// net policies: State holds one chunk's activations; fwd() evaluates the net, G() reads
// G at (tile mt, register q), take_dG() receives dE/dG at (mt, q) once G there has been
// read, back() returns this lane's part of dE/ds (summed over the lane groups by the
// caller)
// ------------------------------------------------------------------------------------
template <class T>
struct NetNative {
  typedef T Tv;
  struct State {
    T t0[2][4], t1[4][4], t2[8][4];
  };
  struct Aux {
    T res1[4][4];
  };
  static constexpr int kFwdBytes = sizeof(T) * kNetElems;   // staged by the forward kernel
  static constexpr int kBwdBytes = sizeof(T) * kNetElems;   // staged by the adjoint kernel
  static constexpr int kBlockBytes = sizeof(T) * kNetElems; // stride of the net blocks
  __device__ static const char* block(const EmbedArgs& A, int pair) {
    return (const char*)A.nets + (size_t)pair * kBlockBytes;
  }
  __device__ static void fwd(const char* sm, T s, int g, int rb, int lane, State& st) {
    chain_fwd<T>((const T*)sm, s, g, rb, st.t0, st.t1, st.t2);
  }
  __device__ static T G(const State& st, int mt, int q) { return g_at(st.t0, st.t1, st.t2, mt, q); }
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
  __device__ static void take_dG(State& st, Aux& ax, int mt, int q, T gG) { chain_take_dG(st.t2, ax.res1, mt, q, gG); }
  __device__ static T back(const char* sm, State& st, Aux& ax, int g, int rb, int lane) {
    return chain_back<NetNative<T>, T>(sm, st, ax.res1, (const T*)sm, g, rb, lane);
  }
};

// Adjoint of the full chain (shared by both operand policies), after chain_take_dG:
// layer 2's adjoint on t2 (now d2), plus the concat skip res1; the concat skip of layer
// 1 passes the undamped dh1 on (dh1[p] + dh1[p + 32]); then dh1 is damped by 1 - t1^2;
// layer 1's adjoint; ds = sum_p dh0 (1 - t0^2) W0.  fn: the float / double part holding
// W0 at kOffW0.
template <class NP, class T>
__device__ __forceinline__ T chain_back(const char* sm, typename NP::State& st, T (&res1)[4][4], const T* fn,
                                        int g, int rb, int lane) {
  T dh1[4][4];
  NP::adj2(sm, st.t2, g, rb, lane, dh1);
  T dh0[2][4];
#pragma unroll
  for (int nt = 0; nt < 4; nt++)
#pragma unroll
    for (int q = 0; q < 4; q++) dh1[nt][q] += res1[nt][q];
#pragma unroll
  for (int nt = 0; nt < 2; nt++)
#pragma unroll
    for (int q = 0; q < 4; q++) dh0[nt][q] = dh1[nt][q] + dh1[nt + 2][q];
#pragma unroll
  for (int nt = 0; nt < 4; nt++)
#pragma unroll
    for (int q = 0; q < 4; q++) dh1[nt][q] *= ((T)1 - st.t1[nt][q] * st.t1[nt][q]);
  {
    T w1d[2][4];
    NP::adj1(sm, dh1, g, rb, lane, w1d);
#pragma unroll
    for (int nt = 0; nt < 2; nt++)
#pragma unroll
      for (int q = 0; q < 4; q++) dh0[nt][q] += w1d[nt][q];
  }
  T dsl = (T)0;
#pragma unroll
  for (int nt = 0; nt < 2; nt++)
#pragma unroll
    for (int q = 0; q < 4; q++)
      dsl += dh0[nt][q] * ((T)1 - st.t0[nt][q] * st.t0[nt][q]) * fn[kOffW0 + 16 * nt + LP(g, q)];
  return dsl;
}

// BF16 operands.  In the packed tiles, lane (g, rb) element j of k chunk kc stands for
// the position 16 (2 kc + j / 4) + 4 g + j % 4 of the layer input: exactly the value the
// lane holds in register j % 4 of tile 2 kc + j / 4, so a chunk of the B operand is two
// accumulator tiles rounded to BF16 in place.
template <int PARTS>
__device__ __forceinline__ bf8 bf_tile(const char* sm, int off, int part, int gs, int t, int lane) {
  return ((const bf8*)(sm + off + part * 2 * gs))[t * 64 + lane];
}
template <int PARTS, int NT>
__device__ __forceinline__ void bf_pack(const float (&v)[NT][4], int kc, bf8& hi, bf8& lo) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; j++) x[j] = v[2 * kc + j / 4][j % 4];
  split8<PARTS>(x, hi, lo);
}

template <int PARTS>
struct NetBF16 {
  typedef float Tv;
  typedef typename NetNative<float>::State State;
  typedef typename NetNative<float>::Aux Aux;
  static constexpr int kFloatBytes = 4 * kBFloat;
  static constexpr int kFwdBytes = kFloatBytes + PARTS * 2 * kBFwd;
  static constexpr int kBwdBytes = kFwdBytes + PARTS * 2 * kBBwd;
  static constexpr int kBlockBytes = 2 * bnet_u16(PARTS);
  __device__ static const char* block(const EmbedArgs& A, int pair) {
    return (const char*)A.nets + (size_t)pair * kBlockBytes;
  }
  __device__ static void fwd(const char* sm, float s, int g, int rb, int lane, State& st) {
    const float* fn = (const float*)sm;
    const int oF = kFloatBytes;
#pragma unroll
    for (int n = 0; n < 2; n++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int p = 16 * n + 4 * g + q;
        st.t0[n][q] = tanh_t(s * fn[kOffW0 + p] + fn[kOffB0 + p]);
      }
    bf8 xh, xl;
    bf_pack<PARTS, 2>(st.t0, 0, xh, xl);
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
      f4v c = {0, 0, 0, 0};
      bf8 wh = bf_tile<PARTS>(sm, oF, 0, kBFwd, mt, lane);
      bf8 wl = PARTS == 2 ? bf_tile<PARTS>(sm, oF, 1, kBFwd, mt, lane) : wh;
      c = mfma_split<PARTS>(wh, wl, xh, xl, c);
#pragma unroll
      for (int q = 0; q < 4; q++) st.t1[mt][q] = tanh_t(c[q] + fn[kOffB1 + 16 * mt + 4 * g + q]);
    }
    __builtin_amdgcn_sched_barrier(0);
    float h1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
      for (int q = 0; q < 4; q++) h1[mt][q] = st.t0[mt & 1][q] + st.t1[mt][q];
    bf8 hh[2], hl[2];
    bf_pack<PARTS, 4>(h1, 0, hh[0], hl[0]);
    bf_pack<PARTS, 4>(h1, 1, hh[1], hl[1]);
#pragma unroll
    for (int mt = 0; mt < 8; mt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 2; kc++) {
        bf8 wh = bf_tile<PARTS>(sm, oF + 2 * kBW1F, 0, kBFwd, 2 * mt + kc, lane);
        bf8 wl = PARTS == 2 ? bf_tile<PARTS>(sm, oF + 2 * kBW1F, 1, kBFwd, 2 * mt + kc, lane) : wh;
        c = mfma_split<PARTS>(wh, wl, hh[kc], hl[kc], c);
      }
#pragma unroll
      for (int q = 0; q < 4; q++) st.t2[mt][q] = tanh_t(c[q] + fn[kOffB2 + 16 * mt + 4 * g + q]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __device__ static float G(const State& st, int mt, int q) { return g_at(st.t0, st.t1, st.t2, mt, q); }
  __device__ static void adj2(const char* sm, const float (&d2)[8][4], int g, int rb, int lane,
                              float (&out)[4][4]) {
    const int oB = kFwdBytes + 2 * kBW1B;
    bf8 xh[4], xl[4];
#pragma unroll
    for (int kc = 0; kc < 4; kc++) bf_pack<PARTS, 8>(d2, kc, xh[kc], xl[kc]);
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 4; kc++) {
        bf8 wh = bf_tile<PARTS>(sm, oB, 0, kBBwd, 4 * nt + kc, lane);
        bf8 wl = PARTS == 2 ? bf_tile<PARTS>(sm, oB, 1, kBBwd, 4 * nt + kc, lane) : wh;
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
    for (int kc = 0; kc < 2; kc++) bf_pack<PARTS, 4>(d1, kc, xh[kc], xl[kc]);
#pragma unroll
    for (int nt = 0; nt < 2; nt++) {
      f4v c = {0, 0, 0, 0};
#pragma unroll
      for (int kc = 0; kc < 2; kc++) {
        bf8 wh = bf_tile<PARTS>(sm, oB, 0, kBBwd, 2 * nt + kc, lane);
        bf8 wl = PARTS == 2 ? bf_tile<PARTS>(sm, oB, 1, kBBwd, 2 * nt + kc, lane) : wh;
        c = mfma_split<PARTS>(wh, wl, xh[kc], xl[kc], c);
      }
#pragma unroll
      for (int q = 0; q < 4; q++) out[nt][q] = c[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ static void take_dG(State& st, Aux& ax, int mt, int q, float gG) {
    chain_take_dG(st.t2, ax.res1, mt, q, gG);
  }
  __device__ static float back(const char* sm, State& st, Aux& ax, int g, int rb, int lane) {
    return chain_back<NetBF16<PARTS>, float>(sm, st, ax.res1, (const float*)sm, g, rb, lane);
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
  // FP32: each lane sums G R over its own rows of every chunk and the 16-row reduction
  // runs once per centre; FP64 (register budget) reduces per chunk
  constexpr bool kLaneAcc = sizeof(T) == 4;
  T acc[8];
#pragma unroll
  for (int j = 0; j < 8; j++) acc[j] = (T)0;
  T part[kLaneAcc ? 128 : 1];
#pragma unroll
  for (int j = 0; j < (kLaneAcc ? 128 : 1); j++) part[j] = (T)0;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_bytes(smem_raw, NP::block(A, pair), NP::kFwdBytes);
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
        const int e = nl[k];
        env_row(m, A.xe, e, xi, v);
        s = (T)v.s;
#pragma unroll
        for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
      }
      typename NP::State st;
      NP::fwd(smem_raw, s, g, rb, lane, st);
      if constexpr (kLaneAcc) {
        // per-lane partial sums over this lane's rows of all chunks
#pragma unroll
        for (int kk = 0; kk < 128; kk++) {
          int mt = kk >> 4, q = (kk >> 2) & 3, c = kk & 3;
          part[kk] += NP::G(st, mt, q) * R[c];
        }
      } else {
        // reduce-scatter of the 128 products G[mt][q] R[c] over the 16 rows
        const bool b3 = rb & 8, b2 = rb & 4, b1 = rb & 2, b0 = rb & 1;
        T vv[64];
#pragma unroll
        for (int kk = 0; kk < 64; kk++) {
          int mt = kk >> 4, q = (kk >> 2) & 3, c = kk & 3;
          T a = NP::G(st, mt, q) * R[c];
          T b = NP::G(st, mt + 4, q) * R[c];
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
  }
  if constexpr (kLaneAcc) {
    // one reduce-scatter of the lane partials over the 16 rows of the wave
    const bool b3 = rb & 8, b2 = rb & 4, b1 = rb & 2, b0 = rb & 1;
    T vv[64];
#pragma unroll
    for (int kk = 0; kk < 64; kk++) {
      T a = part[kk], b = part[kk + 64];
      T send = b3 ? a : b;
      T keep = b3 ? b : a;
      vv[kk] = keep + dpp_mov<DPP_ROR8>(send);
    }
    rs_step<T, 64, DPP_HALF_MIRROR>(vv, b2);
    rs_step<T, 32, DPP_XOR2>(vv, b1);
    rs_step<T, 16, DPP_XOR1>(vv, b0);
#pragma unroll
    for (int j = 0; j < 8; j++) acc[j] = vv[j];
  }
  if (atom < 0) return;
  write_T<T>((T*)A.T + (size_t)row * m.M * 4, acc, rb, g, m.s0, (T)m.inv_norm);
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
  double fi = 0;                  // force component g on the centre (lane groups 0..2)
  double vir[3] = {0, 0, 0};      // virial column g: W[a][g]
  const T inorm = (T)m.inv_norm;
  constexpr bool kMfmaGG = sizeof(T) == 4;
  T ga[kMfmaGG ? 8 : 1];   // MFMA A operand of dE/dG: dE/dT[16 mt + rb][g] / N_m
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    __syncthreads();
    stage_bytes(smem_raw, NP::block(A, pair), NP::kBwdBytes);
    __syncthreads();
    if (atom < 0) continue;
    if (kMfmaGG && beta == 0)
#pragma unroll
      for (int mt = 0; mt < (kMfmaGG ? 8 : 1); mt++) ga[mt] = gt[(16 * mt + rb) * 4 + g] * inorm;
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
        s = (T)v.s;
#pragma unroll
        for (int c = 0; c < 4; c++) R[c] = (T)v.R[c];
      }
      typename NP::State st;
      NP::fwd(smem_raw, s, g, rb, lane, st);
      // dE/dG (Eq. 4 adjoint) and the G.dE/dT part of dE/dR.  dE/dG[p][row] =
      // sum_c (dE/dT[p][c] / N_m) R[row][c] is one 16x16x4 MFMA per position tile: A =
      // dE/dT of the tile (lane (g, i) holds position 16 mt + i, component g), B = R
      // (lane (g, row) holds component g of its row); the result lands in the layout
      // of G itself.  (FP64 keeps the VALU form: its register budget has no room for
      // the operand.)
      T gR[4] = {(T)0, (T)0, (T)0, (T)0};
      typename NP::Aux ax;
      const T Rg = g == 0 ? R[0] : g == 1 ? R[1] : g == 2 ? R[2] : R[3];
#pragma unroll
      for (int mt = 0; mt < 8; mt++) {
        typename Acc4<T>::type gGt = {0, 0, 0, 0};
        if constexpr (kMfmaGG) gGt = mfma4(ga[mt], Rg, gGt);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const T* gp = gt + (16 * mt + LP(g, q)) * 4;
          const T G = NP::G(st, mt, q);
#pragma unroll
          for (int c = 0; c < 4; c++) gR[c] += G * gp[c];
          T gG;
          if constexpr (kMfmaGG) gG = gGt[q];
          else gG = (gp[0] * R[0] + gp[1] * R[1] + gp[2] * R[2] + gp[3] * R[3]) * inorm;
          NP::take_dG(st, ax, mt, q, gG);
        }
      }
      T dsl = NP::back(smem_raw, st, ax, g, rb, lane);
      // sum over the 4 lane groups holding the same row
      dsl += shfl_x(dsl, 16);
      dsl += shfl_x(dsl, 32);
#pragma unroll
      for (int c = 0; c < 4; c++) {
        gR[c] += shfl_x(gR[c], 16);
        gR[c] += shfl_x(gR[c], 32);
      }
      // g_ij = dR^T dE/dR (Eq. 5 differentiated): lane group g < 3 computes component g
      if (valid && g < 3) {
        double gRd[4] = {(double)gR[0] * m.inv_norm + (double)dsl, (double)gR[1] * m.inv_norm,
                         (double)gR[2] * m.inv_norm, (double)gR[3] * m.inv_norm};
        double ir = v.ir;
        double sr = v.s * ir;
        double qf = (v.ds * ir - v.s * ir * ir) * ir;
        double dot = gRd[1] * v.d[0] + gRd[2] * v.d[1] + gRd[3] * v.d[2];
        const double db = g == 0 ? v.d[0] : g == 1 ? v.d[1] : v.d[2];
        const double gRb = g == 0 ? gRd[1] : g == 1 ? gRd[2] : gRd[3];
        const double gv = gRd[0] * v.ds * db * ir + qf * dot * db + sr * gRb;
        fi += gv;
        if (A.gbuf) A.gbuf[((size_t)atom * m.nm + m.sel_off[beta] + k) * 3 + g] = gv;
        else unsafeAtomicAdd(&A.forces[3 * A.eown[e] + g], -gv);
#pragma unroll
        for (int a = 0; a < 3; a++) vir[a] -= v.d[a] * gv;   // W[a][g]
      }
    }
  }
  if (atom < 0) return;
  // reduce over the 16 rows of each lane group (group g < 3 holds component g)
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    fi += __shfl_xor(fi, o);
#pragma unroll
    for (int a = 0; a < 3; a++) vir[a] += __shfl_xor(vir[a], o);
  }
  if (rb == 0 && g < 3) {
    if (A.gbuf) A.forces[3 * atom + g] = fi;   // the -g_ij of other centres are gathered later
    else unsafeAtomicAdd(&A.forces[3 * atom + g], fi);
#pragma unroll
    for (int a = 0; a < 3; a++) A.vir_part[(size_t)row * 9 + 3 * a + g] = vir[a];
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
