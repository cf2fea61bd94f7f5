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
// One wave per centre; each neighbour's environment row is formed once, by one lane, and
// handed to the other lanes through LDS.  The forward runs four independent waves per
// block; lane (k, p) applies hidden unit k = lane % 32 to the rows of parity p = lane / 32,
// so S accumulates inside the lane, and the W2 [k][f] product reads the student blocks (a
// few KB per pair, cache-resident) straight from global memory.  The adjoint runs eight
// centres per block: lane (rb, g) (rb = lane % 16, g = lane / 16) takes neighbour rb of
// each chunk of 16 and the hidden units k = 16 n + 4 g + q (n < 2, q < 4), its per-row sums
// over k closing over the four lane groups; the centres' V products are one small matrix
// product on the MFMA with W2T [f][k] staged in LDS, and each wave pipelines the gathers
// of its neighbour blocks across both species of a pass.
#include <hip/hip_runtime.h>

#include "embed_common.h"

namespace dp {

constexpr int kStuWaves = 4;
#define GAS_T(T) __attribute__((address_space(1))) T
constexpr int kStuS = 37 * 8;   // per wave: S rows k < 32 then rbar (stride 4), or V rows with W1, b1 then u
// V row k of the adjoint (6 words used) at vrow(k): stride 8, skewed by 4 per group of four
// rows so that the four lane groups (rows 4 g + r) read different LDS banks, and by 16
// more for k >= 16 so that the skewed rows never overlap (row 15 ends at 138, row 16
// starts at 144; row 31 ends at 282)
__device__ __forceinline__ int vrow(int k) { return 8 * k + 4 * ((k >> 2) & 3) + 16 * (k >> 4); }
constexpr int kStuU = 284;   // u after the 32 skewed V rows
constexpr int kW2Pad = 32;           // the second staged W2T starts 32 words later (other banks)

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

// one reduce-scatter step over an array of N values: the lane whose "up" bit is set keeps
// the upper half, its DPP partner (bit clear) the lower half, each adding the partner's copy
template <class T, int N, int CTRL>
__device__ __forceinline__ void stu_rs_step(T (&v)[32], bool up) {
#pragma unroll
  for (int k = 0; k < N / 2; k++) {
    const T a = v[k], b = v[k + N / 2];
    const T send = up ? a : b;
    const T keep = up ? b : a;
    v[k] = keep + row_rot<CTRL>(send);
  }
}

// value of lane src (any lane of the wave)
__device__ __forceinline__ float wave_shfl(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double wave_shfl(double v, int src) { return __shfl(v, src, 64); }

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

__device__ __forceinline__ bool stu_out_of_range(double lo, double hi, double s) { return s < lo || s > hi; }

// Environment row of one neighbour (Eq. 5) in FP64 whatever the student's storage type:
// displacement, r, 1/r, the switch s(r) and its derivative, R~ and the force geometry
// stay FP64 (the precision contract of every mode); only s and R~ are rounded to the
// student's type for the tanh layer and the per-centre products.
// The switch is written through om = (rc - r) / (rc - rcs) = 1 - u: the same quintic as
// the full net's, w = om^3 (6 u^2 + 3 u + 1), dw/dr = -30 u^2 om^2 / (rc - rcs), which keeps
// its relative precision (and its sign) as w -> 0 at the cutoff, where the expanded form
// 1 + u^3 (-6 u^2 + 15 u - 10) cancels to a few ulps of 1, possibly below zero; s then
// never leaves a trained range that starts at 0.
struct StuEnv {
  double d[3], ir, s, ds, R[4];
};
__device__ __forceinline__ void stu_env(const ModelC& m, const double xj[3], const double xi[3], StuEnv& v) {
  v.d[0] = xj[0] - xi[0];
  v.d[1] = xj[1] - xi[1];
  v.d[2] = xj[2] - xi[2];
  const double r2 = v.d[0] * v.d[0] + v.d[1] * v.d[1] + v.d[2] * v.d[2];
  const double r = sqrt(r2);
  v.ir = 1.0 / r;
  double w = 0.0, dw = 0.0;
  if (r < m.rcs) {
    w = 1.0;
  } else if (r < m.rc) {
    const double om = (m.rc - r) * m.inv_h, u = 1.0 - om;
    if (m.switch_kind == 1) {
      double sp, cp;
      sincos(M_PI * om, &sp, &cp);   // cos(pi u) = -cos(pi (1 - u)), sin(pi u) = sin(pi (1 - u))
      w = 0.5 - 0.5 * cp;
      dw = -0.5 * M_PI * sp * m.inv_h;
    } else {
      w = om * om * om * (6.0 * u * u + 3.0 * u + 1.0);
      dw = -30.0 * u * u * om * om * m.inv_h;
    }
  }
  v.s = w * v.ir;
  v.ds = (dw - w * v.ir) * v.ir;
  const double sr = v.s * v.ir;
  v.R[0] = v.s;
  v.R[1] = sr * v.d[0];
  v.R[2] = sr * v.d[1];
  v.R[3] = sr * v.d[2];
}

// Software pipeline of the neighbour gathers: the list entry of a chunk is loaded two
// chunks before its use and the coordinates one chunk before, so that no gather waits
// on the list load issued just before it.
// Both loads are unconditional (the slot index clamped into the species block of width
// sel, a -1 entry read as atom 0) so that every lane and path issues the same loads and
// the waits can count down to the older gather only.
__device__ __forceinline__ int stu_index(const int* __restrict__ nl, int k, int nn, int sel) {
  const int v = nl[k < sel ? k : (sel > 0 ? sel - 1 : 0)];
  return k < nn ? v : -1;
}
__device__ __forceinline__ void stu_coords(const double* __restrict__ xe, int e, double (&x)[3]) {
  const int q = e > 0 ? e : 0;
  x[0] = xe[3 * q];
  x[1] = xe[3 * q + 1];
  x[2] = xe[3 * q + 2];
}
// the coordinates and the owner (the atom that receives the neighbour's force)
__device__ __forceinline__ void stu_coords_owner(const double* __restrict__ xe, const int* __restrict__ eown, int e,
                                                 double (&x)[3], int& own) {
  const int q = e > 0 ? e : 0;
  x[0] = xe[3 * q];
  x[1] = xe[3 * q + 1];
  x[2] = xe[3 * q + 2];
  own = eown[q];
}

// student block of a pair, read through global (not generic) pointers
template <class T>
__device__ __forceinline__ const GAS_T(T)* stu_block(const EmbedArgs& A, int pair) {
  return (const GAS_T(T)*)((const T*)A.snets + (size_t)pair * kStuElems);
}

// ------------------------------------------------------------------------------------
// forward: T of each centre
// ------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(64 * kStuWaves) void k_stu_fwd(EmbedArgs A) {
  __shared__ __align__(16) T s_w[kStuWaves][kStuS];
  __shared__ __align__(16) T s_env[kStuWaves][64 * 8];   // per wave: 64 rows [R~ (4), s, pad]
  typedef T t4v __attribute__((ext_vector_type(4)));
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* Sw = s_w[wv];                                     // this wave's S and rbar
  T* Ew = s_env[wv];
  const int row = blockIdx.x * kStuWaves + wv;
  if (row >= A.nrows) return;
  const int alpha = species_of(row, m.ntypes, A.type_row0);
  const int atom = A.row_atom[row];
  if (alpha < 0 || atom < 0) return;   // padding row (uniform over the wave)
  const double xi[3] = {A.xe[3 * atom], A.xe[3 * atom + 1], A.xe[3 * atom + 2]};
  T tacc[2][4];   // T at features lane and lane + 64 (unscaled)
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int c = 0; c < 4; c++) tacc[i][c] = (T)0;
  for (int beta = 0; beta < m.ntypes; beta++) {
    const int pair = alpha * m.ntypes + beta;
    const auto sn = stu_block<T>(A, pair);
    const double slo = A.st_lo[pair], shi = A.st_hi[pair];
    // lane (k, p): hidden unit k = lane % 32 over the rows of parity p = lane / 32, so
    // that S[k][c] = sum over rows of h_k R~_c accumulates inside the lane (the two row
    // parities are added at the end) and no reduction over lanes is needed
    const int hk = lane & 31, hp = lane >> 5;
    const T w1 = sn[kSW1 + hk], b1 = sn[kSB1 + hk];
    T Sp[4] = {(T)0, (T)0, (T)0, (T)0}, rs[4] = {(T)0, (T)0, (T)0, (T)0};
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    // Environment rows 64 at a time, one neighbour per lane (c0 + lane), published in the
    // wave's LDS rows [R~ (4), s]; then every lane reads the rows of its parity (the same
    // row across a half wave: broadcast reads) and applies its hidden unit
    const int sel = m.sel[beta];
    double xn[3] = {0, 0, 0};
    int en = stu_index(nl, lane, nn, sel);   // the next 64 neighbours, fetched a pass ahead
    stu_coords(A.xe, en, xn);
    for (int c0 = 0; c0 < nn; c0 += 64) {
      const int e = en;
      const double xj[3] = {xn[0], xn[1], xn[2]};
      en = stu_index(nl, c0 + 64 + lane, nn, sel);
      stu_coords(A.xe, en, xn);
      T sL = (T)0, RL[4] = {(T)0, (T)0, (T)0, (T)0};
      if (e >= 0) {
        StuEnv v;
        stu_env(m, xj, xi, v);
        if (stu_out_of_range(slo, shi, v.s)) {
          // left to the full net (fallback list); contributes nothing here
          const int p = atomicAdd(A.fb_count, 1);
          if (p < A.fb_cap) A.fb_list[p] = make_int2(row, e);
        } else {
          sL = (T)v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) RL[c] = (T)v.R[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 4; c++) rs[c] += RL[c];
      wave_sync_lds();   // the previous block's rows have been read
      *(t4v*)(Ew + 8 * lane) = t4v{RL[0], RL[1], RL[2], RL[3]};
      Ew[8 * lane + 4] = sL;
      wave_sync_lds();
      const int half = (min(64, nn - c0) + 1) >> 1;   // row pairs holding a neighbour
#pragma unroll 4
      for (int i = 0; i < half; i++) {
        const T* E = Ew + 8 * (2 * i + hp);
        const t4v R = *(const t4v*)E;
        const T h = tanh_t(E[4] * w1 + b1);
#pragma unroll
        for (int c = 0; c < 4; c++) Sp[c] += h * R[c];
      }
    }
    // S[k][c] = both parities' sums; rbar = sum of R~ over the 64 lanes
#pragma unroll
    for (int c = 0; c < 4; c++) {
      Sp[c] += wave_shfl(Sp[c], lane ^ 32);
      rs[c] = sum_g(row_sum16(rs[c]));
    }
    if (hp == 0)
#pragma unroll
      for (int c = 0; c < 4; c++) Sw[hk * 4 + c] = Sp[c];
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < 4; c++) Sw[32 * 4 + c] = rs[c];
    wave_sync_lds();
    // T += W2^T S + b2 rbar^T at this lane's two features (W2 rows read 64 wide)
    const bool two = lane + 64 < kP2;
#pragma unroll 8
    for (int kk = 0; kk < 32; kk++) {
      T s4[4];
#pragma unroll
      for (int c = 0; c < 4; c++) s4[c] = Sw[kk * 4 + c];
      const T wa = sn[kSW2 + kk * kP2 + lane], wb = two ? sn[kSW2 + kk * kP2 + lane + 64] : (T)0;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        tacc[0][c] += wa * s4[c];
        tacc[1][c] += wb * s4[c];
      }
    }
    const T ba = sn[kSB2 + lane], bb = two ? sn[kSB2 + lane + 64] : (T)0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      tacc[0][c] += ba * Sw[32 * 4 + c];
      tacc[1][c] += bb * Sw[32 * 4 + c];
    }
    wave_sync_lds();   // Sw is rewritten by the next pair
  }
  T* Tout = (T*)A.T + (size_t)row * m.M * 4;
  const T scale = (T)m.inv_norm;
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const int f = lane + 64 * i;
    if (f < m.M)
#pragma unroll
      for (int c = 0; c < 4; c++) Tout[f * 4 + c] = tacc[i][c] * scale;
  }
}

// ------------------------------------------------------------------------------------
// adjoint: forces (scattered with atomics to the neighbours' owners) and per-centre virial
// ------------------------------------------------------------------------------------
constexpr int kStuBwdWaves = 8;

// LDS of the adjoint: W2T of two pairs, then per wave V rows (with W1, b1) and u of two,
// then per wave the centre's dE/dT [kP2][4], then per wave s and R~ of the 64 neighbours
// in flight (the same rows then carry their three FP64 force components: at least 24
// bytes per lane)
constexpr int kEnvStride = 6;

size_t stu_bwd_lds_bytes(int elem) {
  return (size_t)elem * (2 * kP2 * kP0 + kW2Pad + kStuBwdWaves * (2 * kStuS + kP2 * 4 + 64 * kEnvStride));
}

template <class T>
__global__ __launch_bounds__(64 * kStuBwdWaves) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_stu_bwd(EmbedArgs A) {
  extern __shared__ __align__(16) char smem[];
  T* w2s = (T*)smem;                                   // W2T of the pass's two pairs [2][kP2][kP0]
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  T* Vall0 = w2s + 2 * kP2 * kP0 + kW2Pad;                     // per wave, per pair of the pass: V rows with W1, b1, then u
  T* Vall = Vall0 + wv * 2 * kStuS;
  const int r0 = blockIdx.x * kStuBwdWaves;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;   // uniform over the block (rows of one species: groups are padded to 64)
  const int row = __builtin_amdgcn_readfirstlane(r0 + wv);
  const int atom = row < A.nrows ? A.row_atom[row] : -1;
  const bool live = atom >= 0;   // padding rows still take part in the block's barriers
  const int M = m.M;
  double xi[3] = {0, 0, 0};
  if (live) {
    xi[0] = A.xe[3 * atom];
    xi[1] = A.xe[3 * atom + 1];
    xi[2] = A.xe[3 * atom + 2];
  }
  // dE/dT of this centre [f][4]: one coalesced load into registers (feature lane and
  // lane + 64), copied to the wave's LDS rows for the broadcast reads of the V product
  T* gts0 = w2s + 2 * kP2 * kP0 + kW2Pad + kStuBwdWaves * 2 * kStuS;
  T* gts = gts0 + wv * kP2 * 4;
  typedef T t4v __attribute__((ext_vector_type(4)));
  t4v gtv[2];
  {
    const t4v* src = (const t4v*)((const T*)A.gT + (size_t)(live ? row : 0) * M * 4);
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const int f = lane + 64 * i;
      gtv[i] = (live && f < M) ? src[f] : t4v{(T)0, (T)0, (T)0, (T)0};
      if (f < kP2) *(t4v*)(gts + 4 * f) = gtv[i];
    }
  }
  double fi[3] = {0.0, 0.0, 0.0};     // this lane's part of the force on the centre
  double vir[3][3] = {};              // and of the centre's virial W[a][b]
  T* envw = w2s + 2 * kP2 * kP0 + kW2Pad + kStuBwdWaves * (2 * kStuS + kP2 * 4) + wv * 64 * kEnvStride;
  const T inorm = (T)m.inv_norm;
  for (int b0 = 0; b0 < m.ntypes; b0 += 2) {
    const int nb = min(2, m.ntypes - b0);
    // The pass's neighbour blocks of 64, (pair q, start c0) flattened over both pairs, run
    // as one software pipeline: list entries two blocks ahead, coordinates and owners one
    // block ahead, so that the first blocks' gathers overlap the V product and the
    // barriers.  Block (q, c0) exists for c0 < nn_q; "q = 2" is the end (a dummy list
    // row with nn = 0, whose loads stay in bounds).
    const int* nlrow = A.nlist + (size_t)(live ? atom : 0) * m.nm;
    const int nnq0 = live ? A.nnei[atom * m.ntypes + b0] : 0;
    const int nnq1 = live && nb > 1 ? A.nnei[atom * m.ntypes + b0 + 1] : 0;
    auto nnq = [&](int q) { return q == 0 ? nnq0 : q == 1 ? nnq1 : 0; };
    auto norm = [&](int& q, int& c) {
      while (q < 2 && c >= nnq(q)) {
        q++;
        c = 0;
      }
    };
    auto blk_index = [&](int q, int c) {
      const int qq = q < 2 ? q : 0;
      return stu_index(nlrow + m.sel_off[b0 + (qq < nb ? qq : 0)], c + lane, nnq(q), m.sel[b0 + (qq < nb ? qq : 0)]);
    };
    int q1 = 0, c1 = 0;
    norm(q1, c1);
    int q2 = q1, c2 = c1 + 64;
    norm(q2, c2);
    int en = blk_index(q1, c1), en2 = blk_index(q2, c2);
    __syncthreads();   // the previous pass's W2T is no longer read
    for (int q = 0; q < nb; q++)
      stage_bytes(w2s + q * (kP2 * kP0 + kW2Pad), (const T*)A.snets + (size_t)(alpha * m.ntypes + b0 + q) * kStuElems + kSW2T,
                  (int)sizeof(T) * kP2 * kP0);
    __syncthreads();
    double xn[3];
    int own_n;
    stu_coords_owner(A.xe, A.eown, en, xn, own_n);
    // V_beta[k][(w, c)] = sum_f W2[k][f] gt_w[f][c] for the block's eight centres w on the
    // MFMA (16x16x4): wave wv takes the output tile of pair q = wv / 4, hidden units
    // 16 kt .. 16 kt + 15 (kt = (wv / 2) % 2) and centres 4 nt .. 4 nt + 3 (nt = wv % 2),
    // four components each; A = W2T rows f (staged above), B = the centres' dE/dT rows
    // (zero at f >= M, so the last k step may run past M)
    {
      const int q = wv >> 2, kt = (wv >> 1) & 1, nt = wv & 1;
      if (q < nb) {
        const int wsrc = 4 * nt + (rb >> 2), c = rb & 3;
        const T* Aw = w2s + q * (kP2 * kP0 + kW2Pad) + 16 * kt + rb;
        const T* Bw = gts0 + wsrc * kP2 * 4 + c;
        typedef T acc4 __attribute__((ext_vector_type(4)));
        acc4 acc = {(T)0, (T)0, (T)0, (T)0};
        for (int f0 = 0; f0 < M; f0 += 4) {
          const int f = f0 + g;
          acc = mfma4(Aw[f * kP0], Bw[4 * f], acc);
        }
        T* Vb = Vall0 + wsrc * 2 * kStuS + q * kStuS;
#pragma unroll
        for (int r = 0; r < 4; r++) Vb[vrow(16 * kt + lpos(T(), g, r)) + c] = acc[r];
      }
    }
    // W1 and b1 beside each V row of the wave's own centre, and u_beta[c] = sum_f b2_beta[f] gt[f][c]
    {
      const int hb = lane >> 5, kk = lane & 31;
      if (hb < nb) {
        const auto sn = stu_block<T>(A, alpha * m.ntypes + b0 + hb);
        T* Vb = Vall + hb * kStuS;
        Vb[vrow(kk) + 4] = sn[kSW1 + kk];
        Vb[vrow(kk) + 5] = sn[kSB1 + kk];
      }
      for (int q = 0; q < nb; q++) {
        const auto sn = stu_block<T>(A, alpha * m.ntypes + b0 + q);
        const int f1 = lane + 64;
        const T bl = lane < M ? sn[kSB2 + lane] : (T)0, bh = f1 < M ? sn[kSB2 + f1] : (T)0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
          T u = bl * gtv[0][c] + bh * gtv[1][c];
          u = sum_g(row_sum16(u));
          if (lane == 0) Vall[q * kStuS + kStuU + c] = u;
        }
      }
    }
    __syncthreads();   // every centre's V rows are complete
    if (!live) continue;
    const double slo0 = A.st_lo[alpha * m.ntypes + b0], shi0 = A.st_hi[alpha * m.ntypes + b0];
    const double slo1 = nb > 1 ? A.st_lo[alpha * m.ntypes + b0 + 1] : 0.0;
    const double shi1 = nb > 1 ? A.st_hi[alpha * m.ntypes + b0 + 1] : 0.0;
    // Each block: lane L forms the FP64 environment row of neighbour c0 + L once and
    // publishes s and R~ (the student's type) in the wave's LDS rows; then in chunks of 16
    // lane (rb, g) takes neighbour rb of the chunk and the hidden units of lane group g.
    // The sums over the lane groups land in every group; lane group q keeps those of
    // chunk q, which are its own neighbours', and assembles their forces.
    while (q1 < 2) {
      const int q = q1, c0 = c1, nn = nnq(q);
      const int e = en, own = own_n;
      const double xj[3] = {xn[0], xn[1], xn[2]};
      int q3 = q2, c3 = c2 + 64;
      norm(q3, c3);
      en = en2;
      en2 = blk_index(q3, c3);
      stu_coords_owner(A.xe, A.eown, en, xn, own_n);
      q1 = q2;
      c1 = c2;
      q2 = q3;
      c2 = c3;
      // V, W1 and b1 of the lane's hidden units are read from LDS inside the chunk loop
      // (held in registers they would cost 48 VGPRs and lower the waves per SIMD)
      const T* Vw = Vall + q * kStuS;
      const double slo = q == 0 ? slo0 : slo1, shi = q == 0 ? shi0 : shi1;
      T uu[4];
#pragma unroll
      for (int c = 0; c < 4; c++) uu[c] = Vw[kStuU + c];
      bool valid = e >= 0;
      StuEnv v;
      T sL = (T)0, RL[4] = {(T)0, (T)0, (T)0, (T)0};
      if (valid) {
        stu_env(m, xj, xi, v);
        if (stu_out_of_range(slo, shi, v.s)) {
          valid = false;   // handled by the fallback kernel
        } else {
          sL = (T)v.s;
#pragma unroll
          for (int c = 0; c < 4; c++) RL[c] = (T)v.R[c];
        }
      }
      wave_sync_lds();   // the previous block's rows have been read
      envw[kEnvStride * lane] = sL;
#pragma unroll
      for (int c = 0; c < 4; c++) envw[kEnvStride * lane + 1 + c] = RL[c];
      wave_sync_lds();
      // gR[c] = sum_p G[p] gt[p][c] = h . V[:, c] + u[c];  dsl = dE/ds through G
      T gRo[4] = {(T)0, (T)0, (T)0, (T)0}, dslo = (T)0;
#pragma unroll
      for (int qc = 0; qc < 4; qc++) {
        if (c0 + 16 * qc >= nn) break;   // uniform over the wave
        const T* E = envw + kEnvStride * (16 * qc + rb);
        const T s = E[0], R[4] = {E[1], E[2], E[3], E[4]};
        T gR[4] = {(T)0, (T)0, (T)0, (T)0}, dsp = (T)0;
        int zo = 0;
        asm volatile("" : "+s"(zo));   // keeps the V loads inside the loop (not hoisted into registers)
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const T* P = Vw + zo + vrow(16 * (j >> 2) + 4 * g + (j & 3));
          const T vk[4] = {P[0], P[1], P[2], P[3]}, w1 = P[4], b1 = P[5];
          const T h = tanh_t(s * w1 + b1);
          T dh = (T)0;
#pragma unroll
          for (int c = 0; c < 4; c++) {
            gR[c] += h * vk[c];
            dh += vk[c] * R[c];
          }
          dsp += dh * ((T)1 - h * h) * w1;
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
          gR[c] = sum_g(gR[c]) + uu[c];
          gRo[c] = g == qc ? gR[c] : gRo[c];
        }
        const T dsl = sum_g(dsp) * inorm;   // dE/ds through G, in the student's type
        dslo = g == qc ? dsl : dslo;
      }
      // g_ij = dR^T dE/dR (Eq. 5 differentiated) in FP64 from the lane's environment row
      // and dE/dR~ (the student's sums): g_b = d_b (dE/dR0 ds/r + qf d.dE/dR) + (s/r) dE/dR_b
      double gv[3] = {0.0, 0.0, 0.0};
      if (valid) {
        const double in = m.inv_norm;
        const double gRd[4] = {(double)gRo[0] * in + (double)dslo, (double)gRo[1] * in, (double)gRo[2] * in,
                               (double)gRo[3] * in};
        const double ir = v.ir;
        const double sr = v.s * ir;
        const double qf = (v.ds * ir - v.s * ir * ir) * ir;
        const double dot = gRd[1] * v.d[0] + gRd[2] * v.d[1] + gRd[3] * v.d[2];
        const double cf = gRd[0] * v.ds * ir + qf * dot;
#pragma unroll
        for (int b = 0; b < 3; b++) {
          gv[b] = cf * v.d[b] + sr * gRd[b + 1];
          fi[b] += gv[b];
#pragma unroll
          for (int a = 0; a < 3; a++) vir[a][b] -= v.d[a] * gv[b];   // W[a][b]
        }
      }
      // the neighbours' forces go out through the LDS rows in the chunk layout, lane
      // (rb, g < 3) adding component g of neighbour rb: one atomic instruction per chunk
      // covers 16 neighbours with their three components side by side (one L2 line each)
      wave_sync_lds();   // the chunks' reads of s and R~ are done
      double* gvw = (double*)envw;
#pragma unroll
      for (int b = 0; b < 3; b++) gvw[3 * lane + b] = gv[b];
      wave_sync_lds();
      const int ownv = valid ? own : -1;
#pragma unroll
      for (int qc = 0; qc < 4; qc++) {
        if (c0 + 16 * qc >= nn) break;   // uniform over the wave
        const int o = __shfl(ownv, 16 * qc + rb, 64);
        const double f = gvw[3 * (16 * qc + rb) + (g < 3 ? g : 0)];
        if (g < 3 && o >= 0) unsafeAtomicAdd(&A.forces[3 * o + g], -f);
      }
    }
    wave_sync_lds();   // the V rows are rewritten in the next pass
  }
  if (!live) return;
  // sums over the wave of the 12 values f = b (force component b on the centre) and
  // f = 3 + 3 a + b (virial W[a][b]): a reduce-scatter inside each 16-lane row (partners
  // xor 8, 7, 2, 1 keep the half of the values their bit selects) leaves lane rb with the
  // row's sum of value rb; the four rows are then added
  double v[32];
#pragma unroll
  for (int b = 0; b < 3; b++) v[b] = fi[b];
#pragma unroll
  for (int k = 0; k < 9; k++) v[3 + k] = vir[k / 3][k % 3];
#pragma unroll
  for (int k = 12; k < 16; k++) v[k] = 0.0;
  stu_rs_step<double, 16, DPP_ROR8>(v, (rb & 8) != 0);
  stu_rs_step<double, 8, DPP_HALF_MIRROR>(v, (rb & 4) != 0);
  stu_rs_step<double, 4, DPP_XOR2>(v, (rb & 2) != 0);
  stu_rs_step<double, 2, DPP_XOR1>(v, (rb & 1) != 0);
  const double t = sum_g(v[0]);
  if (lane < 3) unsafeAtomicAdd(&A.forces[3 * atom + lane], t);
  else if (lane < 12) A.vir_part[(size_t)row * 9 + lane - 3] = t;
}

template <class T>
static void stu_fwd_t(const EmbedArgs& a, hipStream_t st) {
  const int grid = (a.nrows + kStuWaves - 1) / kStuWaves;
  if (grid > 0) hipLaunchKernelGGL(k_stu_fwd<T>, dim3(grid), dim3(64 * kStuWaves), 0, st, a);
}

template <class T>
static void stu_bwd_t(const EmbedArgs& a, hipStream_t st) {
  const int grid = (a.nrows + kStuBwdWaves - 1) / kStuBwdWaves;
  const size_t sh = stu_bwd_lds_bytes(sizeof(T));
  (void)hipFuncSetAttribute((const void*)k_stu_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (grid > 0) hipLaunchKernelGGL(k_stu_bwd<T>, dim3(grid), dim3(64 * kStuBwdWaves), sh, st, a);
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
