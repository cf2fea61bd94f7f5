// Fused embedding-net passes of the parameter gradient (training path, Remark 2's back
// propagation carried forward-over-reverse; FP64 throughout).
//
// The parameter gradient differentiates E along the coordinate direction v = gF: every
// neighbour row carries s with its tangent sd = (ds/dr) (d . dd) / r and R~ with its tangent
// (dR~/dd) dd, dd = v_j - v_i (Eq. 5 differentiated).  Both passes run one wave per centre
// and the embedding chain of 16 neighbours at a time on the FP64 16x16x4 MFMA, in the
// position layout of the force path (embed.hip): the value and the tangent chain share
// every weight fragment, layer 2 goes one 16-position tile at a time so that only layers 0
// and 1 stay in registers with their tangents.
//
//   k_pgf_fwd   T = (1/N_m) sum_j G_j R~_j^T and its tangent sum_j (dG_j R~_j^T + G_j dR~_j^T)
//               (Eq. 4).  The sums over the 16 rows of a chunk are MFMA products with the
//               rows as the k dimension: A = [G | dG] (a chunk tile transposed through a
//               small LDS scratch), B = [R~ dR~ | 0 R~] per row, so that columns 0..3 of the
//               result accumulate T and columns 4..7 its tangent.
//   k_pgf_bwd   with dE/dT and its tangent per centre (from the fitting net's reverse pass):
//               dE/dG_j = (1/N_m) dE/dT R~_j and its tangent, then the chain backwards
//               (layer 2's adjoint accumulated tile by tile, the concatenation skips, the
//               1 - tanh^2 factors and their tangents -2 t dt), writing per neighbour row
//               only what the weight gradients need: the layer inputs X0 = t0, X1 = h1, s
//               (each with a trailing column of ones, zeros in the tangent, for the biases)
//               and the pre-activation adjoints P0, P1, P2, each with its tangent, in
//               feature order.  The weight gradients are then plain products over the
//               rows (launch_param_grad).
// Neither pass stores an activation between the forward and the reverse sweep: the
// reverse pass recomputes the chain.
#include <hip/hip_runtime.h>

#include "embed_common.h"

namespace dp {

constexpr int kPgfWaves = 8;
constexpr int kPgfScrStride = 17;                       // doubles per row of the transpose scratch
constexpr int kPgfScr = 2 * 16 * kPgfScrStride + 16 * 8;  // per wave: G and dG tiles, R~ and dR~ rows

__device__ __forceinline__ int pgf_lp(int g, int q) { return lpos(double(), g, q); }

// feature index of position p in a width-s0 block layout (-1 for a pad position)
__device__ __forceinline__ int pgf_feature(int p, int s0) { return (p % kP0) < s0 ? (p / kP0) * s0 + (p % kP0) : -1; }

// Environment row of a neighbour with its tangent along dd: R~ = (s, s d / r),
// dR~ = (ds (d.dd) / r, qf (d.dd) / r d + (s / r) dd) with qf = d(s/r)/dr
__device__ __forceinline__ void pgf_env(const ModelC& m, const double* __restrict__ xe, const double* __restrict__ vd,
                                        int e, int own, const double xi[3], const double vi[3], double (&R)[4],
                                        double (&Rd)[4]) {
  double d[3], dd[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    d[c] = xe[3 * e + c] - xi[c];
    dd[c] = vd[3 * own + c] - vi[c];
  }
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double ir = 1.0 / r;
  double s, ds;
  smooth_fn_ir(m, r, ir, s, ds);
  const double sr = s * ir;
  const double dot = (d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2]) * ir;
  const double qf = ds * ir - s * ir * ir;
  R[0] = s;
  Rd[0] = ds * dot;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    R[1 + c] = sr * d[c];
    Rd[1 + c] = qf * dot * d[c] + sr * dd[c];
  }
}

// layers 0 and 1 with tangents: t0 = tanh(s W0 + b0), dt0 = (1 - t0^2) W0 sd;
// t1 = tanh(W1^T t0 + b1), dt1 = (1 - t1^2) W1^T dt0
__device__ __forceinline__ void pgf_l01(const double* __restrict__ net, double s, double sd, int g, int rb,
                                        double (&t0)[2][4], double (&dt0)[2][4], double (&t1)[4][4],
                                        double (&dt1)[4][4]) {
#pragma unroll
  for (int n = 0; n < 2; n++)
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int p = 16 * n + pgf_lp(g, q);
      const double w = net[kOffW0 + p];
      const double t = dp_tanh(s * w + net[kOffB0 + p]);
      t0[n][q] = t;
      dt0[n][q] = (1.0 - t * t) * w * sd;
    }
#pragma unroll
  for (int mt = 0; mt < 4; mt++) {
    d4v c = {0, 0, 0, 0}, cd = {0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < 2; n++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double w = net[kOffW1 + (16 * n + pgf_lp(g, q)) * kW1Stride + 16 * mt + rb];
        c = mfma4(w, t0[n][q], c);
        cd = mfma4(w, dt0[n][q], cd);
      }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const double t = dp_tanh(c[q] + net[kOffB1 + 16 * mt + pgf_lp(g, q)]);
      t1[mt][q] = t;
      dt1[mt][q] = (1.0 - t * t) * cd[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// layer 2, tile mt: t2 = tanh(W2^T h1 + b2), dt2 = (1 - t2^2) W2^T dh1, h1 = (t0, t0) + t1
__device__ __forceinline__ void pgf_l2(const double* __restrict__ net, int mt, int g, int rb, const double (&t0)[2][4],
                                       const double (&dt0)[2][4], const double (&t1)[4][4],
                                       const double (&dt1)[4][4], double (&t2)[4], double (&dt2)[4]) {
  d4v c = {0, 0, 0, 0}, cd = {0, 0, 0, 0};
#pragma unroll
  for (int n = 0; n < 4; n++) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const double w = net[kOffW2 + (16 * n + pgf_lp(g, q)) * kW2Stride + 16 * mt + rb];
      c = mfma4(w, t0[n & 1][q] + t1[n][q], c);
      cd = mfma4(w, dt0[n & 1][q] + dt1[n][q], cd);
    }
    __builtin_amdgcn_sched_barrier(0);   // bounds the operands in flight (register budget)
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const double t = dp_tanh(c[q] + net[kOffB2 + 16 * mt + pgf_lp(g, q)]);
    t2[q] = t;
    dt2[q] = (1.0 - t * t) * cd[q];
  }
}

__device__ __forceinline__ void pgf_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------------------
// pass 1: T and its tangent per centre
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(64 * kPgfWaves) void k_pgf_fwd(PgfArgs A) {
  extern __shared__ __align__(16) char smem[];
  double* net = (double*)smem;
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  double* sg = net + kNetElems + wv * kPgfScr;   // [16 positions][kPgfScrStride]: G of the tile
  double* sdg = sg + 16 * kPgfScrStride;          // the same for dG
  double* rr = sdg + 16 * kPgfScrStride;          // [16 rows][8]: R~ then dR~
  const int r0 = blockIdx.x * kPgfWaves;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;   // uniform over the block
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  double xi[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
  if (atom >= 0)
#pragma unroll
    for (int c = 0; c < 3; c++) {
      xi[c] = A.xe[3 * atom + c];
      vi[c] = A.vdir[3 * atom + c];
    }
  d4v acc[8];
#pragma unroll
  for (int mt = 0; mt < 8; mt++) acc[mt] = d4v{0, 0, 0, 0};
  for (int beta = 0; beta < m.ntypes; beta++) {
    __syncthreads();
    stage_bytes(net, A.nets + (size_t)(alpha * m.ntypes + beta) * kNetElems, (int)sizeof(double) * kNetElems);
    __syncthreads();
    if (atom < 0) continue;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int k = c0 + rb;
      double R[4] = {0, 0, 0, 0}, Rd[4] = {0, 0, 0, 0};
      if (k < nn) {
        const int e = nl[k];
        pgf_env(m, A.xe, A.vdir, e, A.eown[e], xi, vi, R, Rd);
      }
      // this chunk's rows of R~ and dR~ for the B operands (lane group g writes two)
      pgf_wave_sync();   // the previous chunk's reads are done
      {
        const double a0 = g == 0 ? R[0] : g == 1 ? R[2] : g == 2 ? Rd[0] : Rd[2];
        const double a1 = g == 0 ? R[1] : g == 1 ? R[3] : g == 2 ? Rd[1] : Rd[3];
        rr[rb * 8 + 2 * g] = a0;
        rr[rb * 8 + 2 * g + 1] = a1;
      }
      double t0[2][4], dt0[2][4], t1[4][4], dt1[4][4];
      pgf_l01(net, R[0], Rd[0], g, rb, t0, dt0, t1, dt1);
#pragma unroll 1
      for (int mt = 0; mt < 8; mt++) {
        double t2[4], dt2[4];
        pgf_l2(net, mt, g, rb, t0, dt0, t1, dt1, t2, dt2);
        pgf_wave_sync();   // the previous tile's transposes have been read
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int pl = pgf_lp(g, q);
          sg[pl * kPgfScrStride + rb] = t0[mt & 1][q] + t1[mt & 3][q] + t2[q];
          sdg[pl * kPgfScrStride + rb] = dt0[mt & 1][q] + dt1[mt & 3][q] + dt2[q];
        }
        pgf_wave_sync();
        // C[position][j] += sum over (row, which) of A B: k steps 0..3 take G rows 4 ks + g,
        // 4..7 the dG rows; B column j of row r is R~[j], dR~[j - 4] (G) or R~[j - 4] (dG)
        d4v c = acc[0];   // acc[mt], selected without indexing registers at run time
#pragma unroll
        for (int t = 1; t < 8; t++) c = mt == t ? acc[t] : c;
#pragma unroll
        for (int ks = 0; ks < 8; ks++) {
          const int r = 4 * (ks & 3) + g;
          const double a = (ks < 4 ? sg : sdg)[rb * kPgfScrStride + r];
          double b;
          if (ks < 4) b = rb < 8 ? rr[r * 8 + rb] : 0.0;
          else b = (rb >= 4 && rb < 8) ? rr[r * 8 + rb - 4] : 0.0;
          c = mfma4(a, b, c);
        }
#pragma unroll
        for (int t = 0; t < 8; t++) acc[t] = mt == t ? c : acc[t];
      }
    }
  }
  if (atom < 0 || rb >= 8) return;
  // lane (j, g) holds C[position 16 mt + lpos(g, r)][j]: j < 4 the value, 4..7 the tangent
  double* out = (rb < 4 ? A.Tm : A.Tmd) + (size_t)row * m.M * 4;
  const int c = rb & 3;
#pragma unroll
  for (int mt = 0; mt < 8; mt++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int f = pgf_feature(16 * mt + pgf_lp(g, r), m.s0);
      if (f >= 0) out[f * 4 + c] = acc[mt][r] * m.inv_norm;
    }
}

// ------------------------------------------------------------------------------------
// pass 2: the reverse chain with tangents and the weight-gradient operands per row
// ------------------------------------------------------------------------------------
// store the values of one position tile (lane (rb, g), register q: position 16 t + lpos(g, q))
// into a feature-order row
__device__ __forceinline__ void pgf_put(double* __restrict__ dst, int width, int s0, int t, int g,
                                        const double (&v)[4]) {
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int f = pgf_feature(16 * t + pgf_lp(g, q), s0);
    if (f >= 0 && f < width) dst[f] = v[q];
  }
}

__global__ __launch_bounds__(64 * kPgfWaves) void k_pgf_bwd(PgfArgs A) {
  extern __shared__ __align__(16) char smem[];
  double* net = (double*)smem;
  const ModelC& m = A.m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, rb = lane & 15, g = lane >> 4;
  double* gts = net + kNetElems + wv * 2 * kP2 * 4;   // dE/dT at positions [kP2][4]
  double* gtd = gts + kP2 * 4;                        // and its tangent
  const int r0 = blockIdx.x * kPgfWaves;
  const int alpha = species_of(r0, m.ntypes, A.type_row0);
  if (alpha < 0) return;
  const int row = r0 + wv;
  const int atom = A.row_atom[row];
  const int M = m.M, s0 = m.s0, s1 = 2 * s0;
  double xi[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
  if (atom >= 0) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      xi[c] = A.xe[3 * atom + c];
      vi[c] = A.vdir[3 * atom + c];
    }
    for (int q = lane; q < kP2 * 4; q += 64) {
      const int f = pgf_feature(q >> 2, s0), c = q & 3;
      gts[q] = f >= 0 ? A.gTm[((size_t)row * M + f) * 4 + c] : 0.0;
      gtd[q] = f >= 0 ? A.gTmd[((size_t)row * M + f) * 4 + c] : 0.0;
    }
  }
  const double inorm = m.inv_norm;
  for (int beta = 0; beta < m.ntypes; beta++) {
    __syncthreads();
    stage_bytes(net, A.nets + (size_t)(alpha * m.ntypes + beta) * kNetElems, (int)sizeof(double) * kNetElems);
    __syncthreads();
    if (atom < 0) continue;
    const int nn = A.nnei[atom * m.ntypes + beta];
    const int* nl = A.nlist + (size_t)atom * m.nm + m.sel_off[beta];
    const size_t pb = (size_t)A.boff[beta] + A.base[beta][row];   // pair index of the centre's first row
    for (int c0 = 0; c0 < nn; c0 += 16) {
      const int k = c0 + rb;
      const bool valid = k < nn;
      double R[4] = {0, 0, 0, 0}, Rd[4] = {0, 0, 0, 0};
      if (valid) {
        const int e = nl[k];
        pgf_env(m, A.xe, A.vdir, e, A.eown[e], xi, vi, R, Rd);
      }
      const size_t p = pb + k;
      double t0[2][4], dt0[2][4], t1[4][4], dt1[4][4];
      pgf_l01(net, R[0], Rd[0], g, rb, t0, dt0, t1, dt1);
      if (valid) {
        // layer inputs with a trailing column (1 for the value, 0 for the tangent): the
        // weight-gradient products then also yield the bias gradients, which follow the
        // weights in theta
        pgf_put(A.X0 + p * (s0 + 1), s0, s0, 0, g, t0[0]);
        pgf_put(A.X0 + p * (s0 + 1), s0, s0, 1, g, t0[1]);
        pgf_put(A.X0d + p * (s0 + 1), s0, s0, 0, g, dt0[0]);
        pgf_put(A.X0d + p * (s0 + 1), s0, s0, 1, g, dt0[1]);
#pragma unroll
        for (int n = 0; n < 4; n++) {
          double h[4], hd[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            h[q] = t0[n & 1][q] + t1[n][q];
            hd[q] = dt0[n & 1][q] + dt1[n][q];
          }
          pgf_put(A.X1 + p * (s1 + 1), s1, s0, n, g, h);
          pgf_put(A.X1d + p * (s1 + 1), s1, s0, n, g, hd);
        }
        if (g == 0) {
          A.X0[p * (s0 + 1) + s0] = 1.0;
          A.X0d[p * (s0 + 1) + s0] = 0.0;
          A.X1[p * (s1 + 1) + s1] = 1.0;
          A.X1d[p * (s1 + 1) + s1] = 0.0;
          A.S[2 * p] = R[0];
          A.S[2 * p + 1] = 1.0;
          A.Sd[2 * p] = Rd[0];
          A.Sd[2 * p + 1] = 0.0;
        }
      }
      // dE/dh1 (layer 1's output) accumulated over the layer-2 tiles: the concatenation
      // skip of G = (h1, h1) + t2 passes dE/dG of tiles mt and mt + 4 to tile mt % 4, and
      // layer 2's adjoint adds W2 P2 tile by tile
      d4v dh1[4], ddh1[4];
#pragma unroll
      for (int n = 0; n < 4; n++) dh1[n] = ddh1[n] = d4v{0, 0, 0, 0};
#pragma unroll 1
      for (int mt = 0; mt < 8; mt++) {
        double t2[4], dt2[4], P2[4], dP2[4];
        pgf_l2(net, mt, g, rb, t0, dt0, t1, dt1, t2, dt2);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int pp = 16 * mt + pgf_lp(g, q);
          const double* gp = gts + pp * 4;
          const double* gq = gtd + pp * 4;
          const double gG = (gp[0] * R[0] + gp[1] * R[1] + gp[2] * R[2] + gp[3] * R[3]) * inorm;
          const double dgG = (gq[0] * R[0] + gq[1] * R[1] + gq[2] * R[2] + gq[3] * R[3] + gp[0] * Rd[0] +
                              gp[1] * Rd[1] + gp[2] * Rd[2] + gp[3] * Rd[3]) * inorm;
          const double u = 1.0 - t2[q] * t2[q];
          P2[q] = gG * u;
          dP2[q] = dgG * u - 2.0 * gG * t2[q] * dt2[q];
#pragma unroll
          for (int n = 0; n < 4; n++) {   // the skip into tile mt % 4, selected
            dh1[n][q] += (mt & 3) == n ? gG : 0.0;
            ddh1[n][q] += (mt & 3) == n ? dgG : 0.0;
          }
        }
        if (valid) {
          pgf_put(A.P2 + p * M, M, s0, mt, g, P2);
          pgf_put(A.P2d + p * M, M, s0, mt, g, dP2);
        }
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
          d4v c = dh1[nt], cd = ddh1[nt];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const double w = net[kOffW2 + (16 * nt + rb) * kW2Stride + 16 * mt + pgf_lp(g, q)];
            c = mfma4(w, P2[q], c);
            cd = mfma4(w, dP2[q], cd);
          }
          dh1[nt] = c;
          ddh1[nt] = cd;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // layer 1: the concatenation skip h1 = (t0, t0) + t1 passes the undamped dE/dh1 of
      // tiles n and n + 2 to t0's tile n; P1 = dE/dh1 (1 - t1^2) and its tangent
      d4v dh0[2], ddh0[2];
#pragma unroll
      for (int n = 0; n < 2; n++) {
        dh0[n] = dh1[n] + dh1[n + 2];
        ddh0[n] = ddh1[n] + ddh1[n + 2];
      }
      double P1[4][4], dP1[4][4];
#pragma unroll
      for (int n = 0; n < 4; n++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const double t = t1[n][q], u = 1.0 - t * t;
          P1[n][q] = dh1[n][q] * u;
          dP1[n][q] = ddh1[n][q] * u - 2.0 * dh1[n][q] * t * dt1[n][q];
        }
      if (valid)
#pragma unroll
        for (int n = 0; n < 4; n++) {
          pgf_put(A.P1 + p * s1, s1, s0, n, g, P1[n]);
          pgf_put(A.P1d + p * s1, s1, s0, n, g, dP1[n]);
        }
#pragma unroll
      for (int nt = 0; nt < 2; nt++) {
        d4v c = dh0[nt], cd = ddh0[nt];
#pragma unroll
        for (int n = 0; n < 4; n++)
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const double w = net[kOffW1 + (16 * nt + rb) * kW1Stride + 16 * n + pgf_lp(g, q)];
            c = mfma4(w, P1[n][q], c);
            cd = mfma4(w, dP1[n][q], cd);
          }
        dh0[nt] = c;
        ddh0[nt] = cd;
      }
      // layer 0: P0 = dE/dt0 (1 - t0^2) and its tangent
      if (valid)
#pragma unroll
        for (int n = 0; n < 2; n++) {
          double P0[4], dP0[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const double t = t0[n][q], u = 1.0 - t * t;
            P0[q] = dh0[n][q] * u;
            dP0[q] = ddh0[n][q] * u - 2.0 * dh0[n][q] * t * dt0[n][q];
          }
          pgf_put(A.P0 + p * s0, s0, s0, n, g, P0);
          pgf_put(A.P0d + p * s0, s0, s0, n, g, dP0);
        }
    }
  }
}

size_t pgf_fwd_lds() { return sizeof(double) * ((size_t)kNetElems + (size_t)kPgfWaves * kPgfScr); }
size_t pgf_bwd_lds() { return sizeof(double) * ((size_t)kNetElems + (size_t)kPgfWaves * 2 * kP2 * 4); }

void launch_pgf_fwd(const PgfArgs& a, hipStream_t st) {
  const size_t sh = pgf_fwd_lds();
  (void)hipFuncSetAttribute((const void*)k_pgf_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  const int grid = (a.nrows + kPgfWaves - 1) / kPgfWaves;
  if (grid > 0) hipLaunchKernelGGL(k_pgf_fwd, dim3(grid), dim3(64 * kPgfWaves), sh, st, a);
}

void launch_pgf_bwd(const PgfArgs& a, hipStream_t st) {
  const size_t sh = pgf_bwd_lds();
  (void)hipFuncSetAttribute((const void*)k_pgf_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  const int grid = (a.nrows + kPgfWaves - 1) / kPgfWaves;
  if (grid > 0) hipLaunchKernelGGL(k_pgf_bwd, dim3(grid), dim3(64 * kPgfWaves), sh, st, a);
}

}  // namespace dp
