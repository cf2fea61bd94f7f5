// Velocity-Verlet integration and thermodynamic output (paper Section 4: velocity
// Verlet, thermo data - kinetic and potential energy, temperature, pressure - every
// few steps).  All state stays on the device in FP64; positions are not wrapped
// (the force path wraps them itself).
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace dp {

constexpr double kAcc = 9.64853321e-3;    // eV / (A amu) in A / fs^2
constexpr double kKb = 8.617333262e-5;    // eV / K
constexpr double kEvA3Bar = 1.602176634e6;

// After a drift: flag (*gate |= 1) when some atom moved more than half the neighbour
// skin since the last list build (or has a non-finite coordinate), and clear the cell
// counters for the rebuild that may follow.  gate == NULL: no check.
__device__ __forceinline__ void vv_check(const VvCheck& c, int i, int n, const double* __restrict__ x) {
  if (!c.gate) return;
  for (int q = i; q < c.nc1 || q < c.nc2; q += gridDim.x * blockDim.x) {
    if (q < c.nc1) c.c1[q] = 0;
    if (q < c.nc2) c.c2[q] = 0;
  }
  bool moved = false;
  if (i < n) {
    const double d0 = x[3 * i] - c.xref[3 * i], d1 = x[3 * i + 1] - c.xref[3 * i + 1],
                 d2 = x[3 * i + 2] - c.xref[3 * i + 2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    moved = !(r2 <= c.lim2);
  }
  if (__ballot(moved) && (threadIdx.x & 63) == 0) atomicOr(c.gate, 1);
}

// v += (dt/2) F / m; optionally x += dt v (one thread per atom)
__global__ __launch_bounds__(256) void k_vv(int n, const int* __restrict__ types, MDMass mass, double half_dt_acc,
                                            double dt, const double* __restrict__ F, double* __restrict__ v,
                                            double* __restrict__ x, int drift, VvCheck chk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int t = types[i];
    const double im = (t >= 0 && t < kMaxTypes) ? mass.inv[t] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int q = 3 * i + c;
      const double vv = v[q] + half_dt_acc * F[q] * im;
      v[q] = vv;
      if (drift) x[q] += dt * vv;
    }
  }
  if (drift) vv_check(chk, i, n, x);
}

// the closing half kick of one step and the opening half kick and drift of the next in
// one pass (the two half kicks are added one after the other, exactly as two launches
// would); F is consumed and cleared for the next force evaluation
__global__ __launch_bounds__(256) void k_vv2(int n, const int* __restrict__ types, MDMass mass, double half_dt_acc,
                                             double dt, double* __restrict__ F, double* __restrict__ v,
                                             double* __restrict__ x, VvCheck chk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int t = types[i];
    const double im = (t >= 0 && t < kMaxTypes) ? mass.inv[t] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int q = 3 * i + c;
      const double f = F[q];
      double vv = v[q] + half_dt_acc * f * im;
      vv = vv + half_dt_acc * f * im;
      v[q] = vv;
      x[q] += dt * vv;
      F[q] = 0.0;
    }
  }
  vv_check(chk, i, n, x);
}

// thermo row [step, PE, KE, T, Etot, P(bar)] in two launches with fixed-order sums: block
// b adds the kinetic energies of atoms [1024 b, 1024 b + 1024) (butterfly shuffles, then
// its four waves in order) into part[b]; one block then adds the parts in order
constexpr int kKePer = 1024;

__global__ __launch_bounds__(256) void k_thermo_part(int n, const int* __restrict__ types, MDMass mass,
                                                     const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double sh[4];
  double ke = 0.0;
#pragma unroll
  for (int k = 0; k < kKePer / 256; k++) {
    const int i = blockIdx.x * kKePer + 256 * k + threadIdx.x;
    if (i < n) {
      const int t = types[i];
      const double m = (t >= 0 && t < kMaxTypes) ? mass.m[t] : 0.0;
      ke += 0.5 * m * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ke += __shfl_xor(ke, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ke;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ __launch_bounds__(1024) void k_thermo(int n, int nparts, const double* __restrict__ part,
                                                 double volume, int step,
                                                 const double* __restrict__ E,
                                                 const double* __restrict__ W,
                                                 double* __restrict__ row) {
  __shared__ double sh[1024];
  double ke = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 1024) ke += part[b];
  sh[threadIdx.x] = ke;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double K = sh[0] / kAcc;
    double T = 2.0 * K / ((3.0 * n - 3.0) * kKb);
    double P = (2.0 * K + (W[0] + W[4] + W[8])) / (3.0 * volume) * kEvA3Bar;
    row[0] = step;
    row[1] = E[0];
    row[2] = K;
    row[3] = T;
    row[4] = E[0] + K;
    row[5] = P;
  }
}

int thermo_parts(int n) { return (n + kKePer - 1) / kKePer; }

void launch_vv(int n, const int* types, const MDMass& mass, double dt, const double* F, double* v,
               double* x, bool drift, const VvCheck& chk, hipStream_t st) {
  hipLaunchKernelGGL(k_vv, dim3((n + 255) / 256), dim3(256), 0, st, n, types, mass, 0.5 * dt * kAcc,
                     dt, F, v, x, drift ? 1 : 0, chk);
}

void launch_vv_merged(int n, const int* types, const MDMass& mass, double dt, double* F, double* v, double* x,
                      const VvCheck& chk, hipStream_t st) {
  hipLaunchKernelGGL(k_vv2, dim3((n + 255) / 256), dim3(256), 0, st, n, types, mass, 0.5 * dt * kAcc, dt, F,
                     v, x, chk);
}

void launch_thermo(int n, const int* types, const MDMass& mass, double volume, int step,
                   const double* v, const double* E, const double* W, double* row, double* part, hipStream_t st) {
  const int np = thermo_parts(n);
  hipLaunchKernelGGL(k_thermo_part, dim3(np), dim3(256), 0, st, n, types, mass, v, part);
  hipLaunchKernelGGL(k_thermo, dim3(1), dim3(1024), 0, st, n, np, part, volume, step, E, W, row);
}

// ------------------------------------------------------------------------------------
// Isobaric MD: the Martyna-Tobias-Klein equations with isotropic box scaling, the
// pressure from the virial (Section 4's thermo pressure) driving the box, and an
// optional Nose-Hoover thermostat on the particles, integrated by the symmetric
// splitting T(dt/2) E(dt/2) P(dt/2) R(dt) [forces] P(dt/2) E(dt/2) T(dt/2):
//   E(h): p_eps += h (alpha 2 KE + tr W - 3 V P_ext)
//   P(h): v <- v exp(-alpha v_eps h) + h a exp(-alpha v_eps h / 2) sinhc(alpha v_eps h / 2)
//   R(h): x <- x exp(v_eps h) + h v exp(v_eps h / 2) sinhc(v_eps h / 2), B <- B exp(v_eps h)
//   T(h): p_xi += h/2 (2 KE - N_f kT); v <- v exp(-h v_xi); xi += h v_xi; p_xi += ...
// The global steps (kinetic energy, the barostat and thermostat variables, the box)
// run in one-block kernels; the thermostat's velocity scale is carried in the state and
// folded into the next velocity update.  The neighbour skin check compares x with the
// reference positions scaled by mu = (box scale) / (box scale at the last build): a pair
// outside the list was at least rl apart at the build, so it stays outside rc while
// every atom's non-affine displacement is below (mu rl - rc) / 2.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double npt_sinhc(double y) {
  return fabs(y) < 1e-4 ? 1.0 + y * y / 6.0 * (1.0 + y * y / 20.0) : sinh(y) / y;
}

// sum of 0.5 m v^2 over the atoms (amu A^2 / fs^2) by one 1024-thread block, fixed order
__device__ double block_ke(int n, const int* __restrict__ types, const MDMass& mass, const double* __restrict__ v,
                           double* sh) {
  double ke = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int t = types[i];
    const double m = (t >= 0 && t < kMaxTypes) ? mass.m[t] : 0.0;
    ke += 0.5 * m * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  }
  sh[threadIdx.x] = ke;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// thermostat half step of length h on the state (kinetic energy updated, velocities not)
__device__ void npt_thermostat(double* S, const NptConst& c) {
  if (!c.thermostat) return;
  double ke = S[NS_KE];
  double pxi = S[NS_PXI] + 0.5 * c.h * (2.0 * ke - c.nf * c.kT);
  const double f = exp(-c.h * pxi / c.Q);
  S[NS_CPEND] *= f;
  ke *= f * f;
  S[NS_XI] += c.h * pxi / c.Q;
  pxi += 0.5 * c.h * (2.0 * ke - c.nf * c.kT);
  S[NS_PXI] = pxi;
  S[NS_KE] = ke;
}

__device__ void npt_row(const double* S, const NptConst& c, int step, double E, const double* W, double* row) {
  const double ke = S[NS_KE], V = S[NS_V];
  row[0] = step;
  row[1] = E;
  row[2] = ke;
  row[3] = 2.0 * ke / (c.nf * kKb);
  row[4] = E + ke;
  row[5] = (2.0 * ke + (W[0] + W[4] + W[8])) / (3.0 * V) * kEvA3Bar;
  row[6] = V;
  row[7] = E + ke + 0.5 * S[NS_PEPS] * S[NS_PEPS] / c.W + c.pext * V +
           (c.thermostat ? 0.5 * S[NS_PXI] * S[NS_PXI] / c.Q + c.nf * c.kT * S[NS_XI] : 0.0);
}

__global__ __launch_bounds__(1024) void k_npt_init(int n, const int* __restrict__ types, MDMass mass,
                                                   const double* __restrict__ v, double* __restrict__ S, NptConst c) {
  __shared__ double sh[1024];
  const double ke = block_ke(n, types, mass, v, sh) / kAcc;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NS_COUNT; k++) S[k] = 0.0;
    S[NS_LAM] = 1.0;
    S[NS_LAMB] = 1.0;
    S[NS_KE] = ke;
    S[NS_CPEND] = 1.0;
    S[NS_V] = c.V0;
  }
}

__global__ void k_npt_open(double* __restrict__ S, NptConst c, const double* __restrict__ W, Frame* __restrict__ frames,
                           int* __restrict__ status) {
  if (threadIdx.x != 0) return;
  npt_thermostat(S, c);
  const double trW = W[0] + W[4] + W[8];
  const double peps = S[NS_PEPS] + c.h * (c.alpha * 2.0 * S[NS_KE] + trW - 3.0 * S[NS_V] * c.pext);
  S[NS_PEPS] = peps;
  const double ve = peps / c.W;
  const double y = c.alpha * ve * c.h;
  const double a1 = exp(-y);
  S[NS_A1] = a1;
  S[NS_A1O] = a1 * S[NS_CPEND];
  S[NS_CPEND] = 1.0;
  S[NS_B1] = c.h * exp(-0.5 * y) * npt_sinhc(0.5 * y);
  const double yr = ve * c.dt;
  const double sx = exp(yr);
  S[NS_SX] = sx;
  S[NS_B2] = c.dt * exp(0.5 * yr) * npt_sinhc(0.5 * yr);
  const double lam = S[NS_LAM] * sx;
  S[NS_LAM] = lam;
  S[NS_V] = c.V0 * lam * lam * lam;
  for (int k = 0; k < 9; k++) {
    frames[0].B[k] = c.B0[k] * lam;
    frames[0].Bi[k] = c.Bi0[k] / lam;
  }
  const double mu = lam / S[NS_LAMB];
  const double L = 0.5 * (mu * c.rl - c.rc);
  S[NS_MU] = mu;
  S[NS_LIM2] = L > 0.0 ? L * L : -1.0;   // -1: rebuild at once
  if (!(lam >= c.min_scale)) atomicOr(&status[STW_FLAGS], ST_CAPACITY);   // the plan no longer covers the box
}

__global__ __launch_bounds__(256) void k_vv_npt_open(int n, const int* __restrict__ types, MDMass mass,
                                                     double* __restrict__ F, double* __restrict__ v,
                                                     double* __restrict__ x, const double* __restrict__ S,
                                                     VvCheck chk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double a1o = S[NS_A1O], b1 = S[NS_B1] * kAcc, sx = S[NS_SX], b2 = S[NS_B2];
  const double mu = S[NS_MU], lim2 = S[NS_LIM2];
  for (int q = i; q < chk.nc1 || q < chk.nc2; q += gridDim.x * blockDim.x) {
    if (q < chk.nc1) chk.c1[q] = 0;
    if (q < chk.nc2) chk.c2[q] = 0;
  }
  bool moved = false;
  if (i < n) {
    const int t = types[i];
    const double im = (t >= 0 && t < kMaxTypes) ? mass.inv[t] : 0.0;
    double r2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const int q = 3 * i + c;
      const double vv = v[q] * a1o + b1 * F[q] * im;
      v[q] = vv;
      const double xn = x[q] * sx + b2 * vv;
      x[q] = xn;
      F[q] = 0.0;
      const double d = xn - mu * chk.xref[q];
      r2 += d * d;
    }
    moved = !(r2 <= lim2);
  }
  if (__ballot(moved) && (threadIdx.x & 63) == 0) atomicOr(chk.gate, 1);
}

__global__ __launch_bounds__(256) void k_vv_npt_close(int n, const int* __restrict__ types, MDMass mass,
                                                      const double* __restrict__ F, double* __restrict__ v,
                                                      const double* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a1 = S[NS_A1], b1 = S[NS_B1] * kAcc;
  const int t = types[i];
  const double im = (t >= 0 && t < kMaxTypes) ? mass.inv[t] : 0.0;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const int q = 3 * i + c;
    v[q] = v[q] * a1 + b1 * F[q] * im;
  }
}

__global__ __launch_bounds__(1024) void k_npt_close(int n, const int* __restrict__ types, MDMass mass,
                                                    const double* __restrict__ v, double* __restrict__ S, NptConst c,
                                                    const double* __restrict__ E, const double* __restrict__ W,
                                                    int step, double* __restrict__ row, int kick) {
  __shared__ double sh[1024];
  const double ke = block_ke(n, types, mass, v, sh) / kAcc;
  if (threadIdx.x != 0) return;
  if (kick) {
    S[NS_KE] = ke;   // the velocities carry no pending scale here
    const double trW = W[0] + W[4] + W[8];
    S[NS_PEPS] += c.h * (c.alpha * 2.0 * ke + trW - 3.0 * S[NS_V] * c.pext);
    npt_thermostat(S, c);
  }
  if (row) npt_row(S, c, step, E[0], W, row);
}

__global__ void k_npt_finish(int n, double* __restrict__ v, const double* __restrict__ S,
                             const Frame* __restrict__ frames, double* __restrict__ box_out,
                             double* __restrict__ state_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double f = S[NS_CPEND];
  if (i < 3 * n) v[i] *= f;
  if (i == 0) {
    if (box_out)
      for (int k = 0; k < 9; k++) box_out[k] = frames[0].B[k];
    if (state_out) {
      state_out[0] = S[NS_PEPS];
      state_out[1] = S[NS_XI];
      state_out[2] = S[NS_PXI];
    }
  }
}

void launch_npt_init(int n, const int* types, const MDMass& mass, const double* v, double* state, const NptConst& c,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_npt_init, dim3(1), dim3(1024), 0, st, n, types, mass, v, state, c);
}
void launch_npt_open(double* state, const NptConst& c, const double* W, Frame* frames, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_npt_open, dim3(1), dim3(64), 0, st, state, c, W, frames, status);
}
void launch_vv_npt_open(int n, const int* types, const MDMass& mass, double* F, double* v, double* x,
                        const double* state, const VvCheck& chk, hipStream_t st) {
  hipLaunchKernelGGL(k_vv_npt_open, dim3((n + 255) / 256), dim3(256), 0, st, n, types, mass, F, v, x, state, chk);
}
void launch_vv_npt_close(int n, const int* types, const MDMass& mass, const double* F, double* v,
                         const double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_vv_npt_close, dim3((n + 255) / 256), dim3(256), 0, st, n, types, mass, F, v, state);
}
void launch_npt_close(int n, const int* types, const MDMass& mass, const double* v, double* state,
                      const NptConst& c, const double* E, const double* W, int step, double* row, bool kick,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_npt_close, dim3(1), dim3(1024), 0, st, n, types, mass, v, state, c, E, W, step, row,
                     kick ? 1 : 0);
}
void launch_npt_finish(int n, double* v, const double* state, const Frame* frames, double* box_out,
                       double* state_out, hipStream_t st) {
  hipLaunchKernelGGL(k_npt_finish, dim3((3 * n + 255) / 256), dim3(256), 0, st, n, v, state, frames, box_out,
                     state_out);
}

}  // namespace dp
