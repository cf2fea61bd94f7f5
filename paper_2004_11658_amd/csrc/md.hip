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

// thermo row [step, PE, KE, T, Etot, P(bar)]: one block, fixed-order reduction
__global__ __launch_bounds__(1024) void k_thermo(int n, const int* __restrict__ types, MDMass mass,
                                                 double volume, int step,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ E,
                                                 const double* __restrict__ W,
                                                 double* __restrict__ row) {
  __shared__ double sh[1024];
  double ke = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    int t = types[i];
    double m = (t >= 0 && t < kMaxTypes) ? mass.m[t] : 0.0;
    ke += 0.5 * m * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  }
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
                   const double* v, const double* E, const double* W, double* row, hipStream_t st) {
  hipLaunchKernelGGL(k_thermo, dim3(1), dim3(1024), 0, st, n, types, mass, volume, step, v, E, W, row);
}

}  // namespace dp
