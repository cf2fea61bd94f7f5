// Deterministic force assembly (the reverse communication of Remark 4 done as a
// gather).  The embedding adjoint stores each pair force g_ij in its neighbour-list
// slot instead of adding -g_ij to atom j with atomics; this file builds, per owner
// atom j, the list of slots (i, k) whose neighbour is an image of j, in increasing
// order of i * N_m + k, and adds -sum g over that list in a fixed order.  The result
// does not depend on the scheduling of the kernels.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace dp {

constexpr int kRevWaves = 4;
constexpr int kRevCap = 2048;   // reverse entries one wave can sort in LDS

// cnt[j] = number of slots whose neighbour is owned by j
__global__ void k_rev_count(int n, int nm, const int* __restrict__ nlist, const int* __restrict__ eown,
                            int* __restrict__ cnt) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * nm) return;
  int e = nlist[q];
  if (e >= 0) atomicAdd(&cnt[eown[e]], 1);
}

// rev[off[j] .. off[j] + cnt[j]) = the slots of owner j, in arrival order
__global__ void k_rev_fill(int n, int nm, const int* __restrict__ nlist, const int* __restrict__ eown,
                           const int* __restrict__ off, int* __restrict__ fill, int* __restrict__ rev) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)n * nm) return;
  int e = nlist[q];
  if (e < 0) return;
  int j = eown[e];
  int p = atomicAdd(&fill[j], 1);
  rev[off[j] + p] = (int)q;
}

// one wave per owner j: sort its slots, then F_j -= sum g in that order
__global__ __launch_bounds__(64 * kRevWaves) void k_rev_gather(int n, const int* __restrict__ off,
                                                              const int* __restrict__ cnt,
                                                              const int* __restrict__ rev,
                                                              const double* __restrict__ gbuf,
                                                              double* __restrict__ forces,
                                                              int* __restrict__ status) {
  __shared__ int s_in[kRevWaves][kRevCap];
  __shared__ int s_out[kRevWaves][kRevCap];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * kRevWaves + wv;
  if (j >= n) return;
  int c = cnt[j];
  if (c > kRevCap) {
    if (lane == 0) atomicOr(&status[STW_FLAGS], ST_CAPACITY);
    c = kRevCap;
  }
  const int* r = rev + off[j];
  for (int p = lane; p < c; p += 64) s_in[wv][p] = r[p];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // rank sort (the slot indices are distinct)
  for (int p = lane; p < c; p += 64) {
    int v = s_in[wv][p], rank = 0;
    for (int u = 0; u < c; u++) rank += s_in[wv][u] < v;
    s_out[wv][rank] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double acc[3] = {0, 0, 0};
  for (int p = lane; p < c; p += 64) {
    size_t q = (size_t)s_out[wv][p] * 3;
#pragma unroll
    for (int b = 0; b < 3; b++) acc[b] += gbuf[q + b];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int b = 0; b < 3; b++) acc[b] += __shfl_xor(acc[b], o);
  if (lane < 3) {
    double v = lane == 0 ? acc[0] : lane == 1 ? acc[1] : acc[2];
    forces[3 * j + lane] -= v;
  }
}

size_t rev_scratch_ints(int n, int nm) { return (size_t)3 * (n + 1) + (size_t)n * nm; }

void launch_rev_gather(int n, int nm, const int* nlist, const int* eown, const double* gbuf, double* forces,
                       int* scratch, int* scan_sums, int* scan_total, int* status, hipStream_t st) {
  int* cnt = scratch;
  int* off = cnt + (n + 1);
  int* fill = off + (n + 1);
  int* rev = fill + (n + 1);
  const size_t tot = (size_t)n * nm;
  launch_zero_int(cnt, n + 1, st);
  launch_zero_int(fill, n + 1, st);
  hipLaunchKernelGGL(k_rev_count, dim3((tot + 255) / 256), dim3(256), 0, st, n, nm, nlist, eown, cnt);
  launch_scan_int(n, cnt, off, scan_sums, scan_total, st);
  hipLaunchKernelGGL(k_rev_fill, dim3((tot + 255) / 256), dim3(256), 0, st, n, nm, nlist, eown, off, fill, rev);
  hipLaunchKernelGGL(k_rev_gather, dim3((n + kRevWaves - 1) / kRevWaves), dim3(64 * kRevWaves), 0, st, n, off,
                     cnt, rev, gbuf, forces, status);
}

}  // namespace dp
