// Neighbour search and formatting on the GPU (paper Section 3.2.2, Alg. 1).
//
// Layout: the local atoms of all frames are followed by their periodic images
// ("ghosts", Section 3.1: a ghost shell at least rc thick around each frame's box).
// Every extended atom e has coordinates xe[e], owner index, species and image code.
// A cell list over the extended region of each frame (cells at least rc wide in
// perpendicular distance) limits the search to 27 cells; each local atom's
// candidates within rc are then ranked by (species, r^2, owner, image) and written
// into per-species blocks of fixed width sel with -1 pads (Alg. 1, Fig. 2a).
//
// Positions that decide integers (inside rc, neighbour order) are computed with
// floating-point contraction off, in a fixed operation order:
//   x_w = x - (m0 B0 + m1 B1) + m2 B2   (m = floor(x . B^-1)),
//   ghost = x_w + (n0 B0 + n1 B1) + n2 B2,  d = ghost - x_w,i,  r^2 = (dx dx + dy dy) + dz dz.
#include <cstring>

#include "common.h"
#include "kernels.h"

namespace dp {

// ------------------------------------------------------------------------------------
// device-wide exclusive scan of int vectors of width W (W counters per element)
// ------------------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

template <int W>
struct IV {
  int v[W];
};

template <int W>
__device__ __forceinline__ IV<W> iv_add(const IV<W>& a, const IV<W>& b) {
  IV<W> c;
#pragma unroll
  for (int q = 0; q < W; q++) c.v[q] = a.v[q] + b.v[q];
  return c;
}

// in: W ints per element produced by a loader; out: exclusive prefix (W ints per
// element); sums: per-block totals.
template <int W, class Load>
__global__ __launch_bounds__(kScanBlock) void k_scan_up(int n, Load load, int* __restrict__ out,
                                                       int* __restrict__ sums, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ IV<W> sh[kScanBlock];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  IV<W> it[kScanItems];
  IV<W> tot;
#pragma unroll
  for (int q = 0; q < W; q++) tot.v[q] = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int i = base + k;
    IV<W> x;
    if (i < n) x = load(i);
    else {
#pragma unroll
      for (int q = 0; q < W; q++) x.v[q] = 0;
    }
    it[k] = tot;  // exclusive within thread
    tot = iv_add<W>(tot, x);
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  // Hillis-Steele inclusive scan of thread totals
  for (int off = 1; off < kScanBlock; off <<= 1) {
    IV<W> v = sh[threadIdx.x];
    IV<W> add;
    bool has = threadIdx.x >= off;
    if (has) add = sh[threadIdx.x - off];
    __syncthreads();
    if (has) sh[threadIdx.x] = iv_add<W>(v, add);
    __syncthreads();
  }
  IV<W> excl;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < W; q++) excl.v[q] = 0;
  } else {
    excl = sh[threadIdx.x - 1];
  }
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    int i = base + k;
    if (i < n) {
      IV<W> v = iv_add<W>(excl, it[k]);
#pragma unroll
      for (int q = 0; q < W; q++) out[(size_t)i * W + q] = v.v[q];
    }
  }
  if (threadIdx.x == kScanBlock - 1) {
#pragma unroll
    for (int q = 0; q < W; q++) sums[blockIdx.x * W + q] = sh[threadIdx.x].v[q];
  }
}

// exclusive scan of nb block sums in place by a single block (looping over chunks);
// total[W] receives the grand total.
template <int W>
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int nb, int* __restrict__ sums,
                                                         int* __restrict__ total, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ IV<W> sh[kScanBlock];
  IV<W> carry;
#pragma unroll
  for (int q = 0; q < W; q++) carry.v[q] = 0;
  for (int c0 = 0; c0 < nb; c0 += kScanBlock) {
    int i = c0 + threadIdx.x;
    IV<W> x;
#pragma unroll
    for (int q = 0; q < W; q++) x.v[q] = i < nb ? sums[i * W + q] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      IV<W> v = sh[threadIdx.x];
      IV<W> add;
      bool has = threadIdx.x >= off;
      if (has) add = sh[threadIdx.x - off];
      __syncthreads();
      if (has) sh[threadIdx.x] = iv_add<W>(v, add);
      __syncthreads();
    }
    IV<W> incl = sh[threadIdx.x];
    if (i < nb) {
#pragma unroll
      for (int q = 0; q < W; q++) sums[i * W + q] = carry.v[q] + incl.v[q] - x.v[q];
    }
    IV<W> last = sh[kScanBlock - 1];
    __syncthreads();
    carry = iv_add<W>(carry, last);
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < W; q++) total[q] = carry.v[q];
  }
}

template <int W>
__global__ __launch_bounds__(kScanBlock) void k_scan_add(int n, int* __restrict__ out,
                                                        const int* __restrict__ sums, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  int i = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; k++) {
    if (i + k < n) {
#pragma unroll
      for (int q = 0; q < W; q++) out[(size_t)(i + k) * W + q] += sums[blockIdx.x * W + q];
    }
  }
}

struct LoadInt {
  const int* p;
  __device__ IV<1> operator()(int i) const { IV<1> r; r.v[0] = p[i]; return r; }
};

template <int W>
struct LoadTypeOneHot {
  const int* types;
  int ntypes;
  __device__ IV<W> operator()(int i) const {
    IV<W> r;
    int t = types[i];
#pragma unroll
    for (int q = 0; q < W; q++) r.v[q] = (q == t) ? 1 : 0;
    return r;
  }
};

// Single-launch exclusive scan of up to kOneTile ints by one 1024-thread block: 16
// consecutive items per thread, wave scans by shuffles, then the 16 wave totals.
constexpr int kOneBlock = 1024;
constexpr int kOneItems = 16;
constexpr int kOneTile = kOneBlock * kOneItems;

template <class Load>
__global__ __launch_bounds__(kOneBlock) void k_scan_one(int n, Load load, int* __restrict__ out,
                                                       int* __restrict__ total, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int wsum[kOneBlock / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int base = t * kOneItems;
  int it[kOneItems];
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kOneItems; k++) {
    const int i = base + k;
    const int x = i < n ? load(i).v[0] : 0;
    it[k] = tot;
    tot += x;
  }
  int incl = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int v = lane < kOneBlock / 64 ? wsum[lane] : 0;
    int sc = v;
#pragma unroll
    for (int off = 1; off < kOneBlock / 64; off <<= 1) {
      const int y = __shfl_up(sc, off, 64);
      if (lane >= off) sc += y;
    }
    if (lane < kOneBlock / 64) wsum[lane] = sc - v;
    if (lane == kOneBlock / 64 - 1) total[0] = sc;
  }
  __syncthreads();
  const int excl = wsum[w] + incl - tot;
#pragma unroll
  for (int k = 0; k < kOneItems; k++) {
    const int i = base + k;
    if (i < n) out[i] = excl + it[k];
  }
}

// scan scratch: sums[nblocks * W]; gate (may be NULL): skip the scan when *gate == 0
template <int W, class Load>
static void scan_launch(int n, Load load, int* out, int* sums, int* total, hipStream_t st,
                        const int* gate = nullptr) {
  if (W == 1 && n <= kOneTile) {
    hipLaunchKernelGGL((k_scan_one<Load>), dim3(1), dim3(kOneBlock), 0, st, n, load, out, total, gate);
    return;
  }
  int nb = (n + kScanTile - 1) / kScanTile;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_scan_up<W, Load>), dim3(nb), dim3(kScanBlock), 0, st, n, load, out, sums, gate);
  hipLaunchKernelGGL((k_scan_sums<W>), dim3(1), dim3(kScanBlock), 0, st, nb, sums, total, gate);
  hipLaunchKernelGGL((k_scan_add<W>), dim3(nb), dim3(kScanBlock), 0, st, n, out, sums, gate);
}

size_t scan_sums_ints(int n, int W) {
  int nb = (n + kScanTile - 1) / kScanTile;
  if (nb < 1) nb = 1;
  return (size_t)nb * W;
}

// ------------------------------------------------------------------------------------
// frame table upload through kernel arguments: a call's frames (box, inverse, cell
// grid) are copied by value into the launch, so no host staging buffer has to outlive
// the call and no host wait is needed
// ------------------------------------------------------------------------------------
constexpr int kFramesPerLaunch = 12;
struct FramePack {
  Frame f[kFramesPerLaunch];
};
static_assert(sizeof(FramePack) + 16 <= 4096, "frame pack exceeds the kernel argument budget");
static_assert(sizeof(Frame) % sizeof(uint32_t) == 0, "Frame is copied in 32-bit words");

__global__ void k_put_frames(FramePack pack, int count, Frame* dst) {
  constexpr int kWords = (int)(sizeof(Frame) / sizeof(uint32_t));
  const uint32_t* src = reinterpret_cast<const uint32_t*>(pack.f);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (int w = threadIdx.x; w < count * kWords; w += blockDim.x) out[w] = src[w];
}

void launch_put_frames(const Frame* frames, int nframes, Frame* dst, hipStream_t st) {
  for (int f0 = 0; f0 < nframes; f0 += kFramesPerLaunch) {
    const int c = nframes - f0 < kFramesPerLaunch ? nframes - f0 : kFramesPerLaunch;
    FramePack pack;
    memcpy(pack.f, frames + f0, sizeof(Frame) * c);
    hipLaunchKernelGGL(k_put_frames, dim3(1), dim3(256), 0, st, pack, c, dst + f0);
  }
}

// ------------------------------------------------------------------------------------
// position arithmetic with contraction off
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void frac_of(const Frame& F, const double x[3], double f[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; k++) f[k] = (x[0] * F.Bi[0 + k] + x[1] * F.Bi[3 + k]) + x[2] * F.Bi[6 + k];
}

__device__ __forceinline__ void shift_of(const Frame& F, int n0, int n1, int n2, double s[3]) {
#pragma clang fp contract(off)
  for (int c = 0; c < 3; c++)
    s[c] = ((double)n0 * F.B[0 + c] + (double)n1 * F.B[3 + c]) + (double)n2 * F.B[6 + c];
}

__device__ __forceinline__ bool in_shell(const Frame& F, const double fw[3], int n0, int n1, int n2) {
  double a = fw[0] + n0, b = fw[1] + n1, c = fw[2] + n2;
  return a >= -F.g[0] && a < 1.0 + F.g[0] && b >= -F.g[1] && b < 1.0 + F.g[1] && c >= -F.g[2] &&
         c < 1.0 + F.g[2];
}

__device__ __forceinline__ int cell_of(const Frame& F, const double f[3]) {
  int c[3];
  for (int k = 0; k < 3; k++) {
    int v = (int)floor((f[k] + F.g[k]) / F.cw[k]);
    c[k] = v < 0 ? 0 : (v >= F.nc[k] ? F.nc[k] - 1 : v);
  }
  return F.cell0 + (c[0] * F.nc[1] + c[1]) * F.nc[2] + c[2];
}

__device__ __forceinline__ int find_frame(const Frame* __restrict__ fr, int nframes, int i) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fr[mid].atom0 <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------------------------
// 1. wrap local atoms, validate, count their ghost images
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void wrap_one(int i, int nframes, const Frame* __restrict__ frames, int ntypes,
                                         const double* __restrict__ x, const int* __restrict__ types,
                                         int* __restrict__ frame_of, double* __restrict__ xw,
                                         double* __restrict__ fw, int* __restrict__ gcount,
                                         int* __restrict__ status, int* __restrict__ wk, double* __restrict__ xref) {
#pragma clang fp contract(off)
  int fi = find_frame(frames, nframes, i);
  frame_of[i] = fi;
  const Frame& F = frames[fi];
  double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
  int t = types[i];
  int bad = 0;
  if (t < 0 || t >= ntypes) bad |= ST_BAD_TYPE;
  if (!isfinite(xi[0]) || !isfinite(xi[1]) || !isfinite(xi[2])) bad |= ST_NONFINITE;
  if (bad) {
    atomicOr(&status[STW_FLAGS], bad);
    xi[0] = xi[1] = xi[2] = 0.0;
  }
  double f[3], s[3], w[3], ff[3];
  frac_of(F, xi, f);
  const int m0 = (int)floor(f[0]), m1 = (int)floor(f[1]), m2 = (int)floor(f[2]);
  shift_of(F, m0, m1, m2, s);
  if (wk) {
    wk[3 * i] = m0;
    wk[3 * i + 1] = m1;
    wk[3 * i + 2] = m2;
    for (int c = 0; c < 3; c++) xref[3 * i + c] = xi[c];
  }
  for (int c = 0; c < 3; c++) w[c] = xi[c] - s[c];
  frac_of(F, w, ff);
  for (int c = 0; c < 3; c++) {
    xw[3 * i + c] = w[c];
    fw[3 * i + c] = ff[c];
  }
  int cnt = 0;
  for (int a = -F.Kg[0]; a <= F.Kg[0]; a++)
    for (int b = -F.Kg[1]; b <= F.Kg[1]; b++)
      for (int c = -F.Kg[2]; c <= F.Kg[2]; c++)
        if ((a | b | c) != 0 && in_shell(F, ff, a, b, c)) cnt++;
  gcount[i] = cnt;
}

__global__ __launch_bounds__(256) void k_wrap(int n, int nframes, const Frame* __restrict__ frames,
                                              int ntypes, const double* __restrict__ x,
                                              const int* __restrict__ types,
                                              int* __restrict__ frame_of,
                                              double* __restrict__ xw, double* __restrict__ fw,
                                              int* __restrict__ gcount, int* __restrict__ status,
                                              const int* __restrict__ gate, int* __restrict__ wk,
                                              double* __restrict__ xref, double* __restrict__ npt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (gate && *gate == 0)) return;
  // isobaric MD: the reference positions written here belong to the current box scale
  if (npt && i == 0) npt[NS_LAMB] = npt[NS_LAM];
  wrap_one(i, nframes, frames, ntypes, x, types, frame_of, xw, fw, gcount, status, wk, xref);
}

// ------------------------------------------------------------------------------------
// 2. write the extended arrays (locals then ghosts) and count cell occupancy
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void ghost_emit_one(
    int i, int n, int ntypes, int ghost_cap, const Frame* __restrict__ frames, const int* __restrict__ frame_of,
    const int* __restrict__ types, const double* __restrict__ xw, const double* __restrict__ fw,
    int q, double* __restrict__ xe,
    int* __restrict__ eown, int* __restrict__ eimg, int* __restrict__ etype,
    int* __restrict__ ecell, int* __restrict__ cell_count, int* __restrict__ eabc) {
#pragma clang fp contract(off)
  const Frame& F = frames[frame_of[i]];
  double w[3] = {xw[3 * i], xw[3 * i + 1], xw[3 * i + 2]};
  double f[3] = {fw[3 * i], fw[3 * i + 1], fw[3 * i + 2]};
  int t = types[i];
  if (t < 0 || t >= ntypes) t = 0;  // already flagged as an error by k_wrap
  for (int c = 0; c < 3; c++) xe[3 * i + c] = w[c];
  eown[i] = i;
  eimg[i] = ((F.K[0]) * (2 * F.K[1] + 1) + F.K[1]) * (2 * F.K[2] + 1) + F.K[2];
  etype[i] = t;
  int cl = cell_of(F, f);
  ecell[i] = cl;
  atomicAdd(&cell_count[cl], 1);
  if (eabc) eabc[3 * i] = eabc[3 * i + 1] = eabc[3 * i + 2] = 0;
  for (int a = -F.Kg[0]; a <= F.Kg[0]; a++)
    for (int b = -F.Kg[1]; b <= F.Kg[1]; b++)
      for (int c = -F.Kg[2]; c <= F.Kg[2]; c++) {
        if ((a | b | c) == 0 || !in_shell(F, f, a, b, c)) continue;
        if (q < ghost_cap) {
          int e = n + q;
          double s[3];
          shift_of(F, a, b, c, s);
          for (int k = 0; k < 3; k++) xe[3 * e + k] = w[k] + s[k];
          eown[e] = i;
          bool codeok = a >= -F.K[0] && a <= F.K[0] && b >= -F.K[1] && b <= F.K[1] &&
                        c >= -F.K[2] && c <= F.K[2];
          eimg[e] = codeok ? ((a + F.K[0]) * (2 * F.K[1] + 1) + (b + F.K[1])) * (2 * F.K[2] + 1) +
                                 (c + F.K[2])
                           : -1;
          etype[e] = t;
          if (eabc) {
            eabc[3 * e] = a;
            eabc[3 * e + 1] = b;
            eabc[3 * e + 2] = c;
          }
          double fg[3] = {f[0] + a, f[1] + b, f[2] + c};
          int cg = cell_of(F, fg);
          ecell[e] = cg;
          atomicAdd(&cell_count[cg], 1);
        }
        q++;
      }
}

__global__ __launch_bounds__(256) void k_ghost_emit(
    int n, int ntypes, int ghost_cap, const Frame* __restrict__ frames, const int* __restrict__ frame_of,
    const int* __restrict__ types, const double* __restrict__ xw, const double* __restrict__ fw,
    const int* __restrict__ goff, const int* __restrict__ gtotal, double* __restrict__ xe,
    int* __restrict__ eown, int* __restrict__ eimg, int* __restrict__ etype,
    int* __restrict__ ecell, int* __restrict__ cell_count, int* __restrict__ status,
    const int* __restrict__ gate, int* __restrict__ eabc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (gate && *gate == 0)) return;
  if (i == 0 && gtotal[0] > ghost_cap) {
    atomicOr(&status[STW_FLAGS], ST_GHOST_CAP);
    atomicMax(&status[STW_GHOSTS], gtotal[0]);
  }
  ghost_emit_one(i, n, ntypes, ghost_cap, frames, frame_of, types, xw, fw, goff[i], xe, eown, eimg, etype, ecell,
                 cell_count, eabc);
}

// Systems of at most kOneTile atoms and kCellScanCap cells skip the two scan launches:
// every block of the ghost pass sums the ghost counts of the atoms before its own and
// scans its 256 in registers, and every block of the cell pass scans all cell counts in
// LDS (block 0 also stores them for the list kernels).  The redundant sums cost a few
// KB of L2 reads per block on a rebuild; a step without one saves two launches.
constexpr int kCellScanCap = 8192;

// exclusive scan of one value per thread over a 256-thread block; *total gets the sum
__device__ __forceinline__ int block_scan256(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int pre = 0;
  for (int k = 0; k < w; k++) pre += wsum[k];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return pre + incl - v;
}

__global__ __launch_bounds__(256) void k_ghost_emit_scan(
    int n, int ntypes, int ghost_cap, const Frame* __restrict__ frames, const int* __restrict__ frame_of,
    const int* __restrict__ types, const double* __restrict__ xw, const double* __restrict__ fw,
    const int* __restrict__ gcount, int* __restrict__ gtotal, double* __restrict__ xe,
    int* __restrict__ eown, int* __restrict__ eimg, int* __restrict__ etype,
    int* __restrict__ ecell, int* __restrict__ cell_count, int* __restrict__ status,
    const int* __restrict__ gate, int* __restrict__ eabc) {
  if (gate && *gate == 0) return;
  __shared__ int wsum[4];
  const int t = threadIdx.x, b0 = blockIdx.x * 256, i = b0 + t;
  int part = 0;
  {
    // b0 is a multiple of 256 and gcount is 16-byte aligned (checked at launch):
    // 16-byte loads, four in flight per thread
    const int4* g4 = (const int4*)gcount;
    const int nq = b0 >> 2;
#pragma unroll 4
    for (int j = t; j < nq; j += 256) {
      const int4 v = g4[j];
      part += (v.x + v.y) + (v.z + v.w);
    }
  }
  int base;
  (void)block_scan256(part, wsum, &base);
  const int c = i < n ? gcount[i] : 0;
  int btot;
  const int q = base + block_scan256(c, wsum, &btot);
  if (blockIdx.x == gridDim.x - 1 && t == 0) {
    const int g = base + btot;
    gtotal[0] = g;
    if (g > ghost_cap) {
      atomicOr(&status[STW_FLAGS], ST_GHOST_CAP);
      atomicMax(&status[STW_GHOSTS], g);
    }
  }
  if (i >= n) return;
  ghost_emit_one(i, n, ntypes, ghost_cap, frames, frame_of, types, xw, fw, q, xe, eown, eimg, etype, ecell,
                 cell_count, eabc);
}

// n_ext = n + min(ghost total, ghost_cap) (ghosts beyond the capacity were not
// emitted), written by thread 0; then every extended atom is placed in its cell.
__global__ __launch_bounds__(256) void k_cell_place(int n, int ghost_cap, const int* __restrict__ gtotal,
                                                    int* __restrict__ n_ext,
                                                    const int* __restrict__ ecell,
                                                    const int* __restrict__ cell_start,
                                                    int* __restrict__ cell_fill,
                                                    int* __restrict__ cell_atoms,
                                                    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int g = gtotal[0];
  const int ne = n + (g < ghost_cap ? g : ghost_cap);
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) n_ext[0] = ne;
  if (e >= ne) return;
  int c = ecell[e];
  int p = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + p] = e;
}

// k_cell_place with the scan of the ncs = ncell + 1 cell counts done by every block in LDS
__global__ __launch_bounds__(256) void k_cell_place_scan(int n, int ghost_cap, const int* __restrict__ gtotal,
                                                         int* __restrict__ n_ext, int ncs,
                                                         const int* __restrict__ cell_count,
                                                         int* __restrict__ cell_start, int* __restrict__ ctotal,
                                                         const int* __restrict__ ecell,
                                                         int* __restrict__ cell_fill,
                                                         int* __restrict__ cell_atoms,
                                                         const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int cs[kCellScanCap];
  __shared__ int wsum[4];
  const int t = threadIdx.x;
  const int per = (ncs + 255) / 256, lo = t * per;
  int tot = 0;
  for (int k = 0; k < per; k++) {
    const int qc = lo + k;
    if (qc < ncs) {
      cs[qc] = tot;
      tot += cell_count[qc];
    }
  }
  int all;
  const int ex = block_scan256(tot, wsum, &all);
  for (int k = 0; k < per; k++) {
    const int qc = lo + k;
    if (qc < ncs) cs[qc] += ex;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int qc = t; qc < ncs; qc += 256) cell_start[qc] = cs[qc];
    if (t == 0) ctotal[0] = all;
  }
  const int g = gtotal[0];
  const int ne = n + (g < ghost_cap ? g : ghost_cap);
  const int e = blockIdx.x * 256 + t;
  if (e == 0) n_ext[0] = ne;
  if (e >= ne) return;
  const int c = ecell[e];
  const int p = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cs[c] + p] = e;
}

// ------------------------------------------------------------------------------------
// 3. formatted neighbour list: one wave per local atom
// ------------------------------------------------------------------------------------
__global__ void k_fill_int(int n, int* __restrict__ p, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

constexpr int kNlWaves = 4;
constexpr int kNlCap = 256;    // candidates within rc staged in LDS by the main kernels
constexpr int kVCap = 512;     // candidates within rc + skin sorted in LDS when Verlet rows are built
constexpr int kSecondPassBlocks = 256;   // grid of the exact second formatting pass (strides over *nbig)

// one candidate in LDS: the 128-bit sort key (species, r^2, owner * nimg + image) as two
// words compared lexicographically: hi = species << 56 | (bits of r^2) >> 8,
// lo = (low 8 bits of r^2) << 56 | owner * nimg + image.  r^2 > 0, so its IEEE bits
// order like its value, and the key is exact (no quantisation of r^2).
struct NlEnt {
  unsigned long long hi, lo;
};

// LDS rows of one wave.  k holds a 32-bit key per candidate, species << 28 | r^2
// quantised to 28 bits (floor(r^2 2^28 / rc^2), non-decreasing in r^2): distinct keys
// order the candidates exactly as the full key does.
struct NlRows {
  NlEnt* ent;
  int* e;
  unsigned* k;
  double qs;   // 2^28 / rc^2
};

// Append the candidates of one 64-wide batch that lie within the cutoff to the wave's
// LDS rows (up to cap); returns the new candidate count (which may exceed cap).
// full 128-bit key of candidate e at distance^2 r2
__device__ __forceinline__ NlEnt nl_key(double r2, int e, const Frame& F, const int* __restrict__ eown,
                                        const int* __restrict__ eimg, const int* __restrict__ etype) {
  const unsigned long long rb = (unsigned long long)__double_as_longlong(r2);
  NlEnt k;
  k.hi = ((unsigned long long)etype[e] << 56) | (rb >> 8);
  k.lo = (rb << 56) | ((unsigned long long)(eown[e] - F.atom0) * (unsigned)F.nimg + (unsigned)eimg[e]);
  return k;
}

// r^2 of the pair (xi, e), in the one evaluation order every list decision uses
// (contraction off, as in the candidate gathers)
__device__ __forceinline__ double nl_r2(const double* __restrict__ xe, int e, const double (&xi)[3]) {
#pragma clang fp contract(off)
  const double d0 = xe[3 * e] - xi[0], d1 = xe[3 * e + 1] - xi[1], d2 = xe[3 * e + 2] - xi[2];
  return (d0 * d0 + d1 * d1) + d2 * d2;
}

// the same r^2 from a packed record: p = (x, y), q = (z, species)
__device__ __forceinline__ double nl_r2q(const double2 p, const double2 q, const double (&xi)[3]) {
#pragma clang fp contract(off)
  const double d0 = p.x - xi[0], d1 = p.y - xi[1], d2 = q.x - xi[2];
  return (d0 * d0 + d1 * d1) + d2 * d2;
}

// Append the candidates of one 64-wide batch that lie within the cutoff to the wave's
// LDS rows (up to cap); returns the new candidate count (which may exceed cap).  With
// 32-bit keys (the main pass) only the key and the index are stored; the full key is
// built later, and only if two 32-bit keys tie.
__device__ __forceinline__ int nl_append(bool keep, double r2, int e, int ncand, int lane, const Frame& F,
                                         const int* __restrict__ eown, const int* __restrict__ eimg,
                                         const int* __restrict__ etype, NlRows rows, int cap) {
  unsigned long long bal = __ballot(keep);
  int pos = ncand + __popcll(bal & ((1ull << lane) - 1ull));
  if (keep && pos < cap) {
    rows.e[pos] = e;
    if (rows.k) rows.k[pos] = ((unsigned)etype[e] << 28) | (unsigned)fmin(r2 * rows.qs, 268435455.0);
    else rows.ent[pos] = nl_key(r2, e, F, eown, eimg, etype);
  }
  return ncand + __popcll(bal);
}

// x precedes y in (species, r^2, owner, image) order
__device__ __forceinline__ int nl_before(const NlEnt& x, const NlEnt& y) {
  return (x.hi < y.hi) | ((x.hi == y.hi) & (x.lo < y.lo));
}

// rk[h] = number of 32-bit keys below that of candidate lane + 64 h (h < NH); every lane
// reads the same four keys per LDS access (broadcast)
typedef unsigned u32x4n __attribute__((ext_vector_type(4)));
template <int NH>
__device__ __forceinline__ void nl_rank32(const unsigned* K, int ncand, int lane, int (&rk)[4]) {
  unsigned y[NH];
#pragma unroll
  for (int h = 0; h < NH; h++) {
    const int q = lane + 64 * h;
    y[h] = q < ncand ? K[q] : 0u;
  }
  int r[NH];
#pragma unroll
  for (int h = 0; h < NH; h++) r[h] = 0;
  int u = 0;
  for (; u + 4 <= ncand; u += 4) {
    const u32x4n x = *(const u32x4n*)(K + u);
#pragma unroll
    for (int h = 0; h < NH; h++) r[h] += (int)(x[0] < y[h]) + (int)(x[1] < y[h]) + (int)(x[2] < y[h]) + (int)(x[3] < y[h]);
  }
  for (; u < ncand; u++) {
    const unsigned x = K[u];
#pragma unroll
    for (int h = 0; h < NH; h++) r[h] += (int)(x < y[h]);
  }
#pragma unroll
  for (int h = 0; h < 4; h++) rk[h] = h < NH ? r[h] : 0;
}

// Ascending bitonic sort of the wave's 64 K (key, value) pairs, element i = 64 k + lane
// (pads carry key 0xffffffff and sort to the end).  The network is fixed, so equal keys
// end in a deterministic order; a pair exchanges only on a strict inequality, so the
// values stay a permutation.
template <int K>
__device__ __forceinline__ void wave_bitonic(unsigned (&key)[K], int (&val)[K], int lane) {
  constexpr int N = 64 * K;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int jr = j >> 6;
#pragma unroll
        for (int k = 0; k < K; k++) {
          const int kp = k ^ jr;
          if (kp > k) {
            const bool up = ((64 * k + lane) & size) == 0;
            const bool sw = up ? key[kp] < key[k] : key[kp] > key[k];
            const unsigned a = key[k], b = key[kp];
            const int va = val[k], vb = val[kp];
            key[k] = sw ? b : a;
            key[kp] = sw ? a : b;
            val[k] = sw ? vb : va;
            val[kp] = sw ? va : vb;
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; k++) {
          const unsigned pk = __shfl_xor(key[k], j, 64);
          const int pv = __shfl_xor(val[k], j, 64);
          const bool up = ((64 * k + lane) & size) == 0;
          const bool lower = (lane & j) == 0;
          const bool take = (lower == up) ? pk < key[k] : pk > key[k];
          key[k] = take ? pk : key[k];
          val[k] = take ? pv : val[k];
        }
      }
    }
  }
}

// Sort the staged (32-bit key, index) rows of one wave (cnt <= 64 K) and write the
// indices in key order to out[0, min(cnt, lim))
template <int K>
__device__ __forceinline__ void wave_sort_rows(const unsigned* sk, const int* se, int cnt, int lane, int* out,
                                               int lim) {
  unsigned key[K];
  int val[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int q = 64 * k + lane;
    key[k] = q < cnt ? sk[q] : 0xffffffffu;
    val[k] = q < cnt ? se[q] : -1;
  }
  wave_bitonic<K>(key, val, lane);
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int q = 64 * k + lane;
    if (q < cnt && q < lim) out[q] = val[k];
  }
}

// Rank the staged candidates of atom i by (species, r^2, owner, image) and write its
// formatted row: per-species blocks of width sel, nearest first, -1 pads (Alg. 1).
// Returns false, having written nothing, when 32-bit keys tie and the rows have no room
// for the full keys (the caller defers the atom to the pass that has).
__device__ __forceinline__ bool nl_format(int i, int ncand, const ModelC& m, NlRows rows, int lane,
                                          int* __restrict__ nlist, int* __restrict__ nnei,
                                          int* __restrict__ status, const Frame& F,
                                          const double* __restrict__ xe, const int* __restrict__ eown,
                                          const int* __restrict__ eimg, const int* __restrict__ etype) {
  if (ncand > kMaxCand) {
    if (lane == 0) {
      atomicOr(&status[STW_FLAGS], ST_CAPACITY);
      atomicMax(&status[STW_MAX_CAND], ncand);
    }
    ncand = kMaxCand;
  }
  // the LDS rows are private to this wave: order its writes before its reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int tcnt[kMaxTypes];
#pragma unroll
  for (int t = 0; t < kMaxTypes; t++) tcnt[t] = 0;
  for (int q = lane; q < ncand; q += 64) {
    int ty = rows.k ? (int)(rows.k[q] >> 28) : (int)(rows.ent[q].hi >> 56);
#pragma unroll
    for (int t = 0; t < kMaxTypes; t++) tcnt[t] += (ty == t);
  }
#pragma unroll
  for (int t = 0; t < kMaxTypes; t++) {
    int v = tcnt[t];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    tcnt[t] = v;
  }
  // rank sort: position of each candidate in (species, r2, owner, image) order; the rank
  // within its species block is that minus the candidates of the smaller species.  A lane
  // ranks two candidates per pass over the rows (every lane reads the same entry: LDS
  // broadcast).
  int* nl = nlist + (size_t)i * m.nm;
  int ovf = 0;
  // Fast path (up to 256 candidates): rank by the 32-bit keys, four candidates per lane.
  // With distinct keys the ranks are a permutation and sum to n (n - 1) / 2; a tie lowers
  // the sum, and then the exact 128-bit ranking below runs instead.
  if (rows.k && ncand <= 256) {
    const int nh = (ncand + 63) >> 6;
    int rk[4];
    if (nh <= 1) nl_rank32<1>(rows.k, ncand, lane, rk);
    else if (nh == 2) nl_rank32<2>(rows.k, ncand, lane, rk);
    else if (nh == 3) nl_rank32<3>(rows.k, ncand, lane, rk);
    else nl_rank32<4>(rows.k, ncand, lane, rk);
    int sum = 0;
#pragma unroll
    for (int h = 0; h < 4; h++) sum += (lane + 64 * h < ncand) ? rk[h] : 0;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if (sum == ncand * (ncand - 1) / 2) {
#pragma unroll
      for (int h = 0; h < 4; h++) {
        const int q = lane + 64 * h;
        if (q >= ncand) break;
        const unsigned t = rows.k[q] >> 28;
        int below = 0;
#pragma unroll
        for (int tt = 0; tt < kMaxTypes; tt++) below += (tt < (int)t) ? tcnt[tt] : 0;
        const int rank = rk[h] - below;
        if (rank < m.sel[t]) nl[m.sel_off[t] + rank] = rows.e[q];
        else ovf = 1;
      }
      ncand = 0;   // formatted: skip the exact ranking
    } else {
      // tied keys: build the full keys for the exact ranking
      if (!rows.ent) return false;
      const double xi[3] = {xe[3 * i], xe[3 * i + 1], xe[3 * i + 2]};
      for (int q = lane; q < ncand; q += 64) {
        const int e = rows.e[q];
        rows.ent[q] = nl_key(nl_r2(xe, e, xi), e, F, eown, eimg, etype);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  for (int q0 = lane; q0 < ncand; q0 += 128) {
    const int q1 = q0 + 64;
    const bool has1 = q1 < ncand;
    const NlEnt y0 = rows.ent[q0];
    const NlEnt y1 = has1 ? rows.ent[q1] : y0;
    int r0 = 0, r1 = 0, u = 0;
    for (; u + 4 <= ncand; u += 4) {
      const NlEnt x0 = rows.ent[u], x1 = rows.ent[u + 1], x2 = rows.ent[u + 2], x3 = rows.ent[u + 3];
      r0 += nl_before(x0, y0) + nl_before(x1, y0) + nl_before(x2, y0) + nl_before(x3, y0);
      r1 += nl_before(x0, y1) + nl_before(x1, y1) + nl_before(x2, y1) + nl_before(x3, y1);
    }
    for (; u < ncand; u++) {
      const NlEnt x = rows.ent[u];
      r0 += nl_before(x, y0);
      r1 += nl_before(x, y1);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
      if (h == 1 && !has1) break;
      const NlEnt& y = h ? y1 : y0;
      const unsigned t = (unsigned)(y.hi >> 56);
      int below = 0;   // candidates of smaller species
#pragma unroll
      for (int tt = 0; tt < kMaxTypes; tt++) below += (tt < (int)t) ? tcnt[tt] : 0;
      const int rank = (h ? r1 : r0) - below;
      if (rank < m.sel[t]) nl[m.sel_off[t] + rank] = rows.e[h ? q1 : q0];
      else ovf = 1;
    }
  }
  // pads
  for (int k = lane; k < m.nm; k += 64) {
    int t = 0;
    while (t + 1 < m.ntypes && k >= m.sel_off[t + 1]) t++;
    int pos = k - m.sel_off[t];
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < kMaxTypes; u++) cnt = (u == t) ? tcnt[u] : cnt;
    int real = cnt < m.sel[t] ? cnt : m.sel[t];
    if (pos >= real) nl[k] = -1;
  }
#pragma unroll
  for (int t = 0; t < kMaxTypes; t++)
    if (lane == t && t < m.ntypes)
      nnei[(size_t)i * m.ntypes + t] = tcnt[t] < m.sel[t] ? tcnt[t] : m.sel[t];
  unsigned long long anyovf = __ballot(ovf);
  if (anyovf && lane == 0) {
    atomicOr(&status[STW_FLAGS], ST_SEL_OVERFLOW);
    atomicAdd(&status[STW_SEL_ROWS], 1);
  }
  return true;
}

// Candidates of atom i in the 27 cells around its own: those with r^2 < rcut2 are
// appended to the LDS rows (LIST = false) or written to the Verlet row vrow (LIST = true).
// The cells' members are taken as one index space (cells in (a, b, c) order, members in
// cell order), 64 lanes per batch and four batches in flight, so the short cells do not
// each cost a batch and a round of dependent loads.
template <bool LIST>
__device__ __forceinline__ int nl_gather_cells(int i, const Frame& F, double rcut2, const double* __restrict__ xe,
                                               const int* __restrict__ eown, const int* __restrict__ eimg,
                                               const int* __restrict__ etype, const int* __restrict__ ecell,
                                               const int* __restrict__ cell_start,
                                               const int* __restrict__ cell_atoms, int lane, NlRows rows, int cap,
                                               int* vrow, int vcap, int& too_close) {
#pragma clang fp contract(off)
  const double xi0 = xe[3 * i], xi1 = xe[3 * i + 1], xi2 = xe[3 * i + 2];
  const int ci = ecell[i] - F.cell0;
  const int c2 = ci % F.nc[2], c1 = (ci / F.nc[2]) % F.nc[1], c0 = ci / (F.nc[2] * F.nc[1]);
  // lane q < 27: member range of cell q = (c0 - 1 + q / 9, c1 - 1 + q / 3 % 3, c2 - 1 + q % 3)
  int cb = 0, cn = 0;
  if (lane < 27) {
    const int a = c0 - 1 + lane / 9, b = c1 - 1 + (lane / 3) % 3, c = c2 - 1 + lane % 3;
    if (a >= 0 && a < F.nc[0] && b >= 0 && b < F.nc[1] && c >= 0 && c < F.nc[2]) {
      const int cell = F.cell0 + (a * F.nc[1] + b) * F.nc[2] + c;
      cb = cell_start[cell];
      cn = cell_start[cell + 1] - cb;
    }
  }
  int incl = cn;
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const int total = __shfl(incl, 26, 64);
  const int excl = incl - cn;   // first flattened index of cell q (non-decreasing in q)
  int ncand = 0;
  for (int p0 = 0; p0 < total; p0 += 256) {
    int e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int p = p0 + 64 * j + lane;
      // the cell holding p: the last q < 27 with excl[q] <= p (all lanes take part)
      int q = 0, exq = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1) {
        const int t = q + step;
        const int ex = __shfl(excl, t < 27 ? t : 26, 64);
        if (t < 27 && ex <= p) {
          q = t;
          exq = ex;
        }
      }
      const int cbq = __shfl(cb, q, 64);
      e[j] = p < total ? cell_atoms[cbq + (p - exq)] : -1;
    }
    double d[4][3];
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (e[j] >= 0) {
        d[j][0] = xe[3 * e[j]];
        d[j][1] = xe[3 * e[j] + 1];
        d[j][2] = xe[3 * e[j] + 2];
      }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (p0 + 64 * j >= total) break;   // uniform over the wave
      bool keep = false;
      double r2 = 0.0;
      if (e[j] >= 0) {
        const double d0 = d[j][0] - xi0, d1 = d[j][1] - xi1, d2 = d[j][2] - xi2;
        r2 = (d0 * d0 + d1 * d1) + d2 * d2;
        keep = (r2 < rcut2) && (e[j] != i);
        if (keep && r2 < 1e-12) too_close = 1;
      }
      if constexpr (LIST) {
        unsigned long long bal = __ballot(keep);
        int pos = ncand + __popcll(bal & ((1ull << lane) - 1ull));
        if (keep && pos < vcap) vrow[pos] = e[j];
        ncand += __popcll(bal);
      } else {
        ncand = nl_append(keep, r2, e[j], ncand, lane, F, eown, eimg, etype, rows, cap);
      }
    }
  }
  return ncand;
}

// Candidates of atom i from its Verlet row (pairs within rc + skin at the last build),
// at the current coordinates; the row is read four batches of 64 at a time so that the
// dependent loads (row entry, then coordinates) of the batches overlap.
__device__ __forceinline__ int nl_gather_verlet(int i, const Frame& F, double rc2, const double* __restrict__ xe,
                                                const int* __restrict__ eown, const int* __restrict__ eimg,
                                                const int* __restrict__ etype, const int* __restrict__ vrow,
                                                int cnt, int lane, NlRows rows, int cap) {
#pragma clang fp contract(off)
  const double xi0 = xe[3 * i], xi1 = xe[3 * i + 1], xi2 = xe[3 * i + 2];
  int ncand = 0;
  for (int p0 = 0; p0 < cnt; p0 += 256) {
    int e[4];
    double d[4][3];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int p = p0 + 64 * j + lane;
      e[j] = p < cnt ? vrow[p] : -1;
    }
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (e[j] >= 0) {
        d[j][0] = xe[3 * e[j]];
        d[j][1] = xe[3 * e[j] + 1];
        d[j][2] = xe[3 * e[j] + 2];
      }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (p0 + 64 * j >= cnt) break;   // uniform over the wave
      bool keep = false;
      double r2 = 0.0;
      if (e[j] >= 0) {
        const double d0 = d[j][0] - xi0, d1 = d[j][1] - xi1, d2 = d[j][2] - xi2;
        r2 = (d0 * d0 + d1 * d1) + d2 * d2;
        keep = r2 < rc2;
      }
      ncand = nl_append(keep, r2, e[j], ncand, lane, F, eown, eimg, etype, rows, cap);
    }
  }
  return ncand;
}

struct NlKArgs {
  int n;
  ModelC m;
  const Frame* frames;
  const int* frame_of;
  const double* xe;
  const int *eown, *eimg, *etype, *ecell, *cell_start, *cell_atoms;
  const int *vlist, *vcnt;   // Verlet rows (NULL: search the cells)
  const double* xq;          // packed [x, y, z, species] records (per-step filter)
  int vcap;
  int *nlist, *nnei, *status;
  int *big, *nbig;           // atoms deferred to the second pass (more than kNlCap candidates,
                             // or tied 32-bit keys); *nbig is zero on entry and left zero
  int* big_done;             // second-pass blocks finished (zero on entry, left zero)
  int *gate, *clear;         // per-step filter: re-armed (zeroed) by its first thread, or NULL
};

// Formatted list, one wave per atom.  CAP = kNlCap: the main pass with 32-bit keys only
// (atoms with more candidates, or with tied keys, are deferred to the list big);
// CAP = kMaxCand: the second pass over that list with the full keys (a fixed grid
// striding over *nbig entries; its last block to finish clears *nbig).
template <int CAP>
__global__ __launch_bounds__(64 * kNlWaves) void k_nlist(NlKArgs A) {
  constexpr bool kMain = CAP <= kNlCap;
  __shared__ NlEnt s_ent[kNlWaves][kMain ? 1 : CAP];
  __shared__ int s_e[kNlWaves][CAP];
  __shared__ __align__(16) unsigned s_k[kNlWaves][kMain ? CAP : 4];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const NlRows rows{kMain ? nullptr : s_ent[wv], s_e[wv], kMain ? s_k[wv] : nullptr, 268435456.0 / A.m.rc2};
  const bool second = CAP > kNlCap;
  const int nwork = second ? *A.nbig : A.n;
  const int stride = second ? gridDim.x * kNlWaves : nwork;
  for (int w = blockIdx.x * kNlWaves + wv; w < nwork; w += stride) {
    const int i = second ? A.big[w] : w;
    const Frame& F = A.frames[A.frame_of[i]];
    int too_close = 0, ncand;
    if (A.vlist)
      ncand = nl_gather_verlet(i, F, A.m.rc2, A.xe, A.eown, A.eimg, A.etype, A.vlist + (size_t)i * A.vcap,
                               A.vcnt[i], lane, rows, CAP);
    else
      ncand = nl_gather_cells<false>(i, F, A.m.rc2, A.xe, A.eown, A.eimg, A.etype, A.ecell, A.cell_start,
                                     A.cell_atoms, lane, rows, CAP, nullptr, 0, too_close);
    if (too_close) atomicOr(&A.status[STW_FLAGS], ST_OVERLAP);
    if (!second && ncand > CAP) {
      if (lane == 0) A.big[atomicAdd(A.nbig, 1)] = i;
      continue;
    }
    if (!nl_format(i, ncand, A.m, rows, lane, A.nlist, A.nnei, A.status, F, A.xe, A.eown, A.eimg, A.etype) &&
        lane == 0)
      A.big[atomicAdd(A.nbig, 1)] = i;
  }
  if (second && nwork > 0) {
    // every block has read *nbig; the last one to finish leaves both counters zero (with no
    // deferred atom there is nothing to reset, and no block pays for the fence)
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(A.big_done, 1) == (int)gridDim.x - 1) {
        *A.nbig = 0;
        *A.big_done = 0;
      }
    }
  }
}

// Verlet candidate rows: every extended atom within rl of atom i (rl = rc + skin),
// rebuilt only when *gate != 0.  Rows of up to kVCap candidates are stored sorted by
// (species, r^2 at the build) through 32-bit keys (a bitonic network); larger rows are
// stored in cell order (the per-step pass then defers their atoms to the exact ranking).
__device__ __forceinline__ void vbuild_wave(
    int i, int lane, int* s_e, unsigned* s_k, double rl2, const Frame* __restrict__ frames,
    const int* __restrict__ frame_of, const double* __restrict__ xe, const int* __restrict__ etype,
    const int* __restrict__ ecell, const int* __restrict__ cell_start, const int* __restrict__ cell_atoms,
    int* __restrict__ vlist, int* __restrict__ vcnt, int vcap, int* __restrict__ status) {
  const Frame& F = frames[frame_of[i]];
  int* vrow = vlist + (size_t)i * vcap;
  int too_close = 0;
  const NlRows rows{nullptr, s_e, s_k, 268435456.0 / rl2};
  int cnt = nl_gather_cells<false>(i, F, rl2, xe, nullptr, nullptr, etype, ecell, cell_start, cell_atoms, lane, rows,
                                   kVCap, nullptr, 0, too_close);
  if (cnt <= kVCap) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int lim = cnt < vcap ? cnt : vcap;
    if (cnt <= 64) wave_sort_rows<1>(s_k, s_e, cnt, lane, vrow, lim);
    else if (cnt <= 128) wave_sort_rows<2>(s_k, s_e, cnt, lane, vrow, lim);
    else if (cnt <= 256) wave_sort_rows<4>(s_k, s_e, cnt, lane, vrow, lim);
    else wave_sort_rows<8>(s_k, s_e, cnt, lane, vrow, lim);
  } else {
    too_close = 0;
    cnt = nl_gather_cells<true>(i, F, rl2, xe, nullptr, nullptr, nullptr, ecell, cell_start, cell_atoms, lane,
                                NlRows{nullptr, nullptr, nullptr, 0.0}, 0, vrow, vcap, too_close);
  }
  if (too_close) atomicOr(&status[STW_FLAGS], ST_OVERLAP);
  if (lane == 0) {
    vcnt[i] = cnt < vcap ? cnt : vcap;
    if (cnt > vcap) {
      atomicOr(&status[STW_FLAGS], ST_CAPACITY);
      atomicMax(&status[STW_MAX_CAND], cnt);
    }
  }
}

__global__ __launch_bounds__(64 * kNlWaves) void k_vbuild(
    int n, double rl2, const Frame* __restrict__ frames, const int* __restrict__ frame_of,
    const double* __restrict__ xe, const int* __restrict__ etype, const int* __restrict__ ecell,
    const int* __restrict__ cell_start, const int* __restrict__ cell_atoms, int* __restrict__ vlist,
    int* __restrict__ vcnt, int vcap, int* __restrict__ status, const int* __restrict__ gate) {
  __shared__ int s_e[kNlWaves][kVCap];
  __shared__ __align__(16) unsigned s_k[kNlWaves][kVCap];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * kNlWaves + wv;
  if (i >= n || (gate && *gate == 0)) return;
  vbuild_wave(i, lane, s_e[wv], s_k[wv], rl2, frames, frame_of, xe, etype, ecell, cell_start, cell_atoms, vlist,
              vcnt, vcap, status);
}

// Per-step list from sorted Verlet rows (MD): the row's candidates still within rc,
// in the row's order (species, then r^2 at the last build), compacted into the species
// blocks; -1 pads.  At a build step this is the order of Alg. 1 (up to ties within the
// 28-bit key); between builds the order is the build's, which changes the descriptor
// only by summation order (Eq. 4 sums over neighbours).  An atom whose row is unsorted
// (more than kVCap candidates) or where a species has more than sel neighbours within
// rc (the nearest sel must then be chosen at the current distances) is deferred to the
// exact second pass.
// Workgroups are dealt to the 8 XCDs round robin (block b on XCD b % 8), each XCD with its
// own L2: the grid is a multiple of 8 and block b takes the atoms of logical block
// (b % 8) (grid / 8) + b / 8, so each XCD filters a contiguous range of atoms, whose
// candidates' coordinates largely coincide and stay in its L2.  NTY > 0 fixes the number of
// species at compile time (the per-species loops then carry no bounds checks); NTY = 0
// takes it from the model, up to kMaxTypes.
template <int NTY>
__global__ __launch_bounds__(64 * kNlWaves) void k_nlist_vstep(NlKArgs A) {
  constexpr int TT = NTY > 0 ? NTY : kMaxTypes;
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int lb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int i = lb * kNlWaves + wv;
  if (i == 0 && lane == 0) {
    // the rebuild (if any) and the refresh are done: the next step's check sets the flag
    if (A.gate) *A.gate = 0;
    if (A.clear) *A.clear = 0;
  }
  if (i >= A.n) return;
  const ModelC& m = A.m;
  const int* vrow = A.vlist + (size_t)i * A.vcap;
  // The first 256 slots of the row are loaded with the count (slots past it are read,
  // clamped into the row, and dropped) and the coordinates and species of the candidates
  // are gathered together, so that an atom costs two dependent memory round trips, not
  // four.  Each candidate is one aligned 32-byte record (two 16-byte loads from one cache
  // line): the gathers are scattered, and their cost is the number of cache lines each
  // load instruction touches, which separate x, y, z and species loads would double.
  int e[4];
#pragma unroll
  for (int j = 0; j < 4; j++) e[j] = vrow[min(64 * j + lane, A.vcap - 1)];
  const int cnt = A.vcnt[i];
  if (cnt > kVCap) {
    if (lane == 0) A.big[atomicAdd(A.nbig, 1)] = i;
    return;
  }
  const double xi[3] = {A.xe[3 * i], A.xe[3 * i + 1], A.xe[3 * i + 2]};
  int* nl = A.nlist + (size_t)i * m.nm;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int nty = NTY > 0 ? NTY : m.ntypes;
  int tc[TT];
#pragma unroll
  for (int t = 0; t < TT; t++) tc[t] = 0;
  for (int p0 = 0; p0 < cnt; p0 += 256) {
    double r2[4];
    int ty[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int p = p0 + 64 * j + lane;
      if (p0 > 0) e[j] = vrow[min(p, A.vcap - 1)];   // a row longer than 256 (rare)
      if (p >= cnt) e[j] = -1;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int q = e[j] >= 0 ? e[j] : 0;   // in bounds whatever the slot holds
      const double2* rec = reinterpret_cast<const double2*>(A.xq) + 2 * (size_t)q;
      const double2 p = rec[0], s = rec[1];
      const double d2 = nl_r2q(p, s, xi);
      ty[j] = (int)s.y;
      r2[j] = e[j] >= 0 ? d2 : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (p0 + 64 * j >= cnt) break;   // uniform over the wave
      const bool keep = e[j] >= 0 && r2[j] < m.rc2;
      const int t = keep ? ty[j] : -1;
#pragma unroll
      for (int T = 0; T < TT; T++) {
        if (NTY == 0 && T >= nty) break;
        const unsigned long long mk = __ballot(t == T);
        if (t == T) {
          const int pos = tc[T] + __popcll(mk & below);
          if (pos < m.sel[T]) nl[m.sel_off[T] + pos] = e[j];
        }
        tc[T] += __popcll(mk);
      }
    }
  }
  bool ovf = false;
#pragma unroll
  for (int T = 0; T < TT; T++) ovf |= T < nty && tc[T] > m.sel[T];
  if (ovf) {
    if (lane == 0) A.big[atomicAdd(A.nbig, 1)] = i;
    return;
  }
  for (int k = lane; k < m.nm; k += 64) {
    // species block of slot k and its count
    int c = tc[0], o = m.sel_off[0];
#pragma unroll
    for (int u = 1; u < TT; u++)
      if (u < nty && k >= m.sel_off[u]) {
        c = tc[u];
        o = m.sel_off[u];
      }
    if (k - o >= c) nl[k] = -1;
  }
#pragma unroll
  for (int t = 0; t < TT; t++)
    if (lane == t && t < nty) A.nnei[(size_t)i * nty + t] = tc[t];
}

// both passes of the formatted list
static void launch_format(const NlKArgs& K, hipStream_t st) {
  hipLaunchKernelGGL((k_nlist<kNlCap>), dim3((K.n + kNlWaves - 1) / kNlWaves), dim3(64 * kNlWaves), 0, st, K);
  hipLaunchKernelGGL((k_nlist<kMaxCand>), dim3(kSecondPassBlocks), dim3(64 * kNlWaves), 0, st, K);
}

// Extended coordinates at the current positions with the wrap and image integers of
// the last rebuild (the same arithmetic as k_wrap / k_ghost_emit).
__device__ __forceinline__ void update_ext_one(int e, int n, const Frame* __restrict__ frames,
                                               const int* __restrict__ frame_of, const double* __restrict__ x,
                                               const int* __restrict__ wk, const int* __restrict__ eown,
                                               const int* __restrict__ eabc, const int* __restrict__ etype,
                                               double* __restrict__ xe, double* __restrict__ xq) {
#pragma clang fp contract(off)
  int i = eown[e];
  const Frame& F = frames[frame_of[i]];
  double s[3], w[3];
  shift_of(F, wk[3 * i], wk[3 * i + 1], wk[3 * i + 2], s);
  for (int c = 0; c < 3; c++) w[c] = x[3 * i + c] - s[c];
  if (e >= n) {
    double g[3];
    shift_of(F, eabc[3 * e], eabc[3 * e + 1], eabc[3 * e + 2], g);
    for (int c = 0; c < 3; c++) w[c] = w[c] + g[c];
  }
  for (int c = 0; c < 3; c++) xe[3 * e + c] = w[c];
  double2* r = reinterpret_cast<double2*>(xq) + 2 * (size_t)e;
  r[0] = make_double2(w[0], w[1]);
  r[1] = make_double2(w[2], (double)etype[e]);
}

// The launch that follows the (gated) rebuild chain of a Verlet step: with the rebuild
// flag set it builds the Verlet rows, one wave per atom (the ghost pass has just written
// the extended coordinates from the current positions); otherwise it refreshes the
// extended coordinates from the moved atoms, one thread per extended atom.  Both ways it
// writes the packed [x, y, z, species] records that the filter gathers.  The flag is
// only read here; the per-step filter that runs next re-arms it.
__global__ __launch_bounds__(64 * kNlWaves) void k_vbuild_refresh(
    int n, double rl2, const Frame* __restrict__ frames, const int* __restrict__ frame_of,
    double* __restrict__ xe, const int* __restrict__ etype, const int* __restrict__ ecell,
    const int* __restrict__ cell_start, const int* __restrict__ cell_atoms, int* __restrict__ vlist,
    int* __restrict__ vcnt, int vcap, int* __restrict__ status, const int* __restrict__ gate, int ne_cap,
    const int* __restrict__ n_ext, const double* __restrict__ x, const int* __restrict__ wk,
    const int* __restrict__ eown, const int* __restrict__ eabc, double* __restrict__ xq) {
  __shared__ int s_e[kNlWaves][kVCap];
  __shared__ __align__(16) unsigned s_k[kNlWaves][kVCap];
  const int ne = min(ne_cap, n_ext[0]);
  if (*gate != 0) {
    // the ghost pass has written xe and etype: pack them (the grid has 64 threads per atom)
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
      double2* r = reinterpret_cast<double2*>(xq) + 2 * (size_t)e;
      r[0] = make_double2(xe[3 * e], xe[3 * e + 1]);
      r[1] = make_double2(xe[3 * e + 2], (double)etype[e]);
    }
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * kNlWaves + wv;
    if (i >= n) return;
    vbuild_wave(i, lane, s_e[wv], s_k[wv], rl2, frames, frame_of, xe, etype, ecell, cell_start, cell_atoms, vlist,
                vcnt, vcap, status);
    return;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x)
    update_ext_one(e, n, frames, frame_of, x, wk, eown, eabc, etype, xe, xq);
}

// *flag |= 1 when some atom moved more than half the skin since the last rebuild
// (or has a non-finite coordinate).  Also clears the cell counters (nc1 and nc2 ints)
// for the rebuild that may follow; nothing else reads them between rebuilds.
__global__ __launch_bounds__(256) void k_disp(int n, const double* __restrict__ x, const double* __restrict__ xref,
                                              double lim2, int* __restrict__ flag, int nc1, int* __restrict__ c1,
                                              int nc2, int* __restrict__ c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int q = i; q < nc1 || q < nc2; q += gridDim.x * blockDim.x) {
    if (q < nc1) c1[q] = 0;
    if (q < nc2) c2[q] = 0;
  }
  bool moved = false;
  if (i < n) {
    double d0 = x[3 * i] - xref[3 * i], d1 = x[3 * i + 1] - xref[3 * i + 1], d2 = x[3 * i + 2] - xref[3 * i + 2];
    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    moved = !(r2 <= lim2);
  }
  if (__ballot(moved) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ------------------------------------------------------------------------------------
// 4. species-grouped row order for the embedding / fitting kernels
// ------------------------------------------------------------------------------------
// rows: for each species t, its atoms in index order, padded to a multiple of kRowPad.
__global__ void k_type_rows(int n, int ntypes, int W, const int* __restrict__ types,
                            const int* __restrict__ tpos, const int* __restrict__ tcount,
                            int* __restrict__ row_of, int* __restrict__ type_row0,
                            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  // type_row0[t] = sum_{t'<t} roundup(count[t'], kRowPad); computed by every thread
  int r0[kMaxTypes + 1];
  r0[0] = 0;
  for (int t = 0; t < ntypes; t++) r0[t + 1] = r0[t] + (tcount[t] + kRowPad - 1) / kRowPad * kRowPad;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0)
    for (int t = 0; t <= ntypes; t++) type_row0[t] = r0[t];
  if (i >= n) return;
  int t = types[i];
  if (t < 0 || t >= ntypes) t = 0;
  row_of[i] = r0[t] + tpos[(size_t)i * W + t];
}


__global__ void k_fill_int_gated(int n, int* __restrict__ p, int v, const int* __restrict__ gate) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (!gate || *gate != 0)) p[i] = v;
}

__global__ void k_row_atoms(int n, const int* __restrict__ row_of, int* __restrict__ row_atom,
                            const int* __restrict__ gate) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (!gate || *gate != 0)) row_atom[row_of[i]] = i;
}

// debug export of the list as (frame-local owner index, image code)
__global__ void k_nlist_export(int n, int nm, const int* __restrict__ nlist,
                               const int* __restrict__ eown, const int* __restrict__ eimg,
                               const int* __restrict__ frame_of, const Frame* __restrict__ frames,
                               int* __restrict__ out_j, int* __restrict__ out_img) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * nm) return;
  int i = q / nm;
  int e = nlist[q];
  int a0 = frames[frame_of[i]].atom0;
  out_j[q] = e < 0 ? -1 : eown[e] - a0;
  if (out_img) out_img[q] = e < 0 ? -1 : eimg[e];
}

// ------------------------------------------------------------------------------------
// host launch sequence
// ------------------------------------------------------------------------------------
static void fill_int(int n, int* p, int v, const int* gate, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_int_gated, dim3((n + 255) / 256), dim3(256), 0, st, n, p, v, gate);
}

// Full build (every kernel skipped when A.gate points at 0): wrap, ghost images, cell
// list, then either the formatted list (k_nlist) or, with A.vlist, the Verlet rows
// within rc + skin (k_vbuild), and the species-grouped row order.
static NlKArgs format_args(const NlistArgs& A) {
  NlKArgs K{};
  K.n = A.ncentre > 0 ? A.ncentre : A.n;
  K.m = A.m;
  K.frames = A.frames;
  K.frame_of = A.frame_of;
  K.xe = A.xe;
  K.xq = A.xq;
  K.eown = A.eown;
  K.eimg = A.eimg;
  K.etype = A.etype;
  K.ecell = A.ecell;
  K.cell_start = A.cell_start;
  K.cell_atoms = A.cell_atoms;
  K.vlist = A.vlist;
  K.vcnt = A.vcnt;
  K.vcap = A.vcap;
  K.nlist = A.nlist;
  K.nnei = A.nnei;
  K.status = A.status;
  K.big = A.big;
  K.nbig = A.nbig;
  K.big_done = A.nbig + 1;
  return K;
}

// zero two int arrays (cell counts and fill pointers) in one launch
__global__ void k_zero2_gated(int n1, int* __restrict__ p1, int n2, int* __restrict__ p2,
                              const int* __restrict__ gate) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (gate && *gate == 0) return;
  if (i < n1) p1[i] = 0;
  if (i < n2) p2[i] = 0;
}

// the (gated) rebuild chain; rows_later: the Verlet rows are built by the launch that
// follows (k_vbuild_refresh)
static void launch_rebuild(const NlistArgs& A, bool rows_later, hipStream_t st) {
  const int n = A.n;
  const int nb = (n + 255) / 256;
  const int* G = A.gate;
  if (!A.cells_zeroed)
    hipLaunchKernelGGL(k_zero2_gated, dim3((A.ncell + 1 + 255) / 256), dim3(256), 0, st, A.ncell + 1,
                       A.cell_count, A.ncell, A.cell_fill, G);
  hipLaunchKernelGGL(k_wrap, dim3(nb), dim3(256), 0, st, n, A.nframes, A.frames, A.m.ntypes, A.x,
                     A.types, A.frame_of, A.xw, A.fw, A.gcount, A.status, G, A.wk, A.xref, A.npt);
  const int ne_cap = n + A.ghost_cap;
  if (n <= kOneTile && A.ncell + 1 <= kCellScanCap && ((uintptr_t)A.gcount & 15) == 0) {
    hipLaunchKernelGGL(k_ghost_emit_scan, dim3(nb), dim3(256), 0, st, n, A.m.ntypes, A.ghost_cap, A.frames,
                       A.frame_of, A.types, A.xw, A.fw, A.gcount, A.gtotal, A.xe, A.eown, A.eimg, A.etype,
                       A.ecell, A.cell_count, A.status, G, A.eabc);
    hipLaunchKernelGGL(k_cell_place_scan, dim3((ne_cap + 255) / 256), dim3(256), 0, st, n, A.ghost_cap, A.gtotal,
                       A.n_ext, A.ncell + 1, A.cell_count, A.cell_start, A.ctotal, A.ecell, A.cell_fill,
                       A.cell_atoms, G);
  } else {
    scan_launch<1>(n, LoadInt{A.gcount}, A.goff, A.scan_sums, A.gtotal, st, G);
    hipLaunchKernelGGL(k_ghost_emit, dim3(nb), dim3(256), 0, st, n, A.m.ntypes, A.ghost_cap, A.frames,
                       A.frame_of, A.types, A.xw, A.fw, A.goff, A.gtotal, A.xe, A.eown, A.eimg, A.etype, A.ecell,
                       A.cell_count, A.status, G, A.eabc);
    scan_launch<1>(A.ncell + 1, LoadInt{A.cell_count}, A.cell_start, A.scan_sums, A.ctotal, st, G);
    hipLaunchKernelGGL(k_cell_place, dim3((ne_cap + 255) / 256), dim3(256), 0, st, n, A.ghost_cap, A.gtotal,
                       A.n_ext, A.ecell, A.cell_start, A.cell_fill, A.cell_atoms, G);
  }
  if (!A.vlist)
    launch_format(format_args(A), st);
  else if (!rows_later)
    hipLaunchKernelGGL(k_vbuild, dim3((n + kNlWaves - 1) / kNlWaves), dim3(64 * kNlWaves), 0, st, n, A.rl2,
                       A.frames, A.frame_of, A.xe, A.etype, A.ecell, A.cell_start, A.cell_atoms, A.vlist, A.vcnt,
                       A.vcap, A.status, G);
  // species-grouped rows (species do not change during MD: built once there)
  if (A.skip_rows) return;
  // rows of the centres only (all atoms unless the caller supplied ghost atoms)
  const int nc = A.ncentre > 0 ? A.ncentre : n;
  const int nbc = (nc + 255) / 256;
  if (A.m.ntypes == 1) {
    scan_launch<1>(nc, LoadTypeOneHot<1>{A.types, 1}, A.tpos, A.scan_sums, A.tcount, st, G);
  } else if (A.m.ntypes == 2) {
    scan_launch<2>(nc, LoadTypeOneHot<2>{A.types, 2}, A.tpos, A.scan_sums, A.tcount, st, G);
  } else if (A.m.ntypes <= 4) {
    scan_launch<4>(nc, LoadTypeOneHot<4>{A.types, 4}, A.tpos, A.scan_sums, A.tcount, st, G);
  } else {
    scan_launch<8>(nc, LoadTypeOneHot<8>{A.types, 8}, A.tpos, A.scan_sums, A.tcount, st, G);
  }
  int W = A.m.ntypes == 1 ? 1 : A.m.ntypes == 2 ? 2 : A.m.ntypes <= 4 ? 4 : 8;
  fill_int(A.nrows, A.row_atom, -1, G, st);
  hipLaunchKernelGGL(k_type_rows, dim3(nbc), dim3(256), 0, st, nc, A.m.ntypes, W, A.types, A.tpos,
                     A.tcount, A.row_of, A.type_row0, G);
  hipLaunchKernelGGL(k_row_atoms, dim3(nbc), dim3(256), 0, st, nc, A.row_of, A.row_atom, G);
}

void launch_nlist(const NlistArgs& A, hipStream_t st) { launch_rebuild(A, false, st); }

// One MD step's list with Verlet reuse: flag a rebuild when some atom moved more
// than half the skin (A.gate is the flag), rebuild if flagged, then refresh the
// extended coordinates and format the list within rc from the Verlet rows.
void launch_nlist_verlet(const NlistArgs& A, double half_skin, bool disp_done, int* clear, hipStream_t st) {
  const int n = A.n;
  if (!disp_done)
    hipLaunchKernelGGL(k_disp, dim3((n + 255) / 256), dim3(256), 0, st, n, A.x, A.xref, half_skin * half_skin,
                       (int*)A.gate, A.ncell + 1, A.cell_count, A.ncell, A.cell_fill);
  NlistArgs B = A;
  B.cells_zeroed = true;
  launch_rebuild(B, true, st);
  const int ne_cap = n + A.ghost_cap;
  hipLaunchKernelGGL(k_vbuild_refresh, dim3((n + kNlWaves - 1) / kNlWaves), dim3(64 * kNlWaves), 0, st, n, A.rl2,
                     A.frames, A.frame_of, A.xe, A.etype, A.ecell, A.cell_start, A.cell_atoms, A.vlist, A.vcnt,
                     A.vcap, A.status, A.gate, ne_cap, A.n_ext, A.x, A.wk, A.eown, A.eabc, A.xq);
  NlKArgs K = format_args(A);
  K.gate = (int*)A.gate;
  K.clear = clear;
  const dim3 vgrid(((K.n + kNlWaves - 1) / kNlWaves + 7) / 8 * 8), vblock(64 * kNlWaves);
  switch (K.m.ntypes) {
    case 1: hipLaunchKernelGGL(k_nlist_vstep<1>, vgrid, vblock, 0, st, K); break;
    case 2: hipLaunchKernelGGL(k_nlist_vstep<2>, vgrid, vblock, 0, st, K); break;
    case 4: hipLaunchKernelGGL(k_nlist_vstep<4>, vgrid, vblock, 0, st, K); break;
    default: hipLaunchKernelGGL(k_nlist_vstep<0>, vgrid, vblock, 0, st, K); break;
  }
  hipLaunchKernelGGL((k_nlist<kMaxCand>), dim3(kSecondPassBlocks), dim3(64 * kNlWaves), 0, st, K);
}

// exclusive scan of n ints (out [n], total [1])
void launch_scan_int(int n, const int* in, int* out, int* sums, int* total, hipStream_t st) {
  scan_launch<1>(n, LoadInt{in}, out, sums, total, st);
}

struct LoadPairCount {
  const int* row_atom;
  const int* nnei;
  int ntypes, beta, nrows;
  __device__ IV<1> operator()(int r) const {
    IV<1> v;
    int a = r < nrows ? row_atom[r] : -1;
    v.v[0] = a >= 0 ? nnei[a * ntypes + beta] : 0;
    return v;
  }
};

// exclusive scan over species-grouped rows of each centre's real neighbours of
// species beta: base [nrows + 1] (base[nrows] = total)
void launch_pair_scan(int nrows, int ntypes, int beta, const int* row_atom, const int* nnei, int* base,
                      int* sums, int* total, hipStream_t st) {
  scan_launch<1>(nrows + 1, LoadPairCount{row_atom, nnei, ntypes, beta, nrows}, base, sums, total, st);
}

__global__ void k_scatter_params_d(size_t n, const int* __restrict__ map, const double* __restrict__ th,
                                   double* __restrict__ dst) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = map[q] >= 0 ? th[map[q]] : 0.0;
}
__global__ void k_scatter_params_f(size_t n, const int* __restrict__ map, const double* __restrict__ th,
                                   float* __restrict__ dst) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = map[q] >= 0 ? (float)th[map[q]] : 0.0f;
}
// weights in the kernels' layouts from the flat parameter vector via an index map
void launch_scatter_params(int prec, size_t n, const int* map, const double* theta, void* dst, hipStream_t st) {
  if (!n) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_scatter_params_d, dim3((n + 255) / 256), dim3(256), 0, st, n, map, theta, (double*)dst);
  else
    hipLaunchKernelGGL(k_scatter_params_f, dim3((n + 255) / 256), dim3(256), 0, st, n, map, theta, (float*)dst);
}

// BF16 operand packing: hi = bf16(f), lo = bf16(f - hi) with f the FP32 value of the
// parameter (round to nearest even in both conversions); f - hi is exact in FP32
__global__ void k_pack_bf16(size_t n, const int* __restrict__ map, const double* __restrict__ theta,
                            uint16_t* __restrict__ dst) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  int code = map[q];
  if (code == -2) return;
  if (code < 0) {
    dst[q] = 0;
    return;
  }
  float f = (float)theta[code >> 2];
  int kind = code & 3;
  if (kind == 2) {
    *(float*)(dst + q) = f;
    return;
  }
  __bf16 h = (__bf16)f;
  __bf16 v = kind == 0 ? h : (__bf16)(f - (float)h);
  dst[q] = __builtin_bit_cast(uint16_t, v);
}
void launch_pack_bf16(size_t n, const int* map, const double* theta, uint16_t* dst, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_pack_bf16, dim3((n + 255) / 256), dim3(256), 0, st, n, map, theta, dst);
}

__global__ void k_axpy(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) y[q] += a * x[q];
}
void launch_fill_int(int* p, int n, int v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, n, p, v);
}
void launch_zero_int(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, n, p, 0);
}

void launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_axpy, dim3((n + 255) / 256), dim3(256), 0, st, n, a, x, y);
}

void launch_nlist_export(int n, int nm, const int* nlist, const int* eown, const int* eimg,
                         const int* frame_of, const Frame* frames, int* out_j, int* out_img,
                         hipStream_t st) {
  long tot = (long)n * nm;
  hipLaunchKernelGGL(k_nlist_export, dim3((tot + 255) / 256), dim3(256), 0, st, n, nm, nlist, eown,
                     eimg, frame_of, frames, out_j, out_img);
}

}  // namespace dp
