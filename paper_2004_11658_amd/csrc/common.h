// Device-side shared definitions of libdp: frame table, status bits, small helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dp {

constexpr int kMaxTypes = 8;
constexpr int kMaxNm = 1024;
constexpr int kMaxCand = 1024;     // candidates within rc kept per atom (DP_MAX_CANDIDATES)

// status word bits (workspace status[0]); counts in status[1..]
enum : int32_t {
  ST_SEL_OVERFLOW = 1,
  ST_CAPACITY = 2,
  ST_GHOST_CAP = 4,
  ST_BAD_TYPE = 8,
  ST_NONFINITE = 16,
  ST_OVERLAP = 32,
};
enum { STW_FLAGS = 0, STW_SEL_ROWS = 1, STW_MAX_CAND = 2, STW_GHOSTS = 3, STW_FALLBACK = 4, STW_N = 16 };

// Per-frame constants, built on the host.
struct Frame {
  double B[9];      // rows = cell vectors
  double Bi[9];     // inverse, f = x . Bi
  double g[3];      // ghost shell thickness, fractional units (rc / width, widened)
  double cw[3];     // fractional cell width
  int K[3];         // image-code range: ceil(rc / width)
  int Kg[3];        // ghost image range: ceil(g)
  int nc[3];        // cells per axis over [-g, 1 + g)
  int nimg;         // (2K0+1)(2K1+1)(2K2+1)
  int atom0, natoms;
  int cell0;        // first global cell id
  int pad_;
};

// Model constants used by the neighbour and embedding kernels.
struct ModelC {
  int ntypes, nm, M, m2;
  int s0;           // first embedding width
  int sel[kMaxTypes];
  int sel_off[kMaxTypes + 1];
  double rc, rcs, rc2;
  int switch_kind, desc_norm;
  double inv_norm;  // 1/N_m or 1
  double inv_h;     // 1 / (rc - rcs)
};

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// s(r) = w(r)/r and ds/dr for the C2 quintic (or cosine) switch between rcs and rc,
// given ir = 1/r.
__device__ __forceinline__ void smooth_fn_ir(const ModelC& m, double r, double ir, double& s, double& ds) {
  double w, dw;
  if (r < m.rcs) {
    w = 1.0;
    dw = 0.0;
  } else if (r < m.rc) {
    double u = (r - m.rcs) * m.inv_h;
    if (m.switch_kind == 1) {
      double sp, cp;
      sincos(M_PI * u, &sp, &cp);
      w = 0.5 * cp + 0.5;
      dw = -0.5 * M_PI * sp * m.inv_h;
    } else {
      w = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
      dw = -30.0 * u * u * (u - 1.0) * (u - 1.0) * m.inv_h;
    }
  } else {
    w = 0.0;
    dw = 0.0;
  }
  s = w * ir;
  ds = (dw - w * ir) * ir;
}
__device__ __forceinline__ void smooth_fn(const ModelC& m, double r, double& s, double& ds) {
  smooth_fn_ir(m, r, 1.0 / r, s, ds);
}

}  // namespace dp
