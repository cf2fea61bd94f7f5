// C ABI of libdp: model loading, validation, workspace planning and the launch
// sequence of one DP-SE evaluation (arXiv 2004.11658, Sections 2 and 3).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/dp.h"
#include "common.h"
#include "kernels.h"

using namespace dp;

struct dp_handle_s {
  // architecture
  int ntypes = 0, n_emb = 0, n_fit = 0, m2 = 0, switch_kind = 0, desc_norm = 0;
  double rc = 0, rcs = 0;
  std::vector<int> emb_w, fit_w, sel;
  std::vector<double> params;
  int nm = 0, M = 0, s0 = 0;
  int64_t nparams = 0;
  dp_options opt{};
  int device = 0;
  // weight region: one caller-owned device buffer (dp_device_bytes / dp_upload) holding
  // the flat parameters, their index maps and every kernel layout built from them
  bool uploaded = false;
  char* d_wbase = nullptr;
  size_t w_total = 0;
  size_t o_theta = 0, o_net_map = 0, o_fit_map = 0, o_bo_map = 0, o_fitb_map = 0, o_nets = 0, o_fit = 0,
         o_bo = 0, o_fitb = 0, o_ptrs = 0, o_net_off = 0;
  void* d_nets = nullptr;          // ntypes^2 embedding net blocks
  void* d_fit = nullptr;           // fitting weights (storage type)
  double* d_bo = nullptr;          // output biases [ntypes]
  void** d_ptrs = nullptr;         // device pointer tables for the fitting kernel
  double* d_theta = nullptr;       // flat FP64 parameters (model-file order)
  int* d_net_map = nullptr;        // net blocks <- theta index (-1: zero)
  int* d_fit_map = nullptr;        // fitting buffer <- theta index
  int* d_bo_map = nullptr;         // output biases <- theta index
  size_t net_elems = 0, fit_elems = 0;
  // BF16 modes: packed MFMA operands (16-bit units) and their index maps
  uint16_t* d_fitb = nullptr;
  int* d_fitb_map = nullptr;
  size_t fitb_elems = 0;
  // host copies of the index maps and layout offsets (built at dp_init, copied by dp_upload)
  std::vector<int> h_nmap, h_fmap, h_bmap, h_bomap;
  std::vector<int> h_pgmap;   // FP64 position-packed nets <- theta (the parameter gradient's)
  std::vector<int64_t> h_noff;
  std::vector<size_t> h_offW, h_offB, h_offO, h_offWb, h_offWf;
  // student embedding nets (blocks and index map in a caller-owned buffer)
  bool student_on = false;
  int student_hidden = 0;
  void* d_student = nullptr;       // [nnet][kStuElems] storage type
  int* d_student_map = nullptr;
  std::vector<int> h_student_map;
  double st_lo[kMaxTypes * kMaxTypes] = {}, st_hi[kMaxTypes * kMaxTypes] = {};
  int64_t* d_net_off = nullptr;    // [nnet][6] parameter offsets of the full nets
  // stage timing
  bool prof_on = false;
  uint32_t prof_mask = 0;          // stages timed while prof_on (bit DP_STAGE_*)
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_rec;
  std::string err;
};

static hipEvent_t prof_event(dp_handle h) {
  if (h->prof_used == h->prof_pool.size()) {
    hipEvent_t e;
    // timing only: no system-scope fence (cache writeback) at each record
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    h->prof_pool.push_back(e);
  }
  return h->prof_pool[h->prof_used++];
}

// records an event pair around a stage when timing is enabled
struct StageTimer {
  dp_handle h;
  int stage;
  hipStream_t st;
  hipEvent_t e0 = nullptr;
  StageTimer(dp_handle h_, int stage_, hipStream_t st_) : h(h_), stage(stage_), st(st_) {
    if (h->prof_on && ((h->prof_mask >> stage) & 1u) && (e0 = prof_event(h))) (void)hipEventRecord(e0, st);
  }
  ~StageTimer() {
    if (h->prof_on && e0) {
      hipEvent_t e1 = prof_event(h);
      if (e1) {
        (void)hipEventRecord(e1, st);
        h->prof_rec.push_back({stage, {e0, e1}});
      }
    }
  }
};

static thread_local std::string g_init_err;

static int fail(dp_handle h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_init_err = msg;
  return code;
}

#define HIPCHECK(h, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(h, DP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------------------------------------
// model file
// ------------------------------------------------------------------------------------
static int parse_model(dp_handle h, const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) return fail(h, DP_ERR_MODEL, std::string("cannot open model file ") + path);
  std::vector<unsigned char> buf;
  fseek(f, 0, SEEK_END);
  long sz = ftell(f);
  fseek(f, 0, SEEK_SET);
  if (sz < 64) {
    fclose(f);
    return fail(h, DP_ERR_MODEL, "model file too short");
  }
  buf.resize(sz);
  size_t got = fread(buf.data(), 1, sz, f);
  fclose(f);
  if ((long)got != sz) return fail(h, DP_ERR_MODEL, "short read of model file");
  auto i32 = [&](size_t o) { int32_t v; memcpy(&v, &buf[o], 4); return v; };
  auto i64 = [&](size_t o) { int64_t v; memcpy(&v, &buf[o], 8); return v; };
  auto f64 = [&](size_t o) { double v; memcpy(&v, &buf[o], 8); return v; };
  if (memcmp(buf.data(), "DPSEMDL1", 8) != 0) return fail(h, DP_ERR_MODEL, "bad magic");
  if (i32(8) != 1) return fail(h, DP_ERR_MODEL, "unsupported model version");
  int hb = i32(12);
  int64_t np = i64(16);
  h->ntypes = i32(24);
  h->n_emb = i32(28);
  h->n_fit = i32(32);
  h->m2 = i32(36);
  h->switch_kind = i32(40);
  h->desc_norm = i32(44);
  h->rc = f64(48);
  h->rcs = f64(56);
  if (h->ntypes < 1 || h->ntypes > kMaxTypes) return fail(h, DP_ERR_MODEL, "ntypes must be 1..8");
  if (h->n_emb != 3) return fail(h, DP_ERR_MODEL, "embedding net must have 3 layers");
  if (h->n_fit < 1 || h->n_fit > 8) return fail(h, DP_ERR_MODEL, "fitting net must have 1..8 hidden layers");
  size_t nint = h->n_emb + h->n_fit + h->ntypes;
  if (64 + 4 * nint > (size_t)hb || hb > sz) return fail(h, DP_ERR_MODEL, "bad header size");
  for (int k = 0; k < h->n_emb; k++) h->emb_w.push_back(i32(64 + 4 * k));
  for (int k = 0; k < h->n_fit; k++) h->fit_w.push_back(i32(64 + 4 * (h->n_emb + k)));
  h->nm = 0;
  for (int t = 0; t < h->ntypes; t++) {
    h->sel.push_back(i32(64 + 4 * (h->n_emb + h->n_fit + t)));
    if (h->sel.back() < 0) return fail(h, DP_ERR_MODEL, "negative sel");
    h->nm += h->sel.back();
  }
  h->s0 = h->emb_w[0];
  h->M = h->emb_w[2];
  if (h->s0 < 1 || h->s0 > 32 || h->emb_w[1] != 2 * h->s0 || h->emb_w[2] != 2 * h->emb_w[1])
    return fail(h, DP_ERR_MODEL, "embedding widths must be s0, 2 s0, 4 s0 with s0 <= 32");
  for (int k = 1; k < h->n_fit; k++)
    if (h->fit_w[k] != h->fit_w[0]) return fail(h, DP_ERR_MODEL, "hidden fitting layers must be square");
  if (h->fit_w[0] < 1 || h->fit_w[0] > 1024) return fail(h, DP_ERR_MODEL, "fitting width out of range");
  if (h->m2 < 1 || h->m2 > h->M) return fail(h, DP_ERR_MODEL, "M< out of range");
  if (h->nm < 1 || h->nm > kMaxNm) return fail(h, DP_ERR_MODEL, "N_m must be 1..1024");
  if (!(h->rc > h->rcs) || h->rcs < 0 || !(h->rc < 64)) return fail(h, DP_ERR_MODEL, "bad cutoffs");
  if (h->switch_kind < 0 || h->switch_kind > 1 || h->desc_norm < 0 || h->desc_norm > 1)
    return fail(h, DP_ERR_MODEL, "bad switch/normalisation flag");
  // parameter count
  int64_t cnt = 0;
  for (int a = 0; a < h->ntypes * h->ntypes; a++) {
    int nin = 1;
    for (int k = 0; k < 3; k++) { cnt += (int64_t)nin * h->emb_w[k] + h->emb_w[k]; nin = h->emb_w[k]; }
  }
  for (int a = 0; a < h->ntypes; a++) {
    int nin = h->M * h->m2;
    for (int k = 0; k < h->n_fit; k++) { cnt += (int64_t)nin * h->fit_w[k] + h->fit_w[k]; nin = h->fit_w[k]; }
    cnt += nin + 1;
  }
  if (cnt != np || hb + 8 * np != sz) return fail(h, DP_ERR_MODEL, "parameter count mismatch");
  h->nparams = np;
  h->params.resize(np);
  memcpy(h->params.data(), &buf[hb], 8 * np);
  return DP_OK;
}

// offsets of each block in the flat parameter vector
struct ParamIndex {
  std::vector<int64_t> eW, eB;   // [net*3 + layer]
  std::vector<int64_t> fW, fB;   // [type*(nfit+1) + layer], layer nfit = output
};
static ParamIndex index_params(dp_handle h) {
  ParamIndex P;
  int64_t off = 0;
  for (int a = 0; a < h->ntypes * h->ntypes; a++) {
    int nin = 1;
    for (int k = 0; k < 3; k++) {
      P.eW.push_back(off); off += (int64_t)nin * h->emb_w[k];
      P.eB.push_back(off); off += h->emb_w[k];
      nin = h->emb_w[k];
    }
  }
  for (int a = 0; a < h->ntypes; a++) {
    int nin = h->M * h->m2;
    for (int k = 0; k <= h->n_fit; k++) {
      int nout = k < h->n_fit ? h->fit_w[k] : 1;
      P.fW.push_back(off); off += (int64_t)nin * nout;
      P.fB.push_back(off); off += nout;
      nin = nout;
    }
  }
  return P;
}

static int storage_bytes(int prec) { return prec == PREC_FP64 ? 8 : 4; }

// position p of a padded layer <-> feature index (p / 32) * s0 + p % 32, pad if p % 32 >= s0
static int pos_feature(int p, int s0) { return (p % kP0) < s0 ? (p / kP0) * s0 + (p % kP0) : -1; }

// index map of one position-padded net block: element -> parameter index (-1 = zero)
static void net_block_map(dp_handle h, const ParamIndex& P, int net, int* blk) {
  int s0 = h->s0, s1 = 2 * s0, s2 = 4 * s0;
  for (int q = 0; q < kNetElems; q++) blk[q] = -1;
  for (int pp = 0; pp < kP0; pp++) {
    int f = pos_feature(pp, s0);
    if (f < 0) continue;
    blk[kOffW0 + pp] = (int)(P.eW[net * 3 + 0] + f);
    blk[kOffB0 + pp] = (int)(P.eB[net * 3 + 0] + f);
  }
  for (int pp = 0; pp < kP1; pp++) {
    int f = pos_feature(pp, s0);
    if (f >= 0) blk[kOffB1 + pp] = (int)(P.eB[net * 3 + 1] + f);
  }
  for (int pp = 0; pp < kP2; pp++) {
    int f = pos_feature(pp, s0);
    if (f >= 0) blk[kOffB2 + pp] = (int)(P.eB[net * 3 + 2] + f);
  }
  for (int pi = 0; pi < kP0; pi++) {
    int fi = pos_feature(pi, s0);
    if (fi < 0) continue;
    for (int po = 0; po < kP1; po++) {
      int fo = pos_feature(po, s0);
      if (fo >= 0) blk[kOffW1 + pi * kW1Stride + po] = (int)(P.eW[net * 3 + 1] + (int64_t)fi * s1 + fo);
    }
  }
  for (int pi = 0; pi < kP1; pi++) {
    int fi = pos_feature(pi, s0);
    if (fi < 0) continue;
    for (int po = 0; po < kP2; po++) {
      int fo = pos_feature(po, s0);
      if (fo >= 0) blk[kOffW2 + pi * kW2Stride + po] = (int)(P.eW[net * 3 + 2] + (int64_t)fi * s2 + fo);
    }
  }
}

static bool bf16_mode(int prec) { return prec == PREC_BF16 || prec == PREC_BF16X3; }

// index map of one BF16 net block (16-bit units, layout in kernels.h): code 4 idx + kind
// with kind 0 / 1 the hi / lo BF16 part and 2 a float over two units (-2 marks the second
// unit), -1 zero.  Packed tile t, lane (g, rb), element j: the k slot stands for input
// position 16 (2 kc + j / 4) + 4 g + j % 4 of the product, the lane row rb for output
// position 16 t' + rb (t = t' * nkc + kc).
static void bnet_block_map(dp_handle h, const ParamIndex& P, int net, int parts, int* blk) {
  int s0 = h->s0, s1 = 2 * s0, s2 = 4 * s0;
  const int nu = bnet_u16(parts);
  for (int q = 0; q < nu; q++) blk[q] = -1;
  std::vector<int> fl(kNetElems);
  net_block_map(h, P, net, fl.data());
  for (int q = 0; q < kBFloat; q++) {
    blk[2 * q] = fl[q] >= 0 ? 4 * fl[q] + 2 : -1;
    blk[2 * q + 1] = fl[q] >= 0 ? -2 : -1;
  }
  // W[in pos][out pos] of layer L (1 or 2) as a parameter index, -1 for pads
  auto widx = [&](int L, int pin, int pout) -> int {
    int fi = pos_feature(pin, s0), fo = pos_feature(pout, s0);
    if (fi < 0 || fo < 0) return -1;
    return (int)(P.eW[net * 3 + L] + (int64_t)fi * (L == 1 ? s1 : s2) + fo);
  };
  // group: base (u16) of part 0, part stride, layer, number of k chunks, forward or adjoint
  auto fill = [&](int base, int pstride, int L, int ntile, int nkc, bool fwd) {
    for (int part = 0; part < parts; part++)
      for (int t = 0; t < ntile; t++)
        for (int kc = 0; kc < nkc; kc++)
          for (int lane = 0; lane < 64; lane++)
            for (int j = 0; j < 8; j++) {
              int g = lane >> 4, rb = lane & 15;
              int kpos = 16 * (2 * kc + j / 4) + 4 * g + j % 4;
              int opos = 16 * t + rb;
              int idx = fwd ? widx(L, kpos, opos) : widx(L, opos, kpos);
              blk[base + part * pstride + ((t * nkc + kc) * 64 + lane) * 8 + j] = idx >= 0 ? 4 * idx + part : -1;
            }
  };
  const int f0 = 2 * kBFloat, b0 = f0 + parts * kBFwd;
  fill(f0, kBFwd, 1, 4, 1, true);
  fill(f0 + kBW1F, kBFwd, 2, 8, 2, true);
  fill(b0, kBBwd, 1, 2, 2, false);
  fill(b0 + kBW1B, kBBwd, 2, 4, 4, false);
}

// device layouts of the weights, rebuilt from d_theta by index maps
static int refresh_weights(dp_handle h, hipStream_t st) {
  if (bf16_mode(h->opt.precision)) {
    launch_pack_bf16(h->net_elems, h->d_net_map, h->d_theta, (uint16_t*)h->d_nets, st);
    launch_pack_bf16(h->fitb_elems, h->d_fitb_map, h->d_theta, h->d_fitb, st);
  } else {
    launch_scatter_params(h->opt.precision == PREC_FP64 ? 0 : 1, h->net_elems, h->d_net_map, h->d_theta,
                          h->d_nets, st);
  }
  launch_scatter_params(h->opt.precision == PREC_FP64 ? 0 : 1, h->fit_elems, h->d_fit_map, h->d_theta,
                        h->d_fit, st);
  launch_scatter_params(0, h->ntypes, h->d_bo_map, h->d_theta, h->d_bo, st);
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

// index maps and layout offsets of the weight region, on the host (dp_init)
static void plan_weights(dp_handle h) {
  ParamIndex P = index_params(h);
  const int sb = storage_bytes(h->opt.precision);
  int nnet = h->ntypes * h->ntypes;
  const bool bf = bf16_mode(h->opt.precision);
  const int parts = prec_parts(h->opt.precision);
  const size_t blk_units = bf ? (size_t)bnet_u16(parts) : (size_t)kNetElems;
  std::vector<int> nmap((size_t)nnet * blk_units);
  for (int net = 0; net < nnet; net++) {
    if (bf) bnet_block_map(h, P, net, parts, nmap.data() + (size_t)net * blk_units);
    else net_block_map(h, P, net, nmap.data() + (size_t)net * blk_units);
  }
  h->h_pgmap.assign((size_t)nnet * kNetElems, -1);
  for (int net = 0; net < nnet; net++) net_block_map(h, P, net, h->h_pgmap.data() + (size_t)net * kNetElems);
  // BF16 GEMM operands per species and layer: W^T [out][in] then W [in][out], each as
  // hi and lo parts, every group padded to a multiple of 8 units (16-byte rows)
  std::vector<int> bmap;
  std::vector<size_t> offWb;
  if (bf)
    for (int a = 0; a < h->ntypes; a++) {
      int nin = h->M * h->m2;
      for (int k = 0; k < h->n_fit; k++) {
        int nout = h->fit_w[k];
        int64_t w0 = P.fW[a * (h->n_fit + 1) + k];
        for (int dir = 0; dir < 2; dir++)
          for (int part = 0; part < 2; part++) {
            offWb.push_back(bmap.size());
            int rows = dir == 0 ? nout : nin, cols = dir == 0 ? nin : nout;
            for (int r = 0; r < rows; r++)
              for (int c = 0; c < cols; c++) {
                int64_t idx = dir == 0 ? w0 + (int64_t)c * nout + r : w0 + (int64_t)r * nout + c;
                bmap.push_back(part < parts ? (int)(4 * idx + part) : -1);
              }
            while (bmap.size() % 8) bmap.push_back(-1);
          }
        nin = nout;
      }
    }
  // the same weights as MFMA operand fragments for the 64-row-tile kernels: per species,
  // layer and direction (0 forward B[k][n] = W[k][n], 1 adjoint B[k][n] = W[n][k]) blocks
  // (ct, ks, part) of 64 lanes x 8, lane l holding B[32 ks + 8 (l / 16) + j][16 ct + l % 16],
  // zero outside B.  Operands whose columns are fitting-layer outputs or inputs of width
  // <= 256 get 16 column tiles (the kernels' waves take four each, unconditionally); the
  // first layer's adjoint (columns = descriptor entries) gets exactly M tiles.
  std::vector<size_t> offWf;
  if (bf && fit_bf_supported(h->M, h->m2, h->fit_w[0]))
    for (int a = 0; a < h->ntypes; a++) {
      int nin = h->M * h->m2;
      for (int k = 0; k < h->n_fit; k++) {
        const int nout = h->fit_w[k];
        const int64_t w0 = P.fW[a * (h->n_fit + 1) + k];
        for (int dir = 0; dir < 2; dir++) {
          offWf.push_back(bmap.size());
          const int K = dir == 0 ? nin : nout, N = dir == 0 ? nout : nin;
          // k steps: the first layer's forward takes all of K = 16 M; every other operand's k
          // dimension is a fitting width, padded to 8 steps (256)
          const int KS = (k == 0 && dir == 0) ? (K + 31) / 32 : 8;
          const int NT = (k == 0 && dir == 1) ? (N + 15) / 16 : 16;
          for (int ct = 0; ct < NT; ct++)
            for (int ks = 0; ks < KS; ks++)
              for (int part = 0; part < parts; part++)
                for (int l = 0; l < 64; l++)
                  for (int j = 0; j < 8; j++) {
                    const int kk = 32 * ks + 8 * (l >> 4) + j, n = 16 * ct + (l & 15);
                    if (kk >= K || n >= N) {
                      bmap.push_back(-1);
                      continue;
                    }
                    const int64_t idx = dir == 0 ? w0 + (int64_t)kk * nout + n : w0 + (int64_t)n * nout + kk;
                    bmap.push_back((int)(4 * idx + part));
                  }
        }
        nin = nout;
      }
    }
  // fitting weights, per species: W_k, b_k for k < nfit, then wo (rows padded to 64)
  std::vector<int> fmap;
  std::vector<size_t> offW, offB, offO;
  std::vector<int> bomap(h->ntypes);
  for (int a = 0; a < h->ntypes; a++) {
    int nin = h->M * h->m2;
    for (int k = 0; k < h->n_fit; k++) {
      int nout = h->fit_w[k];
      offW.push_back(fmap.size());
      for (int64_t q = 0; q < (int64_t)nin * nout; q++) fmap.push_back((int)(P.fW[a * (h->n_fit + 1) + k] + q));
      offB.push_back(fmap.size());
      for (int q = 0; q < nout; q++) fmap.push_back((int)(P.fB[a * (h->n_fit + 1) + k] + q));
      nin = nout;
    }
    offO.push_back(fmap.size());
    for (int q = 0; q < nin; q++) fmap.push_back((int)(P.fW[a * (h->n_fit + 1) + h->n_fit] + q));
    bomap[a] = (int)P.fB[a * (h->n_fit + 1) + h->n_fit];
    while (fmap.size() % 64) fmap.push_back(-1);
  }
  h->net_elems = nmap.size();
  h->fit_elems = fmap.size();
  h->fitb_elems = bmap.size();
  std::vector<int64_t> noff((size_t)nnet * 6);
  for (int net = 0; net < nnet; net++)
    for (int k = 0; k < 3; k++) {
      noff[net * 6 + 2 * k] = P.eW[net * 3 + k];
      noff[net * 6 + 2 * k + 1] = P.eB[net * 3 + k];
    }
  // pointer tables: W [ntypes*nfit], b [ntypes*nfit], wo [ntypes], BF16 operand table
  // [(species * nfit + k) * 4 + dir * 2 + part], BF16 operand fragments
  // [(species * nfit + k) * 2 + dir]
  const size_t nptrs = offW.size() + offB.size() + offO.size() + offWb.size() + offWf.size();
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = (o + bytes + 255) & ~(size_t)255; return r; };
  h->o_theta = take(sizeof(double) * h->nparams);
  h->o_net_map = take(sizeof(int) * nmap.size());
  h->o_fit_map = take(sizeof(int) * fmap.size());
  h->o_bo_map = take(sizeof(int) * bomap.size());
  h->o_fitb_map = take(sizeof(int) * bmap.size());
  h->o_nets = take(bf ? nmap.size() * 2 : nmap.size() * sb);
  h->o_fit = take(fmap.size() * sb);
  h->o_bo = take(h->ntypes * sizeof(double));
  h->o_fitb = take(sizeof(uint16_t) * bmap.size());
  h->o_ptrs = take(nptrs * sizeof(void*));
  h->o_net_off = take(sizeof(int64_t) * noff.size());
  h->w_total = o;
  h->h_nmap = std::move(nmap);
  h->h_fmap = std::move(fmap);
  h->h_bmap = std::move(bmap);
  h->h_bomap = std::move(bomap);
  h->h_noff = std::move(noff);
  h->h_offW = std::move(offW);
  h->h_offB = std::move(offB);
  h->h_offO = std::move(offO);
  h->h_offWb = std::move(offWb);
  h->h_offWf = std::move(offWf);
}

// binds the weight region to a caller buffer: copies the parameters, maps and pointer
// tables in and builds the kernel layouts (synchronises the stream)
static int bind_weights(dp_handle h, void* base, hipStream_t st) {
  char* w = (char*)base;
  h->d_wbase = w;
  h->d_theta = (double*)(w + h->o_theta);
  h->d_net_map = (int*)(w + h->o_net_map);
  h->d_fit_map = (int*)(w + h->o_fit_map);
  h->d_bo_map = (int*)(w + h->o_bo_map);
  h->d_fitb_map = h->h_bmap.empty() ? nullptr : (int*)(w + h->o_fitb_map);
  h->d_nets = w + h->o_nets;
  h->d_fit = w + h->o_fit;
  h->d_bo = (double*)(w + h->o_bo);
  h->d_fitb = h->h_bmap.empty() ? nullptr : (uint16_t*)(w + h->o_fitb);
  h->d_ptrs = (void**)(w + h->o_ptrs);
  h->d_net_off = (int64_t*)(w + h->o_net_off);
  const int sb = storage_bytes(h->opt.precision);
  std::vector<void*> ptrs;
  char* fb = (char*)h->d_fit;
  for (size_t q : h->h_offW) ptrs.push_back(fb + q * sb);
  for (size_t q : h->h_offB) ptrs.push_back(fb + q * sb);
  for (size_t q : h->h_offO) ptrs.push_back(fb + q * sb);
  for (size_t q : h->h_offWb) ptrs.push_back(h->d_fitb + q);
  for (size_t q : h->h_offWf) ptrs.push_back(h->d_fitb + q);
  HIPCHECK(h, hipSetDevice(h->device));
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIPCHECK(h, up(h->d_theta, h->params.data(), sizeof(double) * h->nparams));
  HIPCHECK(h, up(h->d_net_map, h->h_nmap.data(), sizeof(int) * h->h_nmap.size()));
  HIPCHECK(h, up(h->d_fit_map, h->h_fmap.data(), sizeof(int) * h->h_fmap.size()));
  HIPCHECK(h, up(h->d_bo_map, h->h_bomap.data(), sizeof(int) * h->h_bomap.size()));
  if (h->d_fitb_map) HIPCHECK(h, up(h->d_fitb_map, h->h_bmap.data(), sizeof(int) * h->h_bmap.size()));
  HIPCHECK(h, up(h->d_ptrs, ptrs.data(), sizeof(void*) * ptrs.size()));
  HIPCHECK(h, up(h->d_net_off, h->h_noff.data(), sizeof(int64_t) * h->h_noff.size()));
  h->uploaded = true;
  int rc = refresh_weights(h, st);
  if (rc != DP_OK) {
    h->uploaded = false;
    return rc;
  }
  // the host arrays above are read by the copies: wait for them
  HIPCHECK(h, hipStreamSynchronize(st));
  return DP_OK;
}

static int need_weights(dp_handle h) {
  if (!h->uploaded) return fail(h, DP_ERR_ARG, "weights not uploaded: call dp_upload first");
  return DP_OK;
}

// ------------------------------------------------------------------------------------
// boxes and frames
// ------------------------------------------------------------------------------------
// B^-1 as the adjugate over the determinant, evaluated in a fixed order with
// contraction off (integer decisions downstream depend on these bits).
static int box_setup(const double* b9, double rc, Frame& F) {
#pragma clang fp contract(off)
  const double* B = b9;
  double det = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
               B[2] * (B[3] * B[7] - B[4] * B[6]);
  if (!(det > 0) || !std::isfinite(det)) return -1;
  double C[9];
  C[0] = B[4] * B[8] - B[5] * B[7];
  C[1] = B[5] * B[6] - B[3] * B[8];
  C[2] = B[3] * B[7] - B[4] * B[6];
  C[3] = B[2] * B[7] - B[1] * B[8];
  C[4] = B[0] * B[8] - B[2] * B[6];
  C[5] = B[1] * B[6] - B[0] * B[7];
  C[6] = B[1] * B[5] - B[2] * B[4];
  C[7] = B[2] * B[3] - B[0] * B[5];
  C[8] = B[0] * B[4] - B[1] * B[3];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) F.Bi[3 * r + c] = C[3 * c + r] / det;
  memcpy(F.B, B, sizeof(F.B));
  int nimg = 1;
  for (int k = 0; k < 3; k++) {
    double n2 = (F.Bi[0 + k] * F.Bi[0 + k] + F.Bi[3 + k] * F.Bi[3 + k]) + F.Bi[6 + k] * F.Bi[6 + k];
    double width = 1.0 / std::sqrt(n2);
    F.K[k] = (int)std::ceil(rc / width);
    double g = rc / width * (1.0 + 1e-9) + 1e-9;
    F.g[k] = g;
    F.Kg[k] = (int)std::ceil(g);
    int nc = (int)std::floor((1.0 + 2.0 * g) * width / rc);
    if (nc < 1) nc = 1;
    F.nc[k] = nc;
    F.cw[k] = (1.0 + 2.0 * g) / nc;
    nimg *= 2 * F.K[k] + 1;
  }
  F.nimg = nimg;
  return 0;
}

struct Plan {
  size_t total = 0;
  size_t o_frames_red = 0;   // caller-supplied ghosts: frame 0 restricted to the centres (reductions)
  size_t o_status, o_frames, o_frame_of, o_xw, o_fw, o_gcount, o_goff, o_small, o_scan;
  size_t o_xe, o_eown, o_eimg, o_etype, o_ecell, o_ccount, o_cstart, o_cfill, o_catoms;
  size_t o_nlist, o_nnei, o_tpos, o_rowof, o_rowatom, o_T, o_gT, o_D, o_Dg, o_act, o_xs, o_g0,
      o_g1, o_Ei, o_vir, o_tmpj, o_tmpi, o_mdF, o_mdE, o_mdW, o_fb, o_fbcnt;
  // Verlet reuse (MD with a skin)
  bool verlet = false;
  size_t o_wk, o_xref, o_eabc, o_vlist, o_vcnt, o_vflag, o_npt = 0, o_xq = 0;
  int n, nframes, ncell, ghost_cap, nrows, vcap, max_frame_atoms;
  size_t o_redpart;
  size_t o_gbuf = 0, o_rev = 0;   // deterministic force gather
  size_t o_big = 0;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// verlet: lay out the MD Verlet reuse as well (ghost shell and cells for rc + skin,
// image codes over the whole ghost range)
// min_scale < 1 (isobaric MD): the Verlet plan's ghost shell, cells and candidate rows
// also cover the box compressed to min_scale times its linear size
static int make_plan(dp_handle h, int nframes, const int64_t* off, const double* boxes,
                     std::vector<Frame>* frames, Plan& P, bool verlet = false, double min_scale = 1.0) {
  if (nframes < 1) return fail(h, DP_ERR_ARG, "nframes must be >= 1");
  if (off[0] != 0) return fail(h, DP_ERR_ARG, "atom_offsets[0] must be 0");
  int64_t n = off[nframes];
  if (n < 1 || n > (1 << 26)) return fail(h, DP_ERR_ARG, "natoms out of range");
  int64_t ghost_cap = 0, ncell = 0, maxna = 0;
  if (frames) frames->resize(nframes);
  for (int f = 0; f < nframes; f++) {
    int64_t na = off[f + 1] - off[f];
    if (na < 1) return fail(h, DP_ERR_ARG, "every frame needs at least one atom");
    maxna = std::max(maxna, na);
    Frame F{};
    if (box_setup(boxes + 9 * f, verlet ? (h->rc + h->opt.skin) / min_scale : h->rc, F))
      return fail(h, DP_ERR_BOX, "singular or left-handed box");
    if (verlet) {
      F.nimg = 1;
      for (int k = 0; k < 3; k++) {
        F.K[k] = F.Kg[k];
        F.nimg *= 2 * F.K[k] + 1;
      }
    }
    double vol_ext = (1 + 2 * F.g[0]) * (1 + 2 * F.g[1]) * (1 + 2 * F.g[2]);
    double expect = na * (vol_ext - 1.0);
    int64_t maxg = na * ((int64_t)(2 * F.Kg[0] + 1) * (2 * F.Kg[1] + 1) * (2 * F.Kg[2] + 1) - 1);
    int64_t cap = std::min<int64_t>(maxg, (int64_t)std::ceil(1.3 * expect) + 2048);
    F.atom0 = (int)off[f];
    F.natoms = (int)na;
    F.cell0 = (int)ncell;
    ncell += (int64_t)F.nc[0] * F.nc[1] * F.nc[2];
    ghost_cap += cap;
    if (frames) (*frames)[f] = F;
  }
  if (ncell > (1 << 28) || ghost_cap + n > (1LL << 30)) return fail(h, DP_ERR_ARG, "system too large");
  P.n = (int)n;
  P.nframes = nframes;
  P.ncell = (int)ncell;
  P.ghost_cap = (int)ghost_cap;
  P.nrows = (int)(n + (int64_t)h->ntypes * kRowPad);
  int W = h->ntypes == 1 ? 1 : h->ntypes == 2 ? 2 : h->ntypes <= 4 ? 4 : 8;
  int64_t ne = n + ghost_cap;
  int sb = storage_bytes(h->opt.precision);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + bytes); return r; };
  P.o_status = take(sizeof(int) * STW_N);
  P.o_frames = take(sizeof(Frame) * nframes);
  P.o_frames_red = take(sizeof(Frame));
  P.o_frame_of = take(sizeof(int) * n);
  P.o_xw = take(sizeof(double) * 3 * n);
  P.o_fw = take(sizeof(double) * 3 * n);
  P.o_gcount = take(sizeof(int) * n);
  P.o_goff = take(sizeof(int) * (n + 1));
  P.o_small = take(sizeof(int) * 64);
  size_t ns = std::max(scan_sums_ints((int)std::max<int64_t>(n, ncell + 1), 1),
                       scan_sums_ints((int)n, W));
  P.o_scan = take(sizeof(int) * ns);
  P.o_xe = take(sizeof(double) * 3 * ne);
  P.o_eown = take(sizeof(int) * ne);
  P.o_eimg = take(sizeof(int) * ne);
  P.o_etype = take(sizeof(int) * ne);
  P.o_ecell = take(sizeof(int) * ne);
  P.o_ccount = take(sizeof(int) * (ncell + 1));
  P.o_cstart = take(sizeof(int) * (ncell + 1));
  P.o_cfill = take(sizeof(int) * ncell);
  P.o_catoms = take(sizeof(int) * ne);
  P.o_nlist = take(sizeof(int) * n * h->nm);
  P.o_nnei = take(sizeof(int) * n * h->ntypes);
  P.o_big = take(sizeof(int) * n);
  P.o_tpos = take(sizeof(int) * n * W);
  P.o_rowof = take(sizeof(int) * n);
  P.o_rowatom = take(sizeof(int) * P.nrows);
  size_t rows = P.nrows;
  P.o_T = take((size_t)sb * rows * h->M * 4);
  P.o_gT = take((size_t)sb * rows * h->M * 4);
  int K1 = h->M * h->m2, fw = h->fit_w[0];
  P.o_D = take((size_t)sb * rows * K1);
  P.o_Dg = take((size_t)sb * rows * K1);
  P.o_act = take((size_t)sb * rows * fw * h->n_fit);
  P.o_xs = take((size_t)sb * rows * fw * h->n_fit);
  P.o_g0 = take((size_t)sb * rows * fw);
  P.o_g1 = take((size_t)sb * rows * fw);
  P.o_Ei = take(sizeof(double) * rows);
  P.o_vir = take(sizeof(double) * rows * 9);
  P.o_tmpj = take(sizeof(double) * nframes * 10);
  P.max_frame_atoms = (int)maxna;
  P.o_redpart = take(sizeof(double) * 10 * (size_t)nframes * frame_reduce_chunks((int)maxna));
  P.o_tmpi = take(sizeof(int) * 16);
  P.o_mdF = take(sizeof(double) * 3 * n);
  P.o_mdE = take(sizeof(double) * nframes);
  P.o_mdW = take(sizeof(double) * 9 * nframes);
  P.o_fb = h->student_on ? take(sizeof(int2) * n * h->nm) : 0;
  P.o_fbcnt = take(sizeof(int) * 64);
  if (h->opt.deterministic) {
    P.o_gbuf = take(sizeof(double) * 3 * (size_t)n * h->nm);
    P.o_rev = take(sizeof(int) * (rev_scratch_ints((int)n, h->nm) + 16));
  }
  P.verlet = verlet;
  P.vcap = 0;
  if (verlet) {
    // candidates within rc + skin: the rc capacity scaled by the volume ratio
    double q = (h->rc + h->opt.skin) / (h->rc * min_scale);
    P.vcap = (int)std::min<double>(4.0 * kMaxCand, std::ceil(kMaxCand * q * q * q / 64.0) * 64.0);
    P.o_wk = take(sizeof(int) * 3 * n);
    P.o_xref = take(sizeof(double) * 3 * n);
    P.o_eabc = take(sizeof(int) * 3 * ne);
    P.o_xq = take(sizeof(double) * 4 * ne);
    P.o_vlist = take(sizeof(int) * (size_t)n * P.vcap);
    P.o_vcnt = take(sizeof(int) * n);
    P.o_vflag = take(sizeof(int) * 64);
    P.o_npt = take(sizeof(double) * NS_COUNT);
  }
  P.total = o;
  return DP_OK;
}

namespace dp {
int handle_device(dp_handle h) { return h->device; }
int set_error(dp_handle h, int code, const std::string& msg) { return fail(h, code, msg); }
int compute_ws_bytes(dp_handle h, int64_t natoms, const double* box, size_t* bytes) {
  int64_t off[2] = {0, natoms};
  Plan P;
  int rc = make_plan(h, 1, off, box, nullptr, P);
  if (rc != DP_OK) return rc;
  *bytes = P.total;
  return DP_OK;
}
}  // namespace dp

// ------------------------------------------------------------------------------------
// public API
// ------------------------------------------------------------------------------------
static ModelC model_consts(dp_handle h) {
  ModelC m{};
  m.ntypes = h->ntypes;
  m.nm = h->nm;
  m.M = h->M;
  m.m2 = h->m2;
  m.s0 = h->s0;
  int o = 0;
  for (int t = 0; t < kMaxTypes; t++) {
    m.sel[t] = t < h->ntypes ? h->sel[t] : 0;
    m.sel_off[t] = o;
    o += m.sel[t];
  }
  m.sel_off[kMaxTypes] = o;
  m.rc = h->rc;
  m.rcs = h->rcs;
  m.rc2 = h->rc * h->rc;
  m.switch_kind = h->switch_kind;
  m.desc_norm = h->desc_norm;
  m.inv_norm = h->desc_norm == 0 ? 1.0 / (double)h->nm : 1.0;
  m.inv_h = 1.0 / (h->rc - h->rcs);
  return m;
}

struct Ws {
  char* base;
  const Plan* P;
  template <class T>
  T* at(size_t off) const { return (T*)(base + off); }
};

// plans the call, validates the workspace and copies the frame table to the device
static int stage_frames(dp_handle h, int nframes, const int64_t* off, const double* boxes,
                        const double* coords, const int32_t* types, void* ws, size_t ws_bytes,
                        hipStream_t st, Plan& P, NlistArgs& A, bool verlet = false, double min_scale = 1.0) {
  if (need_weights(h) != DP_OK) return DP_ERR_ARG;
  std::vector<Frame> frames;
  int rc = make_plan(h, nframes, off, boxes, &frames, P, verlet, min_scale);
  if (rc != DP_OK) return rc;
  if (!ws || ws_bytes < P.total)
    return fail(h, DP_ERR_WORKSPACE, "workspace too small: need " + std::to_string(P.total) + " bytes");
  if (!coords || !types) return fail(h, DP_ERR_ARG, "null coordinates or types");
  HIPCHECK(h, hipSetDevice(h->device));
  Ws W{(char*)ws, &P};
  // the frame table travels in kernel arguments (no staging memory, no host wait)
  launch_put_frames(frames.data(), nframes, W.at<Frame>(P.o_frames), st);
  A.n = P.n;
  A.nframes = nframes;
  A.ncell = P.ncell;
  A.ghost_cap = P.ghost_cap;
  A.nrows = P.nrows;
  A.m = model_consts(h);
  A.frames = W.at<Frame>(P.o_frames);
  A.x = coords;
  A.types = types;
  A.status = W.at<int>(P.o_status);
  A.frame_of = W.at<int>(P.o_frame_of);
  A.xw = W.at<double>(P.o_xw);
  A.fw = W.at<double>(P.o_fw);
  A.gcount = W.at<int>(P.o_gcount);
  A.goff = W.at<int>(P.o_goff);
  int* small = W.at<int>(P.o_small);
  A.gtotal = small + 0;
  A.ctotal = small + 1;
  A.n_ext = small + 2;
  A.tcount = small + 8;        // up to 8 counters
  A.type_row0 = small + 16;    // up to 9 values
  A.scan_sums = W.at<int>(P.o_scan);
  A.xe = W.at<double>(P.o_xe);
  A.eown = W.at<int>(P.o_eown);
  A.eimg = W.at<int>(P.o_eimg);
  A.etype = W.at<int>(P.o_etype);
  A.ecell = W.at<int>(P.o_ecell);
  A.cell_count = W.at<int>(P.o_ccount);
  A.cell_start = W.at<int>(P.o_cstart);
  A.cell_fill = W.at<int>(P.o_cfill);
  A.cell_atoms = W.at<int>(P.o_catoms);
  A.nlist = W.at<int>(P.o_nlist);
  A.nnei = W.at<int>(P.o_nnei);
  A.tpos = W.at<int>(P.o_tpos);
  A.row_of = W.at<int>(P.o_rowof);
  A.row_atom = W.at<int>(P.o_rowatom);
  A.big = W.at<int>(P.o_big);
  A.nbig = small + 32;         // and its second-pass counter at small + 33
  A.skip_rows = false;
  A.gate = nullptr;
  if (P.verlet) {
    A.wk = W.at<int>(P.o_wk);
    A.xref = W.at<double>(P.o_xref);
    A.eabc = W.at<int>(P.o_eabc);
    A.xq = W.at<double>(P.o_xq);
    A.vlist = W.at<int>(P.o_vlist);
    A.vcnt = W.at<int>(P.o_vcnt);
    A.vcap = P.vcap;
    double rl = h->rc + h->opt.skin;
    A.rl2 = rl * rl;
    A.gate = W.at<int>(P.o_vflag);
    launch_zero_int((int*)A.gate, 1, st);
  }
  // the status word covers the whole call
  launch_zero_int(A.status, STW_N, st);
  launch_zero_int(A.nbig, 2, st);   // deferred-atom count and its pass counter
  return DP_OK;
}

static int stage_nlist(dp_handle h, const NlistArgs& A, hipStream_t st) {
  StageTimer tm(h, DP_STAGE_NLIST, st);
  launch_nlist(A, st);
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

static int stage_frames_and_nlist(dp_handle h, int nframes, const int64_t* off, const double* boxes,
                                  const double* coords, const int32_t* types, void* ws,
                                  size_t ws_bytes, hipStream_t st, Plan& P, NlistArgs& A) {
  int rc = stage_frames(h, nframes, off, boxes, coords, types, ws, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  return stage_nlist(h, A, st);
}

static int run_model(dp_handle h, const Plan& P, const NlistArgs& A, void* ws, hipStream_t st,
                     double* energies, double* forces, double* virials, double* atom_energy,
                     bool want_forces, double* T_out, double* gT_out, bool forces_zeroed = false,
                     bool want_energy = true, bool fb_zeroed = false, double* atom_virial = nullptr,
                     const Frame* reduce_frames = nullptr, int ncentre = 0) {
  Ws W{(char*)ws, &P};
  EmbedArgs E{};
  E.prec = h->opt.precision;
  E.nrows = P.nrows;
  E.n = P.n;
  E.m = A.m;
  E.nets = h->d_nets;
  E.xe = A.xe;
  E.nlist = A.nlist;
  E.nnei = A.nnei;
  E.row_atom = A.row_atom;
  E.type_row0 = A.type_row0;
  E.eown = A.eown;
  E.T = W.at<void>(P.o_T);
  E.gT = W.at<void>(P.o_gT);
  E.forces = forces;
  E.gbuf = h->opt.deterministic ? W.at<double>(P.o_gbuf) : nullptr;
  E.vir_part = W.at<double>(P.o_vir);
  E.frame_of = A.frame_of;
  E.nframes = P.nframes;
  if (h->student_on) {
    E.snets = h->d_student;
    memcpy(E.st_lo, h->st_lo, sizeof(E.st_lo));
    memcpy(E.st_hi, h->st_hi, sizeof(E.st_hi));
    E.fb_list = W.at<int2>(P.o_fb);
    E.fb_count = W.at<int>(P.o_fbcnt);
    E.fb_cap = P.n * h->nm;
    E.fb_note = A.status + STW_FALLBACK;   // reported by dp_fallback_rows
    E.theta = h->d_theta;
    E.net_off = h->d_net_off;
    E.etype = A.etype;
    if (!fb_zeroed) launch_zero_int(E.fb_count, 1, st);
  }
  {
    StageTimer tm(h, DP_STAGE_EMBED_FWD, st);
    if (h->student_on) launch_student_fwd(E, st);
    else launch_embed_fwd(E, st);
  }
  if (h->student_on) {
    StageTimer tm(h, DP_STAGE_FALLBACK, st);
    launch_fallback_fwd(E, st);
  }
  HIPCHECK(h, hipGetLastError());
  FitArgs F{};
  F.prec = h->opt.precision;
  F.nrows = P.nrows;
  F.n = P.n;
  F.m = A.m;
  F.nfit = h->n_fit;
  F.fw = h->fit_w[0];
  F.type_row0 = A.type_row0;
  F.row_atom = A.row_atom;
  F.T = E.T;
  F.gT = W.at<void>(P.o_gT);
  F.W = (const void* const*)h->d_ptrs;
  F.b = (const void* const*)h->d_ptrs + h->ntypes * h->n_fit;
  F.wo = (const void* const*)h->d_ptrs + 2 * h->ntypes * h->n_fit;
  F.Wb = (const void* const*)h->d_ptrs + 2 * h->ntypes * h->n_fit + h->ntypes;
  F.Wf = F.Wb + 4 * h->ntypes * h->n_fit;
  F.bo = h->d_bo;
  F.D = W.at<void>(P.o_D);
  F.Dg = W.at<void>(P.o_Dg);
  F.act = W.at<void>(P.o_act);
  F.xs = W.at<void>(P.o_xs);
  F.g0 = W.at<void>(P.o_g0);
  F.g1 = W.at<void>(P.o_g1);
  F.Ei = W.at<double>(P.o_Ei);
  {
    StageTimer tm(h, DP_STAGE_FIT, st);
    launch_fit(F, st);
  }
  HIPCHECK(h, hipGetLastError());
  if (T_out || gT_out) {
    launch_export_T(h->opt.precision, P.n, h->M, A.row_of, E.T, F.gT, T_out, gT_out, st);
    HIPCHECK(h, hipGetLastError());
  }
  if (want_forces) {
    if (!forces_zeroed) launch_zero(forces, (size_t)P.n * 3, st);
    {
      StageTimer tm(h, DP_STAGE_EMBED_BWD, st);
      if (h->student_on) launch_student_bwd(E, st);
      else launch_embed_bwd(E, st);
    }
    if (h->student_on) {
      StageTimer tm(h, DP_STAGE_FALLBACK, st);
      launch_fallback_bwd(E, st);
    }
    if (E.gbuf) {
      StageTimer tm(h, DP_STAGE_REDUCE, st);
      int* rs = W.at<int>(P.o_rev);
      launch_rev_gather(P.n, h->nm, A.nlist, A.eown, E.gbuf, forces, rs,
                        A.scan_sums, rs + rev_scratch_ints(P.n, h->nm), A.status, st);
    }
  }
  HIPCHECK(h, hipGetLastError());
  if (atom_virial && want_forces) {
    launch_export_atom_virial(ncentre > 0 ? ncentre : P.n, A.row_of, E.vir_part, atom_virial, st);
    HIPCHECK(h, hipGetLastError());
  }
  if (want_energy) {
    StageTimer tm(h, DP_STAGE_REDUCE, st);
    launch_frame_reduce(P.nframes, P.max_frame_atoms, reduce_frames ? reduce_frames : A.frames, A.row_of, F.Ei,
                        want_forces ? E.vir_part : nullptr, energies, virials, atom_energy,
                        W.at<double>(P.o_redpart), st);
  }
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}


extern "C" {

const char* dp_strerror(int code) {
  switch (code) {
    case DP_OK: return "ok";
    case DP_WARN_SEL_OVERFLOW: return "a neighbour-type block exceeded sel; nearest kept";
    case DP_ERR_ARG: return "invalid argument";
    case DP_ERR_MODEL: return "invalid or unsupported model";
    case DP_ERR_BOX: return "singular or left-handed box";
    case DP_ERR_TYPE: return "atom type out of range";
    case DP_ERR_CAPACITY: return "neighbour or ghost capacity exceeded";
    case DP_ERR_WORKSPACE: return "workspace too small";
    case DP_ERR_HIP: return "HIP runtime error";
    case DP_ERR_NONFINITE: return "non-finite coordinate";
    case DP_ERR_OVERLAP: return "two atoms closer than 1e-6 A";
    default: return "unknown status";
  }
}

const char* dp_last_error(dp_handle h) { return h ? h->err.c_str() : g_init_err.c_str(); }

int dp_init(const char* model_path, const dp_options* opt, dp_handle* out) {
  if (!out) return fail(nullptr, DP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!model_path) return fail(nullptr, DP_ERR_ARG, "model_path is NULL");
  dp_handle h = new dp_handle_s();
  if (opt) h->opt = *opt;
  if (h->opt.precision < 0 || h->opt.precision > 3 || !(h->opt.skin >= 0) ||
      (h->opt.deterministic != 0 && h->opt.deterministic != 1)) {
    delete h;
    return fail(nullptr, DP_ERR_ARG, "bad options");
  }
  int rc = parse_model(h, model_path);
  if (rc != DP_OK) {
    g_init_err = h->err;
    delete h;
    return rc;
  }
  if (bf16_mode(h->opt.precision)) {
    bool ok = (h->M * h->m2) % 8 == 0;
    for (int k = 0; k < h->n_fit; k++) ok = ok && h->fit_w[k] % 8 == 0;
    if (!ok) {
      g_init_err = "BF16 modes need M * M< and the fitting widths to be multiples of 8";
      delete h;
      return DP_ERR_ARG;
    }
  }
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, DP_ERR_HIP, "no HIP device");
  }
  if (noalloc_setup(h->device) != DP_OK) {
    delete h;
    return fail(nullptr, DP_ERR_HIP, "cannot resolve the scratch array of dp_compute_noalloc");
  }
  plan_weights(h);
  *out = h;
  return DP_OK;
}

void dp_free(dp_handle h) {
  if (!h) return;
  for (hipEvent_t e : h->prof_pool) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  delete h;
}

int dp_model_info(dp_handle h, int32_t* ntypes, int32_t* nm, int32_t* M, int32_t* m2, double* rc,
                  int64_t* nparams) {
  if (!h) return DP_ERR_ARG;
  if (ntypes) *ntypes = h->ntypes;
  if (nm) *nm = h->nm;
  if (M) *M = h->M;
  if (m2) *m2 = h->m2;
  if (rc) *rc = h->rc;
  if (nparams) *nparams = h->nparams;
  return DP_OK;
}

int dp_device_bytes(dp_handle h, size_t* weight_bytes) {
  if (!h || !weight_bytes) return fail(h, DP_ERR_ARG, "null argument");
  *weight_bytes = h->w_total;
  return DP_OK;
}

int dp_upload(dp_handle h, void* weights, size_t bytes, void* stream) {
  if (!h || !weights) return fail(h, DP_ERR_ARG, "null argument");
  if (bytes < h->w_total)
    return fail(h, DP_ERR_WORKSPACE, "weight buffer too small: need " + std::to_string(h->w_total) + " bytes");
  if (((uintptr_t)weights & 255) != 0) return fail(h, DP_ERR_ARG, "weight buffer must be 256-byte aligned");
  return bind_weights(h, weights, (hipStream_t)stream);
}

int dp_workspace_size(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* boxes,
                      size_t* bytes) {
  if (!h || !atom_offsets || !boxes || !bytes) return fail(h, DP_ERR_ARG, "null argument");
  Plan P;
  int rc = make_plan(h, nframes, atom_offsets, boxes, nullptr, P);
  if (rc != DP_OK) return rc;
  *bytes = P.total;
  if (h->opt.skin > 0 && nframes == 1) {
    Plan V;
    rc = make_plan(h, nframes, atom_offsets, boxes, nullptr, V, true);
    if (rc != DP_OK) return rc;
    *bytes = std::max(*bytes, V.total);
  }
  return DP_OK;
}

int dp_compute_batch(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* coords,
                     const int32_t* types, const double* boxes, double* energies, double* forces,
                     double* virials, double* atom_energy, void* workspace, size_t ws_bytes,
                     void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!atom_offsets || !boxes || !energies || !forces)
    return fail(h, DP_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  Plan P;
  NlistArgs A{};
  int rc = stage_frames_and_nlist(h, nframes, atom_offsets, boxes, coords, types, workspace, ws_bytes,
                                  st, P, A);
  if (rc != DP_OK) return rc;
  return run_model(h, P, A, workspace, st, energies, forces, virials, atom_energy, true, nullptr,
                   nullptr);
}

int dp_compute(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
               const double* box, double* energy, double* forces, double* virial,
               double* atom_energy, void* workspace, size_t ws_bytes, void* stream) {
  int64_t off[2] = {0, natoms};
  return dp_compute_batch(h, 1, off, coords, types, box, energy, forces, virial, atom_energy,
                          workspace, ws_bytes, stream);
}

int dp_compute_atomic(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                      const double* box, double* energy, double* forces, double* virial, double* atom_energy,
                      double* atom_virial, void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!box || !energy || !forces) return fail(h, DP_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  int rc = stage_frames_and_nlist(h, 1, off, box, coords, types, workspace, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  return run_model(h, P, A, workspace, st, energy, forces, virial, atom_energy, true, nullptr, nullptr, false,
                   true, false, atom_virial);
}

// The frame of an evaluation with caller-supplied ghost atoms: an orthogonal box whose
// edges exceed the atoms' extent by rc + 1 A, so that no periodic image of any atom comes
// within rc of another atom and the periodic machinery sees the open cluster.
static int local_box(dp_handle h, const double* bounds, double box[9]) {
  for (int k = 0; k < 3; k++)
    if (!std::isfinite(bounds[k]) || !std::isfinite(bounds[3 + k]) || !(bounds[3 + k] >= bounds[k]))
      return fail(h, DP_ERR_ARG, "bounds must be finite with hi >= lo");
  for (int q = 0; q < 9; q++) box[q] = 0.0;
  for (int k = 0; k < 3; k++) box[4 * k] = (bounds[3 + k] - bounds[k]) + h->rc + 1.0;
  return DP_OK;
}

int dp_compute_local_workspace_size(dp_handle h, int64_t nlocal, int64_t nghost, const double* bounds,
                                    size_t* bytes) {
  if (!h || !bounds || !bytes) return fail(h, DP_ERR_ARG, "null argument");
  if (nlocal < 1 || nghost < 0) return fail(h, DP_ERR_ARG, "nlocal must be >= 1 and nghost >= 0");
  double box[9];
  int rc = local_box(h, bounds, box);
  if (rc != DP_OK) return rc;
  int64_t off[2] = {0, nlocal + nghost};
  Plan P;
  rc = make_plan(h, 1, off, box, nullptr, P);
  if (rc != DP_OK) return rc;
  *bytes = P.total;
  return DP_OK;
}

int dp_compute_local(dp_handle h, int64_t nlocal, int64_t nghost, const double* coords, const int32_t* types,
                     const double* bounds, double* energy, double* forces, double* virial, double* atom_energy,
                     double* atom_virial, void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!bounds || !energy || !forces) return fail(h, DP_ERR_ARG, "null argument");
  if (nlocal < 1 || nghost < 0) return fail(h, DP_ERR_ARG, "nlocal must be >= 1 and nghost >= 0");
  if (h->opt.deterministic)
    return fail(h, DP_ERR_ARG, "caller-supplied ghost atoms are not available in deterministic mode");
  double box[9];
  int rc = local_box(h, bounds, box);
  if (rc != DP_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, nlocal + nghost};
  Plan P;
  NlistArgs A{};
  rc = stage_frames(h, 1, off, box, coords, types, workspace, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  A.ncentre = (int)nlocal;
  // the reductions (energy, virial, E_i) run over the centres only
  Ws W{(char*)workspace, &P};
  {
    Frame Fr{};
    if (box_setup(box, h->rc, Fr)) return fail(h, DP_ERR_BOX, "degenerate bounds");
    Fr.atom0 = 0;
    Fr.natoms = (int)nlocal;
    launch_put_frames(&Fr, 1, W.at<Frame>(P.o_frames_red), st);
  }
  rc = stage_nlist(h, A, st);
  if (rc != DP_OK) return rc;
  return run_model(h, P, A, workspace, st, energy, forces, virial, atom_energy, true, nullptr, nullptr, false,
                   true, false, atom_virial, W.at<Frame>(P.o_frames_red), (int)nlocal);
}

int dp_nlist(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
             const double* box, int32_t* nlist, int32_t* img, int32_t* nnei, void* workspace,
             size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!box || !nlist) return fail(h, DP_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  int rc = stage_frames_and_nlist(h, 1, off, box, coords, types, workspace, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  launch_nlist_export(P.n, h->nm, A.nlist, A.eown, A.eimg, A.frame_of, A.frames, nlist, img, st);
  if (nnei)
    HIPCHECK(h, hipMemcpyAsync(nnei, A.nnei, sizeof(int) * P.n * h->ntypes, hipMemcpyDeviceToDevice, st));
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

int dp_descriptor(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                  const double* box, double* T, double* gT, void* workspace, size_t ws_bytes,
                  void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!box) return fail(h, DP_ERR_ARG, "null box");
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  int rc = stage_frames_and_nlist(h, 1, off, box, coords, types, workspace, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  Ws W{(char*)workspace, &P};
  double* e = W.at<double>(P.o_tmpj);
  return run_model(h, P, A, workspace, st, e, nullptr, nullptr, nullptr, false, T, gT);
}

int dp_md_run(dp_handle h, int64_t natoms, double* x, double* v, const int32_t* types,
              const double* masses, const double* box, double dt_fs, int32_t nsteps,
              int32_t thermo_every, double* thermo, double* forces, void* workspace,
              size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!x || !v || !types || !masses || !box) return fail(h, DP_ERR_ARG, "null argument");
  if (nsteps < 0 || thermo_every < 0 || !(dt_fs > 0) || !std::isfinite(dt_fs))
    return fail(h, DP_ERR_ARG, "bad step count or time step");
  MDMass mm{};
  for (int t = 0; t < h->ntypes; t++) {
    if (!(masses[t] > 0) || !std::isfinite(masses[t])) return fail(h, DP_ERR_ARG, "masses must be > 0");
    mm.m[t] = masses[t];
    mm.inv[t] = 1.0 / masses[t];
  }
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  const bool verlet = h->opt.skin > 0;
  int rc = stage_frames(h, 1, off, box, x, types, workspace, ws_bytes, st, P, A, verlet);
  if (rc != DP_OK) return rc;
  if (verlet) launch_fill_int((int*)A.gate, 1, 1, st);  // build at the first step
  Ws W{(char*)workspace, &P};
  double* F = forces ? forces : W.at<double>(P.o_mdF);
  double* E = W.at<double>(P.o_mdE);
  double* Wv = W.at<double>(P.o_mdW);
  double* kepart = W.at<double>(P.o_redpart);   // free once the frame reduction is done
  const double* B = box;
  double vol = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
               B[2] * (B[3] * B[7] - B[4] * B[6]);
  const int n = (int)natoms;
  // the skin check runs inside every drift of the loop (none before the first force)
  VvCheck chk{};
  if (verlet) {
    chk.xref = A.xref;
    chk.lim2 = 0.25 * h->opt.skin * h->opt.skin;
    chk.gate = (int*)A.gate;
    chk.nc1 = A.ncell + 1;
    chk.c1 = A.cell_count;
    chk.nc2 = A.ncell;
    chk.c2 = A.cell_fill;
  }
  // with the Verlet list, k_update_ext also clears the fallback-row counter of the students
  int* fb_clear = (verlet && h->student_on) ? W.at<int>(P.o_fbcnt) : nullptr;
  // energies and virials are summed only when a thermo row needs them
  auto force = [&](bool f_zeroed, bool disp_done, bool want_energy) -> int {
    if (verlet) {
      StageTimer tm(h, DP_STAGE_NLIST, st);
      launch_nlist_verlet(A, 0.5 * h->opt.skin, disp_done, fb_clear, st);
      A.skip_rows = true;   // the species row order is fixed after the first build
      HIPCHECK(h, hipGetLastError());
    } else {
      int r = stage_nlist(h, A, st);
      if (r != DP_OK) return r;
    }
    return run_model(h, P, A, workspace, st, E, F, Wv, nullptr, true, nullptr, nullptr, f_zeroed, want_energy,
                     fb_clear != nullptr);
  };
  rc = force(false, false, thermo != nullptr);
  if (rc != DP_OK) return rc;
  int row = 0;
  if (thermo) launch_thermo(n, types, mm, vol, 0, v, E, Wv, thermo + 6 * row++, kepart, st);
  // Velocity Verlet: half kick + drift, forces, half kick.  Between two steps without a
  // thermo row the closing half kick and the next opening half kick + drift run as one
  // kernel, which also clears F for the next force evaluation.
  bool opened = false;   // the current step's opening half kick + drift is done
  for (int s = 1; s <= nsteps; s++) {
    if (!opened) {
      StageTimer tm(h, DP_STAGE_MD, st);
      launch_vv(n, types, mm, dt_fs, F, v, x, true, chk, st);
    }
    const bool thermo_row = thermo && thermo_every > 0 && s % thermo_every == 0;
    rc = force(opened, true, thermo_row);
    if (rc != DP_OK) return rc;
    StageTimer tm(h, DP_STAGE_MD, st);
    if (thermo_row || s == nsteps) {
      launch_vv(n, types, mm, dt_fs, F, v, x, false, chk, st);
      if (thermo_row) launch_thermo(n, types, mm, vol, s, v, E, Wv, thermo + 6 * row++, kepart, st);
      opened = false;
    } else {
      launch_vv_merged(n, types, mm, dt_fs, F, v, x, chk, st);
      opened = true;
    }
  }
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

int dp_md_npt_workspace_size(dp_handle h, int64_t natoms, const double* box, double min_scale, size_t* bytes) {
  if (!h || !box || !bytes) return fail(h, DP_ERR_ARG, "null argument");
  if (!(h->opt.skin > 0)) return fail(h, DP_ERR_ARG, "isobaric MD needs a handle with a neighbour skin > 0");
  if (!(min_scale > 0.5 && min_scale <= 1.0)) return fail(h, DP_ERR_ARG, "min_scale must be in (0.5, 1]");
  int64_t off[2] = {0, natoms};
  Plan P;
  int rc = make_plan(h, 1, off, box, nullptr, P, true, min_scale);
  if (rc != DP_OK) return rc;
  *bytes = P.total;
  return DP_OK;
}

int dp_md_run_npt(dp_handle h, int64_t natoms, double* x, double* v, const int32_t* types, const double* masses,
                  const double* box, const dp_npt_options* npt, double dt_fs, int32_t nsteps,
                  int32_t thermo_every, double* thermo, double* box_out, double* state_out, double* forces,
                  void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!x || !v || !types || !masses || !box || !npt) return fail(h, DP_ERR_ARG, "null argument");
  if (!(h->opt.skin > 0)) return fail(h, DP_ERR_ARG, "isobaric MD needs a handle with a neighbour skin > 0");
  if (nsteps < 0 || thermo_every < 0 || !(dt_fs > 0) || !std::isfinite(dt_fs))
    return fail(h, DP_ERR_ARG, "bad step count or time step");
  if (!(npt->tau_p_fs > 0) || !(npt->temperature_K > 0) || !std::isfinite(npt->pressure_bar) ||
      !(npt->tau_t_fs >= 0) || !(npt->min_scale > 0.5 && npt->min_scale <= 1.0))
    return fail(h, DP_ERR_ARG, "bad isobaric options (tau_p > 0, T > 0, tau_t >= 0, min_scale in (0.5, 1])");
  if (natoms < 2) return fail(h, DP_ERR_ARG, "isobaric MD needs at least two atoms");
  MDMass mm{};
  for (int t = 0; t < h->ntypes; t++) {
    if (!(masses[t] > 0) || !std::isfinite(masses[t])) return fail(h, DP_ERR_ARG, "masses must be > 0");
    mm.m[t] = masses[t];
    mm.inv[t] = 1.0 / masses[t];
  }
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  int rc = stage_frames(h, 1, off, box, x, types, workspace, ws_bytes, st, P, A, true, npt->min_scale);
  if (rc != DP_OK) return rc;
  Ws W{(char*)workspace, &P};
  double* S = W.at<double>(P.o_npt);
  A.npt = S;
  launch_fill_int((int*)A.gate, 1, 1, st);   // build at the first step
  // constants of the run; the plan's frame (box_setup at the enlarged radius) carries the
  // initial box and its inverse
  NptConst c{};
  {
    Frame F0{};
    if (box_setup(box, h->rc, F0)) return fail(h, DP_ERR_BOX, "singular or left-handed box");
    for (int k = 0; k < 9; k++) {
      c.B0[k] = F0.B[k];
      c.Bi0[k] = F0.Bi[k];
    }
  }
  const double* B = box;
  c.V0 = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) + B[2] * (B[3] * B[7] - B[4] * B[6]);
  c.nf = 3.0 * (double)natoms - 3.0;
  c.alpha = 1.0 + 3.0 / c.nf;
  c.kT = 8.617333262e-5 * npt->temperature_K;
  c.W = (c.nf + 3.0) * c.kT * npt->tau_p_fs * npt->tau_p_fs;
  c.thermostat = npt->tau_t_fs > 0 ? 1 : 0;
  c.Q = c.thermostat ? c.nf * c.kT * npt->tau_t_fs * npt->tau_t_fs : 1.0;
  c.pext = npt->pressure_bar / 1.602176634e6;
  c.h = 0.5 * dt_fs;
  c.dt = dt_fs;
  c.rl = h->rc + h->opt.skin;
  c.rc = h->rc;
  c.min_scale = npt->min_scale;
  const int n = (int)natoms;
  double* F = forces ? forces : W.at<double>(P.o_mdF);
  double* E = W.at<double>(P.o_mdE);
  double* Wv = W.at<double>(P.o_mdW);
  VvCheck chk{};
  chk.xref = A.xref;
  chk.gate = (int*)A.gate;
  chk.nc1 = A.ncell + 1;
  chk.c1 = A.cell_count;
  chk.nc2 = A.ncell;
  chk.c2 = A.cell_fill;
  int* fb_clear = h->student_on ? W.at<int>(P.o_fbcnt) : nullptr;
  // every step sums energy and virial: the barostat needs tr W
  auto force = [&](bool f_zeroed, bool disp_done) -> int {
    {
      StageTimer tm(h, DP_STAGE_NLIST, st);
      launch_nlist_verlet(A, 0.5 * h->opt.skin, disp_done, fb_clear, st);
      A.skip_rows = true;
      HIPCHECK(h, hipGetLastError());
    }
    return run_model(h, P, A, workspace, st, E, F, Wv, nullptr, true, nullptr, nullptr, f_zeroed, true,
                     fb_clear != nullptr);
  };
  launch_npt_init(n, types, mm, v, S, c, st);
  rc = force(false, false);
  if (rc != DP_OK) return rc;
  int row = 0;
  if (thermo) launch_npt_close(n, types, mm, v, S, c, E, Wv, 0, thermo + 8 * row++, false, st);
  for (int s = 1; s <= nsteps; s++) {
    {
      StageTimer tm(h, DP_STAGE_MD, st);
      launch_npt_open(S, c, Wv, W.at<Frame>(P.o_frames), A.status, st);
      launch_vv_npt_open(n, types, mm, F, v, x, S, chk, st);
    }
    rc = force(true, true);
    if (rc != DP_OK) return rc;
    StageTimer tm(h, DP_STAGE_MD, st);
    launch_vv_npt_close(n, types, mm, F, v, S, st);
    const bool thermo_row = thermo && thermo_every > 0 && s % thermo_every == 0;
    launch_npt_close(n, types, mm, v, S, c, E, Wv, s, thermo_row ? thermo + 8 * row++ : nullptr, true, st);
  }
  launch_npt_finish(n, v, S, W.at<Frame>(P.o_frames), box_out, state_out, st);
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

int dp_set_params(dp_handle h, const double* theta, void* stream) {
  if (!h || !theta) return fail(h, DP_ERR_ARG, "null argument");
  if (need_weights(h) != DP_OK) return DP_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(h, hipMemcpyAsync(h->d_theta, theta, sizeof(double) * h->nparams, hipMemcpyDeviceToDevice, st));
  return refresh_weights(h, st);
}

int dp_get_params(dp_handle h, double* theta, void* stream) {
  if (!h || !theta) return fail(h, DP_ERR_ARG, "null argument");
  if (need_weights(h) != DP_OK) return DP_ERR_ARG;
  HIPCHECK(h, hipMemcpyAsync(theta, h->d_theta, sizeof(double) * h->nparams, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
  return DP_OK;
}

struct PGLayout {
  size_t o_base, o_sums, o_pgmap, o_pgnets, o_gtan, o_scr, scr_bytes, total;
  long np_max;
};

static PGLayout pg_layout(dp_handle h, const Plan& P) {
  PGLayout L{};
  size_t o = P.total;
  auto take = [&](size_t bytes) { size_t r = o; o = al(o + bytes); return r; };
  L.o_base = take(sizeof(int) * (size_t)h->ntypes * (P.nrows + 1));
  L.o_sums = take(sizeof(int) * (scan_sums_ints(P.nrows + 1, 1) + 16));
  L.o_pgmap = take(sizeof(int) * h->h_pgmap.size());        // FP64 position-packed nets <- theta
  L.o_pgnets = take(sizeof(double) * h->h_pgmap.size());
  L.o_gtan = take(sizeof(double) * h->nparams);
  L.np_max = (long)P.n * h->nm;
  L.scr_bytes = param_grad_scratch_bytes(P.nrows, L.np_max, h->M, h->m2, h->s0, h->fit_w[0], h->n_fit);
  L.o_scr = take(L.scr_bytes);
  L.total = o;
  return L;
}

// The batch runs in chunks of whole frames, greedily packed up to max_atoms atoms (a
// larger frame is a chunk of its own): the workspace holds the largest chunk's plan, so it
// is bounded by the chunk size, not by the batch.
static constexpr int64_t kPgChunkAtoms = 32768;

static int pg_chunks(int32_t nframes, const int64_t* off, int64_t max_atoms,
                     const std::function<int(int32_t, int32_t)>& fn) {
  if (max_atoms <= 0) max_atoms = kPgChunkAtoms;
  int32_t f0 = 0;
  while (f0 < nframes) {
    int32_t f1 = f0 + 1;
    while (f1 < nframes && off[f1 + 1] - off[f0] <= max_atoms) f1++;
    int rc = fn(f0, f1);
    if (rc != DP_OK) return rc;
    f0 = f1;
  }
  return DP_OK;
}

static std::vector<int64_t> pg_sub_offsets(const int64_t* off, int32_t f0, int32_t f1) {
  std::vector<int64_t> sub((size_t)(f1 - f0) + 1);
  for (int32_t f = f0; f <= f1; f++) sub[(size_t)(f - f0)] = off[f] - off[f0];
  return sub;
}

int dp_param_grad_workspace_size(dp_handle h, int32_t nframes, const int64_t* atom_offsets,
                                 const double* boxes, int64_t max_atoms, size_t* bytes) {
  if (!h || !atom_offsets || !boxes || !bytes) return fail(h, DP_ERR_ARG, "null argument");
  if (nframes < 1) return fail(h, DP_ERR_ARG, "nframes must be >= 1");
  size_t need = 0;
  int rc = pg_chunks(nframes, atom_offsets, max_atoms, [&](int32_t f0, int32_t f1) {
    const std::vector<int64_t> sub = pg_sub_offsets(atom_offsets, f0, f1);
    Plan P;
    int r = make_plan(h, f1 - f0, sub.data(), boxes + 9 * (size_t)f0, nullptr, P);
    if (r != DP_OK) return r;
    need = std::max(need, pg_layout(h, P).total);
    return (int)DP_OK;
  });
  if (rc != DP_OK) return rc;
  *bytes = need;
  return DP_OK;
}

static int param_grad_chunk(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* coords,
                            const int32_t* types, const double* boxes, const double* gE, const double* gF,
                            double* gtheta, void* workspace, size_t ws_bytes, hipStream_t st);

int dp_param_grad(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* coords,
                  const int32_t* types, const double* boxes, const double* gE, const double* gF,
                  double* gtheta, int64_t max_atoms, void* workspace, size_t ws_bytes, void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!atom_offsets || !boxes || !gE || !gF || !gtheta || !coords || !types)
    return fail(h, DP_ERR_ARG, "null argument");
  if (nframes < 1) return fail(h, DP_ERR_ARG, "nframes must be >= 1");
  return pg_chunks(nframes, atom_offsets, max_atoms, [&](int32_t f0, int32_t f1) {
    const std::vector<int64_t> sub = pg_sub_offsets(atom_offsets, f0, f1);
    const int64_t a0 = atom_offsets[f0];
    return param_grad_chunk(h, f1 - f0, sub.data(), coords + 3 * a0, types + a0, boxes + 9 * (size_t)f0, gE + f0,
                            gF + 3 * a0, gtheta, workspace, ws_bytes, (hipStream_t)stream);
  });
}

// one chunk of frames (offsets rebased to its first atom)
static int param_grad_chunk(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* coords,
                            const int32_t* types, const double* boxes, const double* gE, const double* gF,
                            double* gtheta, void* workspace, size_t ws_bytes, hipStream_t st) {
  Plan P;
  NlistArgs A{};
  {
    Plan Q;
    int rc = make_plan(h, nframes, atom_offsets, boxes, nullptr, Q);
    if (rc != DP_OK) return rc;
    if (!workspace || ws_bytes < pg_layout(h, Q).total)
      return fail(h, DP_ERR_WORKSPACE, "workspace too small for dp_param_grad");
  }
  int rc = stage_frames_and_nlist(h, nframes, atom_offsets, boxes, coords, types, workspace, ws_bytes, st,
                                  P, A);
  if (rc != DP_OK) return rc;
  PGLayout L = pg_layout(h, P);
  Ws W{(char*)workspace, &P};
  const int nt = h->ntypes, nrows = P.nrows;
  int* base = W.at<int>(L.o_base);
  int* sums = W.at<int>(L.o_sums);
  // the scans' totals go after their block sums (scan_sums_ints ints, one per block of a
  // multi-block scan): totals inside that range would overwrite a block's prefix
  int* totals = sums + scan_sums_ints(nrows + 1, 1) + 8;
  for (int b = 0; b < nt; b++)
    launch_pair_scan(nrows, nt, b, A.row_atom, A.nnei, base + (size_t)b * (nrows + 1), sums, totals + b, st);
  HIPCHECK(h, hipGetLastError());
  // the pair-row groups size the GEMMs: read them back (one synchronisation)
  std::vector<int> hb((size_t)nt * (nrows + 1)), tr0(nt + 1);
  HIPCHECK(h, hipMemcpyAsync(hb.data(), base, sizeof(int) * hb.size(), hipMemcpyDeviceToHost, st));
  HIPCHECK(h, hipMemcpyAsync(tr0.data(), A.type_row0, sizeof(int) * (nt + 1), hipMemcpyDeviceToHost, st));
  HIPCHECK(h, hipStreamSynchronize(st));
  int32_t stw[STW_N];
  HIPCHECK(h, hipMemcpy(stw, A.status, sizeof(stw), hipMemcpyDeviceToHost));
  if (stw[STW_FLAGS] & (ST_BAD_TYPE | ST_NONFINITE | ST_OVERLAP | ST_GHOST_CAP | ST_CAPACITY))
    return dp_status(h, workspace, st, nullptr, nullptr);
  PGradArgs G{};
  G.m = A.m;
  G.nrows = nrows;
  G.fw = h->fit_w[0];
  G.nfit = h->n_fit;
  long np = 0;
  for (int b = 0; b < nt; b++) {
    G.base[b] = base + (size_t)b * (nrows + 1);
    G.boff[b] = (int)np;
    np += hb[(size_t)b * (nrows + 1) + nrows];
  }
  if (np > L.np_max) return fail(h, DP_ERR_CAPACITY, "pair rows exceed the workspace plan");
  G.np = (int)np;
  for (int a = 0; a < nt; a++)
    for (int b = 0; b < nt; b++) {
      const int* bb = hb.data() + (size_t)b * (nrows + 1);
      G.group[(a * nt + b) * 2] = G.boff[b] + bb[tr0[a]];
      G.group[(a * nt + b) * 2 + 1] = bb[tr0[a + 1]] - bb[tr0[a]];
    }
  for (int t = 0; t <= nt; t++) G.type_row0_h[t] = tr0[t];
  // the embedding nets in FP64 at the force path's positions, whatever the precision option
  int* pgmap = W.at<int>(L.o_pgmap);
  double* pgnets = W.at<double>(L.o_pgnets);
  HIPCHECK(h, hipMemcpyAsync(pgmap, h->h_pgmap.data(), sizeof(int) * h->h_pgmap.size(), hipMemcpyHostToDevice, st));
  launch_scatter_params(0, h->h_pgmap.size(), pgmap, h->d_theta, pgnets, st);
  G.nets = pgnets;
  G.type_row0 = A.type_row0;
  ParamIndex PI = index_params(h);
  G.eW = PI.eW.data();
  G.eB = PI.eB.data();
  G.fW = PI.fW.data();
  G.fB = PI.fB.data();
  G.theta = h->d_theta;
  double* gtan = W.at<double>(L.o_gtan);
  launch_zero(gtan, h->nparams, st);
  G.gtheta_tan = gtan;
  G.row_atom = A.row_atom;
  G.nnei = A.nnei;
  G.nlist = A.nlist;
  G.eown = A.eown;
  G.xe = A.xe;
  G.vdir = gF;
  G.gE = gE;
  G.frame_of = A.frame_of;
  G.scratch = W.at<void>(L.o_scr);
  G.scratch_bytes = L.scr_bytes;
  if (launch_param_grad(G, st) != 0) return fail(h, DP_ERR_WORKSPACE, "param-grad scratch too small");
  launch_axpy(h->nparams, -1.0, gtan, gtheta, st);
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

// bytes of the student region: the index map, then the blocks in the storage type
static size_t student_map_bytes(dp_handle h) {
  return (sizeof(int) * (size_t)h->ntypes * h->ntypes * kStuElems + 255) & ~(size_t)255;
}
static size_t student_region_bytes(dp_handle h) {
  return student_map_bytes(h) + (size_t)h->ntypes * h->ntypes * kStuElems * storage_bytes(h->opt.precision);
}

int dp_student_bytes(dp_handle h, size_t* bytes) {
  if (!h || !bytes) return fail(h, DP_ERR_ARG, "null argument");
  *bytes = student_region_bytes(h);
  return DP_OK;
}

int dp_set_student(dp_handle h, int32_t hidden, const double* theta_s, const double* s_lo,
                   const double* s_hi, int32_t enable, void* student_mem, size_t student_bytes,
                   void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!enable) {
    h->student_on = false;
    return DP_OK;
  }
  if (!theta_s || !s_lo || !s_hi || hidden < 1 || hidden > kP0)
    return fail(h, DP_ERR_ARG, "student: bad arguments (hidden must be 1..32)");
  if (h->opt.deterministic) return fail(h, DP_ERR_ARG, "student nets are not available in deterministic mode");
  if (!student_mem || ((uintptr_t)student_mem & 255) != 0)
    return fail(h, DP_ERR_ARG, "student buffer must be non-NULL and 256-byte aligned");
  if (student_bytes < student_region_bytes(h))
    return fail(h, DP_ERR_WORKSPACE,
                "student buffer too small: need " + std::to_string(student_region_bytes(h)) + " bytes");
  for (int q = 0; q < h->ntypes * h->ntypes; q++)
    if (!(s_lo[q] <= s_hi[q]) || !std::isfinite(s_lo[q]) || !std::isfinite(s_hi[q]))
      return fail(h, DP_ERR_ARG, "student: every range needs finite s_lo <= s_hi");
  const int nnet = h->ntypes * h->ntypes, M = h->M;
  const size_t size = 2 * (size_t)hidden + (size_t)hidden * M + M;
  // student blocks: FP64 in the FP64 mode, FP32 otherwise (the student kernels have no
  // per-neighbour matrix product, so the BF16 operand modes do not apply to them)
  const size_t blk = (size_t)kStuElems;
  std::vector<int>& map = h->h_student_map;
  map.assign((size_t)nnet * blk, -1);
  for (int net = 0; net < nnet; net++) {
    int* b = map.data() + (size_t)net * blk;
    size_t o = net * size;
    for (int j = 0; j < hidden; j++) {
      b[kSW1 + j] = (int)(o + j);
      b[kSB1 + j] = (int)(o + hidden + j);
    }
    for (int f = 0; f < M; f++) {
      b[kSB2 + f] = (int)(o + 2 * hidden + (size_t)hidden * M + f);
      for (int j = 0; j < hidden; j++) {
        b[kSW2 + j * kP2 + f] = (int)(o + 2 * hidden + (size_t)j * M + f);
        b[kSW2T + f * kP0 + j] = (int)(o + 2 * hidden + (size_t)j * M + f);
      }
    }
  }
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(h, hipSetDevice(h->device));
  h->d_student_map = (int*)student_mem;
  h->d_student = (char*)student_mem + student_map_bytes(h);
  h->student_hidden = hidden;
  HIPCHECK(h, hipMemcpyAsync(h->d_student_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice, st));
  launch_scatter_params(h->opt.precision == PREC_FP64 ? 0 : 1, (size_t)nnet * kStuElems, h->d_student_map, theta_s,
                        h->d_student, st);
  HIPCHECK(h, hipGetLastError());
  // the host map above is read by the copy: wait for it
  HIPCHECK(h, hipStreamSynchronize(st));
  for (int q = 0; q < nnet; q++) {
    h->st_lo[q] = s_lo[q];
    h->st_hi[q] = s_hi[q];
  }
  h->student_on = true;
  return DP_OK;
}

int dp_student_samples(dp_handle h, int32_t alpha, int32_t beta, int64_t natoms, const double* coords,
                       const int32_t* types, const double* box, const float* uniforms, double keep_prob,
                       double* s_out, int64_t cap, int64_t* count, void* workspace, size_t ws_bytes,
                       void* stream) {
  if (!h) return DP_ERR_ARG;
  if (!box || !uniforms || !s_out || !count || cap < 0) return fail(h, DP_ERR_ARG, "null argument");
  if (alpha < 0 || alpha >= h->ntypes || beta < 0 || beta >= h->ntypes) return fail(h, DP_ERR_ARG, "bad species");
  hipStream_t st = (hipStream_t)stream;
  int64_t off[2] = {0, natoms};
  Plan P;
  NlistArgs A{};
  size_t extra = al(sizeof(int) * (size_t)natoms * h->nm) * 2 + al(sizeof(int) * (scan_sums_ints((int)(natoms * h->nm), 1) + 16));
  {
    Plan Q;
    int rc = make_plan(h, 1, off, box, nullptr, Q);
    if (rc != DP_OK) return rc;
    if (!workspace || ws_bytes < Q.total + extra) return fail(h, DP_ERR_WORKSPACE, "workspace too small");
  }
  int rc = stage_frames_and_nlist(h, 1, off, box, coords, types, workspace, ws_bytes, st, P, A);
  if (rc != DP_OK) return rc;
  char* base = (char*)workspace + P.total;
  int* flag = (int*)base;
  int* pos = (int*)(base + al(sizeof(int) * (size_t)natoms * h->nm));
  int* sums = (int*)(base + 2 * al(sizeof(int) * (size_t)natoms * h->nm));
  int* total = sums + scan_sums_ints((int)(natoms * h->nm), 1) + 8;
  launch_student_gather((int)natoms, A.m, alpha, beta, types, A.nnei, A.nlist, A.xe, uniforms, (float)keep_prob,
                        flag, pos, sums, total, (long)cap, s_out, st);
  HIPCHECK(h, hipGetLastError());
  int tot = 0;
  HIPCHECK(h, hipMemcpyAsync(&tot, total, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(h, hipStreamSynchronize(st));
  *count = tot;
  return dp_status(h, workspace, stream, nullptr, nullptr);
}

int dp_student_samples_workspace_size(dp_handle h, int64_t natoms, const double* box, size_t* bytes) {
  if (!h || !box || !bytes) return DP_ERR_ARG;
  int64_t off[2] = {0, natoms};
  Plan P;
  int rc = make_plan(h, 1, off, box, nullptr, P);
  if (rc != DP_OK) return rc;
  *bytes = P.total + al(sizeof(int) * (size_t)natoms * h->nm) * 2 +
           al(sizeof(int) * (scan_sums_ints((int)(natoms * h->nm), 1) + 16));
  return DP_OK;
}

int dp_embed_eval(dp_handle h, int32_t alpha, int32_t beta, int64_t n, const double* s, double* G, void* stream) {
  if (!h || !s || !G || n < 0) return fail(h, DP_ERR_ARG, "bad argument");
  if (alpha < 0 || alpha >= h->ntypes || beta < 0 || beta >= h->ntypes) return fail(h, DP_ERR_ARG, "bad species");
  if (need_weights(h) != DP_OK) return DP_ERR_ARG;
  ParamIndex PI = index_params(h);
  int net = alpha * h->ntypes + beta;
  const double* th[6];
  for (int k = 0; k < 3; k++) {
    th[2 * k] = h->d_theta + PI.eW[net * 3 + k];
    th[2 * k + 1] = h->d_theta + PI.eB[net * 3 + k];
  }
  launch_full_eval((long)n, h->s0, th, s, G, (hipStream_t)stream);
  HIPCHECK(h, hipGetLastError());
  return DP_OK;
}

int dp_student_scratch_size(int32_t hidden, int32_t M, int64_t n, size_t* bytes) {
  if (!bytes || hidden < 1 || M < 1 || n < 0) return DP_ERR_ARG;
  *bytes = student_scratch_bytes((long)n, hidden, M);
  return DP_OK;
}

int dp_student_loss_grad(int32_t hidden, int32_t M, int64_t n, const double* s, const double* G,
                         const double* theta_s, double* loss, double* grad, void* scratch,
                         size_t scratch_bytes, void* stream) {
  if (!s || !G || !theta_s || !loss || !grad || !scratch || hidden < 1 || M < 1 || n < 1) return DP_ERR_ARG;
  if (scratch_bytes < student_scratch_bytes((long)n, hidden, M)) return DP_ERR_WORKSPACE;
  launch_student_loss_grad((long)n, hidden, M, s, G, theta_s, loss, grad, scratch, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DP_OK : DP_ERR_HIP;
}

int dp_student_lsq_scratch_size(int32_t hidden, int32_t M, int64_t n, size_t* bytes) {
  if (!bytes || hidden < 1 || hidden > 32 || M < 1 || n < 0) return DP_ERR_ARG;
  *bytes = student_lsq_scratch_bytes((long)n, hidden, M);
  return DP_OK;
}

int dp_student_lsq(int32_t hidden, int32_t M, int64_t n, const double* s, const double* G, double* theta_s,
                   double ridge, void* scratch, size_t scratch_bytes, void* stream) {
  if (!s || !G || !theta_s || !scratch || hidden < 1 || hidden > 32 || M < 1 || n < 1 || !(ridge >= 0))
    return DP_ERR_ARG;
  if (scratch_bytes < student_lsq_scratch_bytes((long)n, hidden, M)) return DP_ERR_WORKSPACE;
  launch_student_lsq((long)n, hidden, M, s, G, theta_s, ridge, scratch, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DP_OK : DP_ERR_HIP;
}

int dp_adam(int64_t n, double* theta, double* m, double* v, const double* g, int32_t step, double lr,
            double beta1, double beta2, double eps, void* stream) {
  if (!theta || !m || !v || !g || n < 0 || step < 1) return DP_ERR_ARG;
  launch_adam((size_t)n, theta, m, v, g, lr, beta1, beta2, eps, step, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? DP_OK : DP_ERR_HIP;
}

int dp_profile_stages(dp_handle h, uint32_t stage_mask) {
  if (!h) return DP_ERR_ARG;
  if (stage_mask) {
    // the pooled events are reused: wait for the ones still in flight
    for (auto& r : h->prof_rec) (void)hipEventSynchronize(r.second.second);
    h->prof_rec.clear();
    h->prof_used = 0;
  }
  h->prof_on = stage_mask != 0;
  h->prof_mask = stage_mask;
  return DP_OK;
}

int dp_profile(dp_handle h, int32_t enable) {
  return dp_profile_stages(h, enable ? (1u << DP_NSTAGES) - 1u : 0u);
}

int dp_profile_read(dp_handle h, int32_t stage, double* total_ms, int64_t* launches) {
  if (!h || stage < 0 || stage >= DP_NSTAGES) return DP_ERR_ARG;
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : h->prof_rec) {
    if (r.first != stage) continue;
    HIPCHECK(h, hipEventSynchronize(r.second.second));
    float ms = 0.f;
    HIPCHECK(h, hipEventElapsedTime(&ms, r.second.first, r.second.second));
    tot += ms;
    cnt++;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return DP_OK;
}

int dp_fallback_rows(dp_handle h, const void* workspace, void* stream, int64_t* rows) {
  if (!h || !workspace || !rows) return DP_ERR_ARG;
  int st_host[STW_N];
  HIPCHECK(h, hipMemcpyAsync(st_host, workspace, sizeof(st_host), hipMemcpyDeviceToHost,
                             (hipStream_t)stream));
  HIPCHECK(h, hipStreamSynchronize((hipStream_t)stream));
  *rows = st_host[STW_FALLBACK];
  return DP_OK;
}

int dp_status(dp_handle h, const void* workspace, void* stream, int32_t* flags, int64_t* detail) {
  if (!h || !workspace) return DP_ERR_ARG;
  int st_host[STW_N];
  HIPCHECK(h, hipMemcpyAsync(st_host, workspace, sizeof(st_host), hipMemcpyDeviceToHost,
                             (hipStream_t)stream));
  HIPCHECK(h, hipStreamSynchronize((hipStream_t)stream));
  int f = st_host[STW_FLAGS];
  if (flags) *flags = f;
  int code = DP_OK;
  int64_t det = 0;
  if (f & ST_BAD_TYPE) code = DP_ERR_TYPE;
  else if (f & ST_NONFINITE) code = DP_ERR_NONFINITE;
  else if (f & ST_OVERLAP) code = DP_ERR_OVERLAP;
  else if (f & ST_GHOST_CAP) { code = DP_ERR_CAPACITY; det = st_host[STW_GHOSTS]; }
  else if (f & ST_CAPACITY) { code = DP_ERR_CAPACITY; det = st_host[STW_MAX_CAND]; }
  else if (f & ST_SEL_OVERFLOW) { code = DP_WARN_SEL_OVERFLOW; det = st_host[STW_SEL_ROWS]; }
  if (detail) *detail = det;
  if (code < 0) fail(h, code, dp_strerror(code));
  return code;
}

}  // extern "C"
