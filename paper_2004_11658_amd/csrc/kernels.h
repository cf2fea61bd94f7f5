// Host-side launch interfaces between the C ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "common.h"

struct dp_handle_s;

namespace dp {

constexpr int kRowPad = 64;   // species row groups are padded to this many rows

// ---------------------------------------------------------------- neighbour list
struct NlistArgs {
  int n, nframes, ncell, ghost_cap, nrows;
  ModelC m;
  const Frame* frames;
  const double* x;
  const int* types;
  int* status;
  int* frame_of;
  double *xw, *fw;
  int *gcount, *goff, *gtotal, *ctotal, *n_ext, *scan_sums;
  double* xe;
  int *eown, *eimg, *etype, *ecell;
  int *cell_count, *cell_start, *cell_fill, *cell_atoms;
  int *nlist, *nnei;
  int *tpos, *tcount, *row_of, *type_row0, *row_atom;
  // build kernels are skipped while *gate == 0 (NULL: always build)
  const int* gate;
  // Verlet reuse (NULL vlist: format directly within rc): wrap integers [n][3] and
  // reference positions [n][3] of the last build, image offsets [ne][3], candidate rows
  // within rl = rc + skin [n][vcap] with their counts
  int* wk;
  double* xref;
  int* eabc;
  int *vlist, *vcnt;
  int vcap;
  double rl2;
  // [ne][4]: x, y, z and the species (as a double) of each extended atom, refreshed with
  // xe at every Verlet step: one aligned 32-byte record per candidate of the per-step filter
  double* xq;
  bool skip_rows;   // leave the species-grouped row order as it is (MD after its first step)
  bool cells_zeroed;   // cell counters already cleared by the caller (MD displacement check)
  int *big, *nbig;  // atoms deferred to the second formatting pass (too many candidates or tied
                    // short keys); nbig[0] is zero on entry and left zero, nbig[1] its pass counter
  double* npt;      // isobaric MD state (NULL otherwise): a rebuild records the box scale
                    // at which the rows were built (npt[NS_LAMB] = npt[NS_LAM])
  int ncentre;      // > 0: only atoms [0, ncentre) are centres (formatted lists, species rows);
                    // the others (caller-supplied ghost atoms) are neighbours only
};
size_t scan_sums_ints(int n, int W);
// copies nframes frames from host memory to dst on the stream through kernel arguments
void launch_put_frames(const Frame* frames, int nframes, Frame* dst, hipStream_t st);
void launch_nlist(const NlistArgs& a, hipStream_t st);
// disp_done: the skin check (and the clearing of the cell counters) ran with the drift;
// clear (may be NULL): one int zeroed for the coming evaluation
void launch_nlist_verlet(const NlistArgs& a, double half_skin, bool disp_done, int* clear, hipStream_t st);
void launch_nlist_export(int n, int nm, const int* nlist, const int* eown, const int* eimg,
                         const int* frame_of, const Frame* frames, int* out_j, int* out_img,
                         hipStream_t st);

// ---------------------------------------------------------------- embedding nets
// Position-padded per-net weight block (see embed.hip): P0 = 32, P1 = 64, P2 = 128.
constexpr int kP0 = 32, kP1 = 64, kP2 = 128;
constexpr int kW1Stride = kP1 + 1, kW2Stride = kP2 + 1;
// element offsets inside one net block (same for every storage type)
constexpr int kOffW0 = 0, kOffB0 = kP0, kOffB1 = 2 * kP0, kOffB2 = 2 * kP0 + kP1;
constexpr int kOffW1 = 2 * kP0 + kP1 + kP2;
constexpr int kOffW2 = kOffW1 + kP0 * kW1Stride;
constexpr int kNetElems = kOffW2 + kP1 * kW2Stride;

enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2, PREC_BF16X3 = 3 };
inline int prec_parts(int prec) { return prec == PREC_BF16X3 ? 2 : 1; }

// BF16 net block, in 16-bit units: the float part (W0, b0, b1, b2 at the float offsets
// kOffW0 .. kOffB2 above, 256 floats), then the MFMA A operands pre-packed per lane
// (8 bf16 = 16 bytes per lane and tile): forward W1 (4 output tiles x 1 k chunk of 32)
// and W2 (8 x 2), one copy per part (hi, and lo for the split mode), then the adjoint
// W1 (2 x 2) and W2 (4 x 4), one copy per part.
constexpr int kBFloat = 256;                       // floats in the float part
constexpr int kBW1F = 4 * 1 * 512, kBW2F = 8 * 2 * 512;
constexpr int kBW1B = 2 * 2 * 512, kBW2B = 4 * 4 * 512;
constexpr int kBFwd = kBW1F + kBW2F, kBBwd = kBW1B + kBW2B;
inline constexpr int bnet_u16(int parts) { return 2 * kBFloat + parts * (kBFwd + kBBwd); }

// Student block (1 -> H <= 32 tanh -> M <= 128 affine), zero-padded: W1, b1 at hidden
// units 0..31, b2 [128], W2 [32][128] by (hidden unit, output feature) and its
// transpose W2T [128][32].
constexpr int kSW1 = 0, kSB1 = kP0, kSB2 = 2 * kP0, kSW2 = 2 * kP0 + kP2, kSW2T = kSW2 + kP0 * kP2;
constexpr int kStuElems = kSW2T + kP2 * kP0;

struct EmbedArgs {
  int prec;
  int nrows;           // padded species-grouped rows
  int n;               // local atoms
  ModelC m;
  const void* nets;    // [ntypes*ntypes] net blocks in the precision's storage layout
                       // (kNetElems T for FP64 / FP32, bnet_u16(parts) 16-bit units for BF16)
  const double* xe;
  const int* nlist;
  const int* nnei;
  const int* row_atom;
  const int* type_row0;
  const int* eown;
  void* T;             // [nrows][M][4] (double for FP64, float otherwise)
  const void* gT;      // backward: dE/dT, same layout
  double* forces;      // backward: [n][3] accumulated with atomics
  double* gbuf;        // deterministic mode (else NULL): g_ij per list slot [n][N_m][3]
  double* vir_part;    // backward: per-centre virial [nrows][9]
  const int* frame_of;
  int nframes;
  // student inference
  const void* snets;         // [ntypes*ntypes] student blocks (storage type)
  double st_lo[kMaxTypes * kMaxTypes], st_hi[kMaxTypes * kMaxTypes];
  int2* fb_list;             // fallback rows (species row, extended neighbour index)
  int* fb_count;
  int fb_cap;
  int* fb_note;              // if set, the forward fallback kernel stores the row count here
  const double* theta;       // flat FP64 parameters (fallback rows use the full net)
  const int64_t* net_off;    // [ntypes*ntypes][6] offsets of W0, b0, W1, b1, W2, b2
  const int* etype;
};
void launch_embed_fwd(const EmbedArgs& a, hipStream_t st);
void launch_student_fwd(const EmbedArgs& a, hipStream_t st);
void launch_student_bwd(const EmbedArgs& a, hipStream_t st);
void launch_fallback_fwd(const EmbedArgs& a, hipStream_t st);
void launch_fallback_bwd(const EmbedArgs& a, hipStream_t st);
void launch_embed_bwd(const EmbedArgs& a, hipStream_t st);
int embed_bwd_blocks(int nrows);

void launch_scan_int(int n, const int* in, int* out, int* sums, int* total, hipStream_t st);
// deterministic force gather: F_j -= sum of g over the list slots whose neighbour is an
// image of j, in slot order.  scratch: rev_scratch_ints(n, N_m) ints
size_t rev_scratch_ints(int n, int nm);
void launch_rev_gather(int n, int nm, const int* nlist, const int* eown, const double* gbuf, double* forces,
                       int* scratch, int* scan_sums, int* scan_total, int* status, hipStream_t st);

// ---------------------------------------------------------------- fitting net
struct FitArgs {
  int prec;
  int nrows, n;
  ModelC m;
  int nfit;            // hidden layers
  int fw;              // hidden width (square layers after the first)
  const int* type_row0;
  const int* row_atom;
  const void* T;       // [nrows][M][4]
  void* gT;            // out: dE/dT [nrows][M][4]
  // per species weights in storage type (double for FP64, float otherwise):
  // W1 [M*m2][fw], b1, W2.., wo [fw], bo [1]
  const void* const* W;  // [ntypes][nfit] device pointers (row major [in][out])
  const void* const* b;  // [ntypes][nfit]
  const void* const* wo; // [ntypes]
  // BF16 modes: GEMM operands per species and layer, [(species * nfit + k) * 4 + dir * 2 + part]
  // with dir 0 = W^T [out][in] (forward), dir 1 = W [in][out] (adjoint), part 0 hi, 1 lo
  const void* const* Wb;
  // BF16 modes: the same weights as MFMA operand fragments, [(species * nfit + k) * 2 + dir]
  // (dir 0 forward, 1 adjoint), used by the 64-row-tile kernels when fit_bf_supported()
  const void* const* Wf;
  const double* bo;      // [ntypes] device
  void *D, *Dg;        // [nrows][M*m2]
  void* act;           // [nfit][nrows][fw]  tanh outputs
  void* xs;            // [nfit][nrows][fw]  layer outputs
  void *g0, *g1;       // [nrows][fw] gradient ping-pong
  double* Ei;          // [nrows]
};
void launch_fit(const FitArgs& a, hipStream_t st);
bool fit_bf_supported(int M, int m2, int N);
void launch_fit_bf(const FitArgs& a, hipStream_t st);

// ---------------------------------------------------------------- reductions, MD
void launch_zero(double* p, size_t n, hipStream_t st);
// part: frame_reduce_chunks(max atoms of a frame) * nframes * 10 doubles of scratch
int frame_reduce_chunks(int max_frame_atoms);
void launch_frame_reduce(int nframes, int max_frame_atoms, const Frame* frames, const int* row_of,
                         const double* Ei, const double* vir_rows, double* energies, double* virials,
                         double* atom_energy, double* part, hipStream_t st);
void launch_export_T(int prec, int n, int M, const int* row_of, const void* Tm, const void* gT,
                     double* To, double* gTo, hipStream_t st);
// per-atom virial [n][9] of the centres from the per-centre rows
void launch_export_atom_virial(int n, const int* row_of, const double* vir_rows, double* out, hipStream_t st);

// ---------------------------------------------------------------- parameter gradient
struct PGradArgs {
  ModelC m;
  int nrows, np, fw, nfit;
  const double* theta;       // flat FP64 parameters (model-file order)
  double* gtheta_tan;        // tangent part of the parameter adjoint (accumulated)
  const int* row_atom;
  const int* nnei;
  const int* nlist;
  const int* eown;
  const double* xe;
  const double* vdir;        // gF [n][3]: tangent direction of the coordinates
  const double* gE;          // [nframes]
  const int* frame_of;
  const int* base[kMaxTypes];  // per neighbour species: exclusive scan over rows [nrows+1]
  int boff[kMaxTypes];         // first pair row of each neighbour-species block
  int group[2 * kMaxTypes * kMaxTypes];  // (first pair row, count) per species pair
  int type_row0_h[kMaxTypes + 1];
  const int64_t *eW, *eB, *fW, *fB;      // parameter offsets (host)
  const double* nets;                    // FP64 position-packed embedding nets (device)
  const int* type_row0;                  // species row groups (device)
  void* scratch;
  size_t scratch_bytes;
};
// fused embedding passes of the parameter gradient (pgrad_fused.hip): one wave per centre
struct PgfArgs {
  ModelC m;
  int nrows;
  const int* type_row0;
  const int* row_atom;
  const int* nnei;
  const int* nlist;
  const int* eown;
  const double* xe;
  const double* vdir;          // tangent direction of the coordinates [n][3]
  const double* nets;          // FP64 position-packed nets [ntypes^2][kNetElems]
  double *Tm, *Tmd;            // pass 1 out: T and its tangent [nrows][M][4]
  const double *gTm, *gTmd;    // pass 2 in: dE/dT and its tangent [nrows][M][4]
  const int* base[kMaxTypes];  // per neighbour species: exclusive scan of the rows' counts
  int boff[kMaxTypes];         // first pair index of each neighbour-species block
  // pass 2 out, per pair (feature order): layer inputs and pre-activation adjoints with tangents
  double *X0, *X0d, *X1, *X1d, *P0, *P0d, *P1, *P1d, *P2, *P2d, *S, *Sd;
};
void launch_pgf_fwd(const PgfArgs& a, hipStream_t st);
void launch_pgf_bwd(const PgfArgs& a, hipStream_t st);
size_t param_grad_scratch_bytes(int nrows, long np_max, int M, int m2, int s0, int fw, int nfit);
int launch_param_grad(const PGradArgs& a, hipStream_t st);
void launch_pair_scan(int nrows, int ntypes, int beta, const int* row_atom, const int* nnei, int* base,
                      int* sums, int* total, hipStream_t st);
void launch_scatter_params(int prec, size_t n, const int* map, const double* theta, void* dst, hipStream_t st);
// 16-bit-unit map: code = 4 idx + kind (0 bf16 hi, 1 bf16 lo, 2 float over two units),
// -1 zero, -2 second unit of a float
void launch_pack_bf16(size_t n, const int* map, const double* theta, uint16_t* dst, hipStream_t st);
void launch_axpy(size_t n, double a, const double* x, double* y, hipStream_t st);
void launch_zero_int(int* p, int n, hipStream_t st);
void launch_fill_int(int* p, int n, int v, hipStream_t st);

// ---------------------------------------------------------------- student net
void launch_student_gather(int n, const ModelC& m, int alpha, int beta, const int* types, const int* nnei,
                           const int* nlist, const double* xe, const float* u, float keep, int* flag,
                           int* pos, int* sums, int* total, long cap, double* out, hipStream_t st);
void launch_full_eval(long n, int s0, const double* th_net[6], const double* s, double* G, hipStream_t st);
size_t student_scratch_bytes(long n, int H, int M);
void launch_student_loss_grad(long n, int H, int M, const double* s, const double* G, const double* th,
                              double* loss, double* grad, void* scratch, hipStream_t st);
size_t student_lsq_scratch_bytes(long n, int H, int M);
void launch_student_lsq(long n, int H, int M, const double* s, const double* G, double* th, double ridge,
                        void* scratch, hipStream_t st);
void launch_adam(size_t n, double* th, double* m, double* v, const double* g, double lr, double b1, double b2,
                 double eps, int t, hipStream_t st);
size_t scan_sums_ints(int n, int W);

// C ABI helpers shared by the entry-point files (dp_api.cpp, noalloc.hip)
int handle_device(dp_handle_s* h);
int set_error(dp_handle_s* h, int code, const std::string& msg);
// workspace bytes of a one-frame force evaluation (dp_compute)
int compute_ws_bytes(dp_handle_s* h, int64_t natoms, const double* box, size_t* bytes);
// records the device address of the no-allocation scratch array of the current device
int noalloc_setup(int device);

struct MDMass {
  double m[kMaxTypes];
  double inv[kMaxTypes];
};
// neighbour-skin check fused into a drift (gate == NULL: none): *gate |= 1 when some
// atom moved more than sqrt(lim2) from xref; the cell counters c1[nc1], c2[nc2] are cleared
struct VvCheck {
  const double* xref;
  double lim2;
  int* gate;
  int nc1;
  int* c1;
  int nc2;
  int* c2;
};
// Isobaric MD (isotropic Martyna-Tobias-Klein barostat, optional Nose-Hoover thermostat
// on the particles): constants of a run and the device state (doubles, in the workspace)
struct NptConst {
  double alpha;         // 1 + 3 / N_f
  double nf, kT;        // N_f = 3N - 3, k_B T (eV)
  double W, Q;          // barostat and thermostat masses (eV fs^2)
  double pext;          // P_ext (eV / A^3)
  double h, dt;         // dt / 2, dt (fs)
  double rl, rc;        // list radius rc + skin at a build, cutoff
  double min_scale;     // smallest linear box scale the workspace plan covers
  int thermostat;       // 0: isoenthalpic
  double B0[9], Bi0[9], V0;   // initial box, its inverse and volume
};
enum {
  NS_PEPS = 0, NS_XI, NS_PXI,   // barostat momentum (eV fs), thermostat position and momentum
  NS_LAM, NS_LAMB,              // box scale vs the initial box; scale at the last list build
  NS_KE,                        // kinetic energy of v times NS_CPEND^2 (eV)
  NS_CPEND,                     // thermostat scale not yet applied to v
  NS_A1O, NS_A1, NS_B1,         // velocity factors: opening (with the pending scale), plain, force term
  NS_SX, NS_B2,                 // position factors of the drift
  NS_MU, NS_LIM2,               // scale since the last build, squared displacement limit of the skin check
  NS_V,                         // volume (A^3)
  NS_COUNT = 16
};
void launch_npt_init(int n, const int* types, const MDMass& mass, const double* v, double* state, const NptConst& c,
                     hipStream_t st);
// one thread: T(dt/2), E(dt/2), the step's factors, the box update of frame 0, skin limit
void launch_npt_open(double* state, const NptConst& c, const double* W, Frame* frames, int* status, hipStream_t st);
// P(dt/2) + R(dt) with the skin check (scaled reference positions); clears F
void launch_vv_npt_open(int n, const int* types, const MDMass& mass, double* F, double* v, double* x,
                        const double* state, const VvCheck& chk, hipStream_t st);
// P(dt/2) after the force evaluation
void launch_vv_npt_close(int n, const int* types, const MDMass& mass, const double* F, double* v,
                         const double* state, hipStream_t st);
// kinetic energy, E(dt/2), T(dt/2); a thermo row [step, PE, KE, T, Etot, P(bar), V, H] if row != NULL
void launch_npt_close(int n, const int* types, const MDMass& mass, const double* v, double* state,
                      const NptConst& c, const double* E, const double* W, int step, double* row, bool kick,
                      hipStream_t st);
// applies the pending thermostat scale to v; box_out [9] and state_out [3] (p_eps, xi, p_xi) may be NULL
void launch_npt_finish(int n, double* v, const double* state, const Frame* frames, double* box_out,
                       double* state_out, hipStream_t st);

// closing half kick of a step + opening half kick and drift of the next; clears F
void launch_vv_merged(int n, const int* types, const MDMass& mass, double dt, double* F, double* v, double* x,
                      const VvCheck& chk, hipStream_t st);
void launch_vv(int n, const int* types, const MDMass& mass, double dt, const double* F, double* v,
               double* x, bool drift, const VvCheck& chk, hipStream_t st);
// part: scratch of at least thermo_parts(n) doubles (the frame reduction's, which is free by then)
int thermo_parts(int n);
void launch_thermo(int n, const int* types, const MDMass& mass, double volume, int step,
                   const double* v, const double* E, const double* W, double* row, double* part, hipStream_t st);

}  // namespace dp
