/*
 * dp.h - C ABI of the MI355X (gfx950) Deep Potential smooth-edition library (libdp.so).
 *
 * The library evaluates a DP-SE model (arXiv 2004.11658, Section 2) for energy,
 * forces and virial of periodic systems, entirely in hand-written HIP kernels:
 * neighbour search and formatting (Alg. 1), environment matrix (Eq. 5, Alg. 2),
 * embedding net (Eq. 6-9), descriptor (Eq. 4), fitting net (Eq. 1-3) and the adjoint
 * for forces (Eq. 10) and virial, plus velocity-Verlet MD (Section 4).
 *
 * Conventions (all calls):
 *   - Units: Angstrom, eV, fs, amu ("metal" units).
 *   - Boxes: 3x3 row-major double, rows are the cell vectors a, b, c (right handed);
 *     fractional coordinates f satisfy x = f . B (row vectors).
 *   - Device pointers are HIP device memory owned by the caller (e.g. torch tensors);
 *     host pointers are ordinary host memory.  The caller owns every device buffer:
 *     inputs, outputs, workspaces, the weight region (dp_device_bytes / dp_upload) and
 *     the student region (dp_student_bytes / dp_set_student).  The library never
 *     allocates device or pinned host memory; it owns only its handle (host metadata).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Compute calls
 *     only enqueue work on it and return after host-side validation; they never
 *     synchronise.  Conditions found on the device are written to a status word in
 *     the workspace and read back by dp_status (which synchronises the stream).
 *   - Return codes: DP_OK (0); > 0 warnings (results valid); < 0 errors (outputs
 *     undefined).  dp_last_error gives a readable reason for the last failing call.
 *   - A handle may be used from one host thread at a time.  Calls on different
 *     workspaces may run concurrently on different streams.
 */
#ifndef DP_H
#define DP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_handle_s* dp_handle;

enum {
  DP_OK = 0,
  DP_WARN_SEL_OVERFLOW = 1,  /* a neighbour-type block held more than sel atoms; the
                                nearest sel were kept (Alg. 1 padding width exceeded) */
  DP_ERR_ARG = -1,           /* null pointer, bad size or bad option */
  DP_ERR_MODEL = -2,         /* unreadable model file or unsupported architecture */
  DP_ERR_BOX = -3,           /* singular or left-handed box */
  DP_ERR_TYPE = -4,          /* atom type outside [0, ntypes) (found on the device) */
  DP_ERR_CAPACITY = -5,      /* more than DP_MAX_CANDIDATES atoms within rc of one atom,
                                or more ghost images than the workspace plan allowed */
  DP_ERR_WORKSPACE = -6,     /* workspace smaller than dp_workspace_size reported */
  DP_ERR_HIP = -7,           /* a HIP runtime call failed */
  DP_ERR_NONFINITE = -8,     /* non-finite coordinate (found on the device) */
  DP_ERR_OVERLAP = -9        /* two atoms closer than 1e-6 A (found on the device) */
};

#define DP_MAX_CANDIDATES 1024

enum { DP_PREC_FP64 = 0, DP_PREC_FP32 = 1, DP_PREC_BF16 = 2, DP_PREC_BF16X3 = 3 };

typedef struct {
  int32_t precision;  /* DP_PREC_*: operand precision of the embedding and fitting
                         GEMMs.  FP64: everything in double.  FP32 / BF16: GEMM
                         operands in that type with FP32 accumulation; BF16X3: BF16
                         operands split as hi + lo (three MFMAs per product).
                         Coordinates, distances, the environment matrix, force and
                         virial accumulation, energy sums and integration stay FP64. */
  int32_t deterministic; /* 1: forces independent of kernel scheduling (each pair force
                         is stored in its list slot and gathered per atom in slot
                         order, Remark 4's reverse sum) instead of FP64 atomics;
                         not combinable with student nets.  0: atomics. */
  double skin;        /* MD neighbour skin (A): dp_md_run rebuilds the list of pairs
                         within rc + skin only when some atom moved more than skin/2
                         (checked on the device every step) and formats it within rc
                         at every step; 0 = rebuild everything every step */
} dp_options;

/* Read a model file ("DPSEMDL1" format: architecture + FP64 parameters in the
 * documented flat order) and plan its weight layouts for the current HIP device (host
 * work only; nothing is allocated on the device).  Before any compute call the caller
 * provides the weight region with dp_device_bytes + dp_upload.
 * Supported architecture: 1..8 species, embedding nets of three layers
 * 1 -> s0 -> 2 s0 -> 4 s0 = M with s0 <= 32 (Section 2, Eq. 7-9), square hidden
 * fitting layers after the first (Eq. 3), M< <= M, N_m = sum(sel) <= 1024.
 * opt may be NULL (FP64, atomics, skin 0).  On error *out is NULL. */
int dp_init(const char* model_path, const dp_options* opt, dp_handle* out);
/* Releases the handle (host memory only; caller buffers are untouched). */
void dp_free(dp_handle h);

/* Bytes of the weight region (Section 2's network parameters in the kernels' layouts:
 * the flat FP64 parameter vector, its index maps, the precision's embedding net
 * blocks (Eq. 7-9) and fitting weights (Eq. 1-3), pointer tables).  Depends only on the
 * model and the precision option. */
int dp_device_bytes(dp_handle h, size_t* weight_bytes);
/* Binds the weight region to weights (device, >= dp_device_bytes bytes, 256-byte
 * aligned, owned by the caller and kept alive and unmodified while the handle uses it),
 * copies the model file's parameters in and builds the kernel layouts on stream.
 * Synchronises the stream.  May be called again to move the region (the model file's
 * parameters are reinstalled).  Errors: DP_ERR_ARG (NULL, misaligned),
 * DP_ERR_WORKSPACE (too small), DP_ERR_HIP. Every other device call on the handle
 * returns DP_ERR_ARG until this has succeeded. */
int dp_upload(dp_handle h, void* weights, size_t bytes, void* stream);

/* Architecture summary. Any output pointer may be NULL. */
int dp_model_info(dp_handle h, int32_t* ntypes, int32_t* nm, int32_t* M, int32_t* m2,
                  double* rc, int64_t* nparams);

/* Bytes of device workspace needed for a batch of nframes frames with the given host
 * arrays atom_offsets [nframes+1] (frame f owns atoms [atom_offsets[f], atom_offsets[f+1]))
 * and boxes [nframes][9].  The workspace carries the neighbour list, ghost images,
 * per-atom descriptors and status words; one workspace serves calls of at most that
 * size and equal or smaller ghost shells.  Every frame must hold at least one atom and
 * the batch at most 2^26 atoms: an empty frame, a decreasing atom_offsets or a larger
 * batch returns DP_ERR_ARG here and from every evaluation entry point, before anything
 * is launched (an empty frame's energy is zero by Eq. 1; the caller skips it). */
int dp_workspace_size(dp_handle h, int32_t nframes, const int64_t* atom_offsets,
                      const double* boxes, size_t* bytes);

/* Energy, forces and virial of one periodic frame (Eq. 1 and 10).
 *   coords [natoms][3] device, types [natoms] device int32 in [0, ntypes),
 *   box [9] host, energy [1] device, forces [natoms][3] device (overwritten),
 *   virial [9] device or NULL (W_ab = -sum_pairs d_a dE/dd_b),
 *   atom_energy [natoms] device or NULL (E_i). */
int dp_compute(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
               const double* box, double* energy, double* forces, double* virial,
               double* atom_energy, void* workspace, size_t ws_bytes, void* stream);

/* dp_compute for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the workspace is the
 * library's built-in scratch array of 64 MiB per device (a file-scope device array held
 * until the process ends; enough for about 1,000 water atoms in FP64).  Arguments as
 * dp_compute without workspace and ws_bytes; the weight region must be uploaded.
 * Returns DP_ERR_WORKSPACE, launching nothing, when the frame needs more workspace than
 * the array holds.  Every call on one device shares that device's array: calls that
 * overlap in time on one device (other streams or threads) race and give undefined
 * results.  The status word lives in the array, so device-detected conditions
 * (DP_ERR_TYPE, DP_ERR_NONFINITE, DP_ERR_OVERLAP, DP_ERR_CAPACITY, the sel warning) are
 * not reported: validate unfamiliar inputs with dp_compute first. */
int dp_compute_noalloc(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                       const double* box, double* energy, double* forces, double* virial,
                       double* atom_energy, void* stream);

/* dp_compute with the per-atom virial: atom_virial [natoms][9] device (row-major 3x3, or
 * NULL), W_i = -sum_j d_ij (x) dE_i/dd_ij over the neighbours j of centre i (each pair
 * term of the virial assigned to its centre; sum_i W_i = virial).  Since E_i depends only
 * on the vectors d_ij of its environment (Eq. 1-5), W_i = -dE_i/d(eps) under the strain
 * x -> x (I + eps), and W_i is symmetric.  Workspace as dp_compute. */
int dp_compute_atomic(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                      const double* box, double* energy, double* forces, double* virial, double* atom_energy,
                      double* atom_virial, void* workspace, size_t ws_bytes, void* stream);

/* Engine-facing evaluation (an MD engine's pair interface, Section 3.1's domain
 * decomposition): the caller supplies its nlocal local atoms followed by nghost ghost
 * atoms (copies of other domains' or periodic images' atoms that lie within rc of a
 * local atom), with no periodic box: coords [nlocal + nghost][3] and types device;
 * bounds (host [6]: xlo, ylo, zlo, xhi, yhi, zhi) enclose every local and ghost atom.
 * Only local atoms are centres: energy [1] = sum of E_i over local atoms, atom_energy
 * [nlocal] and atom_virial [nlocal][9] (may be NULL) per local atom, virial [9] (may be
 * NULL) the sum of the local atoms' W_i.  forces [nlocal + nghost][3] receives the forces
 * on local AND ghost atoms: the force of each pair goes to the atom the caller supplied
 * (Remark 4), so the caller adds each ghost's force to the atom it copies (reverse
 * communication) to obtain the forces of its local energy.  Not available with
 * deterministic = 1 (DP_ERR_ARG).  Workspace: dp_compute_local_workspace_size. */
int dp_compute_local_workspace_size(dp_handle h, int64_t nlocal, int64_t nghost, const double* bounds,
                                    size_t* bytes);
int dp_compute_local(dp_handle h, int64_t nlocal, int64_t nghost, const double* coords, const int32_t* types,
                     const double* bounds, double* energy, double* forces, double* virial, double* atom_energy,
                     double* atom_virial, void* workspace, size_t ws_bytes, void* stream);

/* The same for a batch of independent frames of uneven size, in one launch per kernel.
 *   atom_offsets [nframes+1] host, coords/types/forces/atom_energy concatenated over
 *   frames, boxes [nframes][9] host, energies [nframes] and virials [nframes][9] device
 *   (virials may be NULL). */
int dp_compute_batch(dp_handle h, int32_t nframes, const int64_t* atom_offsets,
                     const double* coords, const int32_t* types, const double* boxes,
                     double* energies, double* forces, double* virials, double* atom_energy,
                     void* workspace, size_t ws_bytes, void* stream);

/* Formatted neighbour list of one frame (Alg. 1): nlist [natoms][N_m] device int32,
 * type blocks of width sel in species order, each sorted by (r, owner index, image
 * code) with -1 pads; img [natoms][N_m] device int32 image codes
 * ((n0+K0)(2K1+1) + n1+K1)(2K2+1) + n2+K2 with K_k = ceil(rc / width_k); nnei
 * [natoms][ntypes] device int32 real counts. img and nnei may be NULL. */
int dp_nlist(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
             const double* box, int32_t* nlist, int32_t* img, int32_t* nnei,
             void* workspace, size_t ws_bytes, void* stream);

/* Descriptor intermediates of one frame, for parity checks: T [natoms][M][4]
 * (= G^T R / N_m, Eq. 4), and dE_i/dT [natoms][M][4], device doubles; either may
 * be NULL.  Runs the same kernels as dp_compute. */
int dp_descriptor(dp_handle h, int64_t natoms, const double* coords, const int32_t* types,
                  const double* box, double* T, double* gT, void* workspace,
                  size_t ws_bytes, void* stream);

/* Velocity-Verlet molecular dynamics of one frame (paper Section 4), nsteps steps of
 * dt_fs femtoseconds with a fresh force evaluation per step:
 *   v += dt/2 F/m;  x += dt v;  F = F(x);  v += dt/2 F/m
 * x [natoms][3] and v [natoms][3] (A/fs) are device arrays updated in place (x is not
 * wrapped into the box); masses [ntypes] host (amu).  thermo (device, may be NULL)
 * receives rows [step, E_pot, E_kin, T(K), E_tot, P(bar)] at step 0 and every
 * thermo_every steps: 1 + nsteps / thermo_every rows of 6 doubles.  forces [natoms][3]
 * (device, may be NULL) receives the forces of the final positions.  The workspace is
 * the one dp_workspace_size reports for this frame. */
int dp_md_run(dp_handle h, int64_t natoms, double* x, double* v, const int32_t* types,
              const double* masses, const double* box, double dt_fs, int32_t nsteps,
              int32_t thermo_every, double* thermo, double* forces, void* workspace,
              size_t ws_bytes, void* stream);

/* Isobaric molecular dynamics (an extension of Section 4's velocity Verlet: the
 * pressure from the virial, the thermo quantity of Section 4, drives an isotropic box
 * scaling).  Equations of motion of Martyna, Tobias and Klein with an optional
 * Nose-Hoover thermostat on the particles, N_f = 3N - 3, alpha = 1 + 3 / N_f:
 *   dx/dt = v + v_eps x,  dv/dt = F/m - alpha v_eps v - v_xi v,  dV/dt = 3 V v_eps,
 *   dp_eps/dt = alpha 2 KE + tr W - 3 V P_ext,  dp_xi/dt = 2 KE - N_f k_B T
 * with v_eps = p_eps / W_b, W_b = (N_f + 3) k_B T tau_p^2, v_xi = p_xi / Q,
 * Q = N_f k_B T tau_t^2, integrated by the symmetric splitting
 * T(dt/2) E(dt/2) P(dt/2) R(dt) [forces] P(dt/2) E(dt/2) T(dt/2) (each part exact),
 * which conserves H = E_pot + KE + p_eps^2/(2 W_b) + P_ext V (+ p_xi^2/(2Q) + N_f k_B T xi)
 * to O(dt^2).  Any right-handed box (triclinic included) keeps its shape. */
typedef struct {
  double pressure_bar;   /* P_ext (bar) */
  double tau_p_fs;       /* barostat time scale (> 0) */
  double temperature_K;  /* T of the thermostat and of the barostat mass (> 0) */
  double tau_t_fs;       /* thermostat time scale; 0: no thermostat (isoenthalpic) */
  double min_scale;      /* smallest linear box scale, relative to the initial box, that
                            the workspace plan covers, in (0.5, 1]; a run that compresses
                            further reports DP_ERR_CAPACITY through dp_status */
} dp_npt_options;

/* Workspace bytes of dp_md_run_npt for one frame of natoms atoms in box (host [9]). */
int dp_md_npt_workspace_size(dp_handle h, int64_t natoms, const double* box, double min_scale, size_t* bytes);

/* nsteps isobaric MD steps of dt_fs on one frame; needs a handle with skin > 0 (the list
 * of pairs within rc + skin is rebuilt when some atom's displacement beyond the affine
 * box scaling exceeds (mu (rc + skin) - rc) / 2, mu = box scale relative to the last
 * build).  x, v device [natoms][3] updated in place (x not wrapped); box host [9] is the
 * initial box and is not modified; thermo (device, may be NULL) receives rows of 8
 * [step, E_pot, E_kin, T(K), E_pot + E_kin, P(bar), V(A^3), H(eV)] at step 0 and every
 * thermo_every steps; box_out (device [9], may be NULL) the final box; state_out (device
 * [3], may be NULL) p_eps (eV fs), xi, p_xi (eV fs) at the end; forces (device
 * [natoms][3], may be NULL) the final forces.  The run starts with p_eps = xi = p_xi = 0.
 * Errors as dp_md_run; DP_ERR_ARG for bad options or a handle without a skin. */
int dp_md_run_npt(dp_handle h, int64_t natoms, double* x, double* v, const int32_t* types, const double* masses,
                  const double* box, const dp_npt_options* npt, double dt_fs, int32_t nsteps,
                  int32_t thermo_every, double* thermo, double* box_out, double* state_out, double* forces,
                  void* workspace, size_t ws_bytes, void* stream);

/* Replace the model parameters by theta (device, FP64, nparams values in the model
 * file's flat order) and rebuild the kernels' weight layouts on stream.  Later calls
 * on the handle use the new parameters.  dp_get_params copies the current ones out. */
int dp_set_params(dp_handle h, const double* theta, void* stream);
int dp_get_params(dp_handle h, double* theta, void* stream);

/* Parameter gradient of an energy + force loss for a batch of frames (training):
 *   gtheta += sum_f gE[f] dE_f/dtheta + sum_i gF[i] . dF_i/dtheta      (F = -dE/dr, Eq. 10)
 * with gE [nframes] and gF [natoms][3] device doubles (the loss gradients with respect
 * to the energies and forces) and gtheta [nparams] device doubles (accumulated: zero
 * it first).  Computed exactly (forward-over-reverse, FP64, any precision option).
 * Batch arguments as dp_compute_batch.  The library runs the batch in chunks of whole
 * frames of at most max_atoms atoms together (0: 32768; a larger frame is a chunk of its
 * own), so the workspace, dp_param_grad_workspace_size bytes for the same max_atoms,
 * is that of the largest chunk (roughly 8 KB per neighbour pair of it), whatever the
 * batch size.  Synchronises the stream once per chunk. */
int dp_param_grad_workspace_size(dp_handle h, int32_t nframes, const int64_t* atom_offsets,
                                 const double* boxes, int64_t max_atoms, size_t* bytes);
int dp_param_grad(dp_handle h, int32_t nframes, const int64_t* atom_offsets, const double* coords,
                  const int32_t* types, const double* boxes, const double* gE, const double* gF,
                  double* gtheta, int64_t max_atoms, void* workspace, size_t ws_bytes, void* stream);

/* ---- student embedding net (a narrower G_s(s) = tanh(s W1 + b1) W2 + b2, 1 -> H -> M,
 * trained to reproduce the full embedding net on the s range the model visits) ---- */

/* s values of the real neighbours of species beta around centres of species alpha in
 * one frame, each kept when its uniform number (uniforms [natoms][N_m] device floats,
 * one per neighbour slot) is below keep_prob, written to s_out [cap] (device) in slot
 * order.  *count (host) receives the number kept (may exceed cap: the rest are
 * dropped).  Synchronises the stream.  The workspace must hold
 * dp_student_samples_workspace_size bytes. */
int dp_student_samples_workspace_size(dp_handle h, int64_t natoms, const double* box, size_t* bytes);
int dp_student_samples(dp_handle h, int32_t alpha, int32_t beta, int64_t natoms, const double* coords,
                       const int32_t* types, const double* box, const float* uniforms, double keep_prob,
                       double* s_out, int64_t cap, int64_t* count, void* workspace, size_t ws_bytes,
                       void* stream);

/* The full embedding net G^{alpha,beta} (Eq. 7-9) at n given s (device), in FP64 with the
 * current parameters: G [n][M] device. */
int dp_embed_eval(dp_handle h, int32_t alpha, int32_t beta, int64_t n, const double* s, double* G,
                  void* stream);

/* Student MSE loss L = mean over samples and outputs of (G_s(s) - G)^2 and its gradient:
 * theta_s [2H + H M + M] device (W1 [H], b1 [H], W2 [H][M] row major, b2 [M]),
 * s [n], G [n][M] device; loss [1] device is ADDED to; grad device is overwritten.
 * scratch: dp_student_scratch_size bytes of device memory. */
int dp_student_scratch_size(int32_t hidden, int32_t M, int64_t n, size_t* bytes);
int dp_student_loss_grad(int32_t hidden, int32_t M, int64_t n, const double* s, const double* G,
                         const double* theta_s, double* loss, double* grad, void* scratch,
                         size_t scratch_bytes, void* stream);

/* Least-squares output layer of a student: with W1, b1 of theta_s fixed, sets W2, b2 to
 * the minimiser of sum (G_s(s) - G)^2 by the normal equations with a ridge of
 * ridge * max diag (Cholesky on the device); hidden <= 32.  scratch:
 * dp_student_lsq_scratch_size bytes of device memory. */
int dp_student_lsq_scratch_size(int32_t hidden, int32_t M, int64_t n, size_t* bytes);
int dp_student_lsq(int32_t hidden, int32_t M, int64_t n, const double* s, const double* G, double* theta_s,
                   double ridge, void* scratch, size_t scratch_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) on n device doubles: theta, moments m, v. */
int dp_adam(int64_t n, double* theta, double* m, double* v, const double* g, int32_t step, double lr,
            double beta1, double beta2, double eps, void* stream);

/* Bytes of the student region for dp_set_student (index map + ntypes^2 padded student
 * blocks in the precision's storage type). */
int dp_student_bytes(dp_handle h, size_t* bytes);

/* Install (enable = 1) or remove (enable = 0) student embedding nets for inference.
 * theta_s (device, FP64): ntypes^2 consecutive student parameter blocks, species pair
 * (alpha, beta) at index alpha * ntypes + beta, each laid out as for
 * dp_student_loss_grad with hidden width 1..32.  s_lo, s_hi (host [ntypes^2], finite,
 * s_lo <= s_hi): the s range each student was trained on.  student_mem (device,
 * >= dp_student_bytes bytes, 256-byte aligned, caller-owned, kept alive while enabled)
 * receives the student layouts.  While enabled, every compute, MD and descriptor
 * call uses the student for neighbours with s in [s_lo, s_hi] and the full net (FP64)
 * for the others.  Workspaces must be sized after this call.  Synchronises the stream.
 * DP_ERR_ARG on a handle made with deterministic = 1 or bad ranges; DP_ERR_WORKSPACE if
 * student_bytes is too small.  With enable = 0 the other arguments are ignored. */
int dp_set_student(dp_handle h, int32_t hidden, const double* theta_s, const double* s_lo,
                   const double* s_hi, int32_t enable, void* student_mem, size_t student_bytes,
                   void* stream);

/* Stage timing with HIP events recorded on the call's stream around each stage
 * (neighbour list, embedding forward, fitting net, embedding adjoint, reductions,
 * integration, and with student nets the full-net fallback rows of both passes;
 * each of EMBED_FWD and EMBED_BWD is then one kernel launch).  dp_profile(h, 1) clears the records and enables timing,
 * dp_profile(h, 0) stops recording and keeps the records for dp_profile_read.
 * dp_profile_read synchronises the events and returns the summed milliseconds and the
 * number of launches of one stage (DP_STAGE_*). */
enum { DP_STAGE_NLIST = 0, DP_STAGE_EMBED_FWD = 1, DP_STAGE_FIT = 2, DP_STAGE_EMBED_BWD = 3,
       DP_STAGE_REDUCE = 4, DP_STAGE_MD = 5, DP_STAGE_FALLBACK = 6, DP_NSTAGES = 7 };
int dp_profile(dp_handle h, int32_t enable);
int dp_profile_read(dp_handle h, int32_t stage, double* total_ms, int64_t* launches);
/* As dp_profile(h, 1), but timing only the stages whose bit (1 << DP_STAGE_*) is set in
 * stage_mask (0: stop recording).  Each timed stage adds two event records per call to
 * the stream, so timing one stage perturbs a run less than timing all of them. */
int dp_profile_stages(dp_handle h, uint32_t stage_mask);

/* Synchronise stream and read the status word of the last call that used workspace.
 * flags (may be NULL) receives the raw flag bits; detail (may be NULL) the count
 * attached to the first condition.  Returns DP_OK, DP_WARN_SEL_OVERFLOW or a
 * negative DP_ERR_* for device-detected conditions. */
int dp_status(dp_handle h, const void* workspace, void* stream, int32_t* flags,
              int64_t* detail);

/* Synchronise stream and read how many neighbour rows the last force evaluation that
 * used workspace handed from the student nets to the full net (their s lay outside the
 * students' trained ranges; the fallback of the student embedding).  0 without
 * students.  Returns DP_OK or DP_ERR_ARG (NULL argument). */
int dp_fallback_rows(dp_handle h, const void* workspace, void* stream, int64_t* rows);

const char* dp_strerror(int code);
const char* dp_last_error(dp_handle h);

#ifdef __cplusplus
}
#endif
#endif
