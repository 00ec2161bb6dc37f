/*
 * mdpl: short-range molecular-dynamics pair loops on AMD Instinct MI355X
 * (gfx950), behind a plain C ABI.
 *
 * The operations follow the problem statement of Saunders, Grant & Mueller,
 * "A Domain Specific Language for Performance Portable Molecular Dynamics
 * Algorithms" (arXiv:1704.03329): N particles with positions, velocities
 * and mass in a periodic box (Sec. 3.5), a cutoff r_c and an extra shell
 * delta for neighbour-list reuse (Eq. extended_cutoff), the Lennard-Jones
 * pair loop (Eqs. LJpotential, LJforce), the velocity-Verlet particle loops
 * (Alg. VelocityVerlet), the bond-order analysis (Sec. 4.1) and the
 * common-neighbour analysis (Sec. 4.2).
 *
 * Conventions (all entry points):
 *  - Every pointer argument is a DEVICE pointer unless its name ends in
 *    _host.  Arrays are structure-of-arrays, contiguous, length n (the
 *    caller's particle count, no padding).  Forces are float or double
 *    according to mdpl_lj_params.precision.
 *  - The caller owns every array and the workspace; the library allocates no
 *    device memory.  Pointers must stay valid until the stream reaches the
 *    enqueued work.
 *  - Work is enqueued on the hipStream_t given at creation (or per call for
 *    the analysis entry points) and the call returns at once.  Only
 *    mdpl_check, mdpl_nlist_export and mdpl_kernel_time synchronise.
 *  - Errors are returned as mdpl_status codes, never thrown.  Argument
 *    errors are detected on the host before any device work is enqueued.
 *    Errors found by kernels (capacity, skin, non-finite) raise flag bits
 *    that mdpl_check reports.
 *  - One mdpl_sim must not be used from two host threads at once.
 */
#ifndef MDPL_H
#define MDPL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mdpl_status;
#define MDPL_OK 0
#define MDPL_EINVAL 1     /* null pointer, n <= 0, box <= 0, rc <= 0, skin < 0, dt <= 0, ... */
#define MDPL_EBOX 2       /* fewer than 3 cells of side >= rc+skin along some axis */
#define MDPL_ECAPACITY 3  /* a neighbour list had more entries than max_nb */
#define MDPL_ESKIN 4      /* a particle moved >= skin/2 between two list builds */
#define MDPL_ENONFINITE 5 /* a non-finite velocity appeared */
#define MDPL_EHIP 6       /* a HIP runtime call failed; see mdpl_last_hip_error */
#define MDPL_ESTATE 7     /* call out of order (e.g. forces before a build) */
#define MDPL_EWORKSPACE 8 /* workspace too small or misaligned (256 B) */
#define MDPL_ESCRATCH 9   /* input larger than the library's static scratch (mdpl_boa_noalloc) */

/* Flag bits reported by mdpl_check. */
#define MDPL_FLAG_NL_OVERFLOW 1u
#define MDPL_FLAG_SKIN 2u
#define MDPL_FLAG_NONFINITE 4u

/* Energy shift of the Lennard-Jones potential.
 * NONE:   V = 4 eps [(s/r)^12 - (s/r)^6]            (V(2^(1/6) s) = -eps)
 * PAPER:  V + eps, the form printed in Eq. LJpotential (with its +1/4)
 * CUTOFF: V - V(rc), continuous at the cutoff
 * Forces are identical in all modes. */
#define MDPL_SHIFT_NONE 0
#define MDPL_SHIFT_PAPER 1
#define MDPL_SHIFT_CUTOFF 2

/* Force precision.  FP64: every pair computed and accumulated in double,
 * forces stored as double.  FP32: separations and the cutoff test in double,
 * pair force in float, per-atom float sum, forces stored as float; energies
 * and the virial are always double. */
#define MDPL_FP64 0
#define MDPL_FP32 1

/* How the pair loop finds the pairs within rc.
 * FULL:  a neighbour list of every ordered pair within rc+skin, rebuilt
 *        every reuse_every steps (Sec. 3.5); the pass writes only to the
 *        first particle of a pair (Sec. 2), so no atomics and bit-reproducible
 *        forces.
 * HALF:  each pair listed once and its reaction applied to the second
 *        particle (Newton's third law; Sec. 2, the comment on it beside the
 *        pair loop); reactions are summed with atomics, so the last bits of
 *        the forces vary from run to run.
 * CELLS: no neighbour list: every force pass scans the 27-cell stencil of
 *        the cell list built every reuse_every steps (cells of side >=
 *        rc+skin, Sec. 3.5); bit-reproducible like FULL.
 * The learned-potential entry points need FULL (MDPL_EINVAL otherwise);
 * mdpl_nlist_export and mdpl_nlist_entries need a list (MDPL_ESTATE with
 * CELLS). */
#define MDPL_PAIRS_FULL 0
#define MDPL_PAIRS_HALF 1
#define MDPL_PAIRS_CELLS 2

/* When the runs rebuild the cell and neighbour lists (Sec. 3.5, Eq.
 * extended_cutoff and the IntegratorRange paragraph, which takes the time
 * step, the velocities, a largest reuse count and the shell thickness).
 * FIXED: every reuse_every steps.
 * VMAX:  every reuse_every steps, and also as soon as
 *        2 * sum over the steps since the last build of dt * max_i |v_i| >= skin,
 *        the condition of Eq. extended_cutoff under which no pair inside rc
 *        can be missing from the list.  The largest speed of every step is
 *        found on the device by the kernel that moves the particles; the host
 *        waits for the stream only when a prediction from the speeds it has
 *        already seen (allowed to double) says the threshold may be reached,
 *        and then decides on the exact value.  Each context holds
 *        64 x 32 bytes of pinned host memory for these records.
 * In both modes every rebuild checks the displacement of the last positions
 * used with the old list against skin/2 (MDPL_FLAG_SKIN). */
#define MDPL_REBUILD_FIXED 0
#define MDPL_REBUILD_VMAX 1

/* How a run starts.
 * SETUP:    bin the particles, build the list and compute F(r0) (and the
 *           energy of step 0 if sampled).
 * CONTINUE: take over the state that the last run of the same force field
 *           (LJ, with or without thermostat, or learned) on this context left
 *           in the SAME arrays: its list, its forces (no F(r0) pass) and its
 *           count of steps since the last build (the rebuild schedule goes
 *           on).  The caller must not have changed positions, forces or ids
 *           since; velocities may have been changed (e.g. rescaled).  With
 *           unchanged velocities the result is bit-identical to one longer
 *           run.  MDPL_ESTATE if there is no such state (other arrays,
 *           another force field, an mdpl_build since). */
#define MDPL_RUN_SETUP 0
#define MDPL_RUN_CONTINUE 1

typedef struct {
  int64_t n;          /* number of particles, 1 .. 2^26 */
  double box[3];      /* periodic box [0,Lx) x [0,Ly) x [0,Lz) */
  double rc;          /* interaction cutoff r_c (> 0) */
  double skin;        /* extra shell delta = rbar_c - r_c (>= 0), Eq. extended_cutoff */
  double eps, sigma;  /* Lennard-Jones parameters (> 0) */
  double mass;        /* particle mass (> 0) */
  double dt;          /* time step (> 0) */
  int32_t reuse_every;/* rebuild the cell and neighbour lists every this many steps (>= 1) */
  int32_t shift;      /* MDPL_SHIFT_* */
  int32_t precision;  /* MDPL_FP64 or MDPL_FP32 */
  int32_t max_nb;     /* neighbour-list capacity per particle (1 .. 1024) */
  int32_t pairs;      /* MDPL_PAIRS_*: how the pair loop finds the pairs within rc */
  int32_t rebuild;    /* MDPL_REBUILD_*: when the runs rebuild the lists */
} mdpl_lj_params;

typedef struct mdpl_sim mdpl_sim;

/* Human-readable name of a status code (static string). */
const char* mdpl_status_string(mdpl_status s);

/* Last hipError_t seen by any entry point of this process (0 if none). */
int32_t mdpl_last_hip_error(void);

/* ------------------------------------------------------------------ LJ state
 * Bytes of device workspace needed for these parameters (cell list, sorted
 * copies, neighbour list, reduction partials, flags).  Host only. */
mdpl_status mdpl_workspace_bytes(const mdpl_lj_params* p, size_t* bytes_host);

/* Create a simulation context on `workspace` (device, >= mdpl_workspace_bytes,
 * 256-byte aligned).  `stream` is a hipStream_t (NULL = default stream).
 * Validates p (MDPL_EINVAL / MDPL_EBOX); enqueues the clearing of the flags. */
mdpl_status mdpl_sim_create(const mdpl_lj_params* p, void* workspace, size_t workspace_bytes,
                            void* stream, mdpl_sim** out_host);

/* Release the host-side context (the workspace stays the caller's). */
mdpl_status mdpl_sim_destroy(mdpl_sim* sim);

/* Cell binning and neighbour-list construction for the given positions
 * (Sec. 3.5: cells of side >= rc+skin, 27-cell stencil, list of every j != i
 * with |r_i - r_j| < rc+skin under the minimum image; with MDPL_PAIRS_HALF
 * each pair once, with MDPL_PAIRS_CELLS the binning only).  Positions are first
 * folded into the box, x - L floor(x / L) (then x - L if that rounds to L),
 * and the list is that of the folded positions, tested exactly as
 * (dx*dx + dy*dy) + dz*dz < (rc+skin)^2 in double with the conditional
 * minimum image dx -/+ L.  Particles are counting-sorted by cell into
 * workspace copies (with full lists, each cell's particles in the lower half
 * of the cell along x first); the caller's arrays are not modified. */
mdpl_status mdpl_build(mdpl_sim* sim, const double* x, const double* y, const double* z);

/* Copy the list of the last mdpl_build as directed pairs (i, j) in the
 * caller's particle indices, unordered (with MDPL_PAIRS_HALF each pair
 * appears once, in one direction).  Writes min(count, cap) pairs,
 * returns the total in *count_host.  Synchronises the stream. */
mdpl_status mdpl_nlist_export(mdpl_sim* sim, int32_t* i_out, int32_t* j_out, int64_t cap,
                              int64_t* count_host);

/* Lennard-Jones forces (Eq. LJforce, F_i = sum_j f(r_i, r_j), INC_ZERO)
 * for positions x,y,z (caller order) using the list of the last mdpl_build;
 * the positions may have moved by less than skin/2 since then.
 * fx,fy,fz: float* or double* per precision, caller order, overwritten.
 * pe_w: nullable, 2 doubles receiving the potential energy sum_{i<j} V and
 * the virial sum_{i<j} r_ij . f_ij.  e_atom: nullable, n doubles receiving
 * 1/2 sum_j V(r_ij). */
mdpl_status mdpl_forces(mdpl_sim* sim, const double* x, const double* y, const double* z,
                        void* fx, void* fy, void* fz, double* pe_w, double* e_atom);

/* Reverse-mode derivative of the potential energy E(x) = sum_{i<j} V:
 * g_i = grad_e[0] * dE/dr_i = -grad_e[0] * F_i, in double, caller order,
 * using the list of the last mdpl_build.  grad_e: 1 double (device). */
mdpl_status mdpl_lj_backward(mdpl_sim* sim, const double* x, const double* y, const double* z,
                             const double* grad_e, double* gx, double* gy, double* gz);

/* Integrate nsteps of velocity Verlet (Alg. VelocityVerlet): F(r0) first,
 * then per step v += dt/(2m) F; r += dt v; F = forces(r); v += dt/(2m) F.
 * The cell and neighbour lists are rebuilt at the start (start =
 * MDPL_RUN_SETUP) and then as mdpl_lj_params.rebuild says; with
 * MDPL_RUN_CONTINUE the run goes on from the previous run's state (see
 * MDPL_RUN_CONTINUE; row 0 of thermo is then that state's, taken from the
 * previous run's last row when it sampled its last step).  At every rebuild
 * the particles are reordered by cell IN PLACE in all ten arrays (positions folded into [0, L)), so that
 * ids[k] always holds the original id of the particle in slot k.
 * thermo: nullable; if sample_every > 0 it receives
 * (nsteps / sample_every + 1) rows of 4 doubles: KE, PE, virial, and the
 * largest displacement of any particle from its position at the list build,
 * over the reuse periods completed so far; rows are taken at step 0 and
 * every sample_every steps (KE after the second half kick).  On sampled
 * steps the force pass also forms PE and the virial in FP64.  If the last
 * positions used with a list had moved skin/2 or more from those of its
 * build (a pair inside rc could then be missing from the list),
 * MDPL_FLAG_SKIN is raised; see mdpl_check.  The MDPL_REBUILD_VMAX rule
 * rebuilds before that can happen (Eq. extended_cutoff). */
mdpl_status mdpl_run(mdpl_sim* sim, double* x, double* y, double* z, double* vx, double* vy,
                     double* vz, void* fx, void* fy, void* fz, int32_t* ids, int64_t nsteps,
                     int32_t sample_every, double* thermo, int32_t start);

/* mdpl_run with the Andersen thermostat of the crystallisation run (Sec.
 * 5.2; the paper gives neither the collision rule nor the random numbers,
 * so these are readings): after the kick that completes step g (after its
 * thermo sample), each particle collides with probability p =
 * collision_rate * dt (must be <= 1) and takes a velocity with components
 * sqrt(temperature / mass) * N(0, 1).  The draws come from Philox4x64-10
 * (Salmon et al., SC'11) with key (seed, 0) and counter (g, id, block, 0),
 * id = the particle's value in `ids` at the call (its original id), so they
 * do not depend on the in-place reordering: with block 0 = (b0..b3) and
 * block 1 = (b4, ...), U(b) = (b >> 11) 2^-53, the particle collides iff
 * U(b0) < p and then takes sqrt(-2 ln(1 - U(b1))) (cos, sin)(2 pi U(b2)) and
 * sqrt(-2 ln(1 - U(b3))) cos(2 pi U(b4)).  Global steps are step0 + 1 ..
 * step0 + nsteps, so a run continued with step0 += nsteps continues the
 * streams.  temperature 0 stops the collided particles.  The kicks are not
 * fused into the force pass.  Arguments otherwise as mdpl_run; MDPL_EINVAL
 * for a negative temperature, rate or step0. */
mdpl_status mdpl_run_andersen(mdpl_sim* sim, double* x, double* y, double* z, double* vx,
                              double* vy, double* vz, void* fx, void* fy, void* fz, int32_t* ids,
                              int64_t nsteps, int32_t sample_every, double* thermo,
                              double temperature, double collision_rate, uint64_t seed,
                              int64_t step0, int32_t start);

/* Synchronise the stream and read the device flags (MDPL_FLAG_* bits) and
 * the largest neighbour count seen (so max_nb can be raised).  Returns
 * MDPL_ECAPACITY, MDPL_ESKIN or MDPL_ENONFINITE if the matching bit is set
 * (in that priority), else MDPL_OK.  Either output may be NULL. */
mdpl_status mdpl_check(mdpl_sim* sim, uint32_t* flags_host, int32_t* max_count_host);

/* Clear the device flags and the largest-count record (enqueued). */
mdpl_status mdpl_clear_flags(mdpl_sim* sim);

/* Kernel timing on the context's stream with HIP events.  When on, the runs
 * bracket launches 0, every, 2 every, ... of each force kernel (every >= 1;
 * 1: all of them) with an event pair: each pair makes the stream wait for
 * the kernel before it and costs a few microseconds of step time, so a
 * stride above 1 times a sample of the launches at a fraction of that cost.
 * on > 1 creates events for that many launches up front, so that none is
 * created while a timed run is enqueued (events are reused afterwards).
 * mdpl_kernel_time synchronises and returns the summed milliseconds and the
 * number of timed launches for `which` = 0 (plain force pass) or 1 (force
 * pass with energy and virial), then resets the record.  MDPL_EINVAL for
 * on < 0 or every < 1. */
mdpl_status mdpl_set_timing(mdpl_sim* sim, int32_t on, int32_t every);
mdpl_status mdpl_kernel_time(mdpl_sim* sim, int32_t which, double* ms_host, int64_t* launches_host);

/* Rebuilds of the runs of this context so far (host counters, no
 * synchronisation): all, those the VMAX rule made before reuse_every steps,
 * and the times the host waited for the stream to decide.  Any output may
 * be NULL. */
mdpl_status mdpl_rebuild_stats(mdpl_sim* sim, int64_t* rebuilds_host, int64_t* early_host,
                               int64_t* syncs_host);

/* Number of neighbour-list entries of the current list (sum of the
 * per-particle counts), after mdpl_build or mdpl_run.  Synchronises. */
mdpl_status mdpl_nlist_entries(mdpl_sim* sim, int64_t* entries_host);

/* ------------------------------------------------------- structure analysis
 * Both analyses use bonds |r_i - r_j| < rc (minimum image, strict, tested
 * in double exactly as (dx*dx + dy*dy) + dz*dz < rc*rc).  Outputs are in the
 * caller's particle order.  Workspace as above; host-validated. */
mdpl_status mdpl_analysis_workspace_bytes(int64_t n, const double* box_host, double rc,
                                          int32_t max_nb, size_t* bytes_host);

/* Steinhardt bond order (Sec. 4.1, Eqs. Qell and qellm; Algs. sph_I, sph_II):
 * q4, q6 (float, required), q5 (nullable) and nnb (int32, bond count |N(i)|;
 * Q_l = 0 when nnb = 0). */
mdpl_status mdpl_boa(const double* x, const double* y, const double* z, int64_t n,
                     const double* box_host, double rc, float* q4, float* q5, float* q6,
                     int32_t* nnb, void* workspace, size_t workspace_bytes, void* stream);

/* mdpl_boa without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The workspace of mdpl_boa is taken from a static
 * device array of MDPL_SCRATCH_BYTES per GPU, which every GPU the library
 * runs on holds until the process ends; nothing is allocated or freed.
 * Returns MDPL_ESCRATCH (and enqueues nothing) if the analysis needs more
 * than MDPL_SCRATCH_BYTES, i.e. if mdpl_analysis_workspace_bytes(n, box,
 * rc, 1) exceeds it (about 54 bytes per particle plus 4 per cell: some 10^6
 * particles at rho = 1, rc = 1.42).  Outputs as mdpl_boa.  Every call on one
 * GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (other streams or threads) race and must be serialised by the caller. */
#define MDPL_SCRATCH_BYTES (64ull << 20)
mdpl_status mdpl_boa_noalloc(const double* x, const double* y, const double* z, int64_t n,
                             const double* box_host, double rc, float* q4, float* q5, float* q6,
                             int32_t* nnb, void* stream);

/* Common-neighbour analysis (Sec. 4.2, Eqs. Ei and Ei_ordered; Algs. cna_I,
 * cna_II, cna_III and max_cluster_size).  1 <= max_nb <= 64 is the capacity
 * of a particle's bond list (the static size of Sec. 4.2, which must cover
 * the largest bond count for every triplet to be computed).  Per particle:
 * nnb[i] = number of bonds (may exceed max_nb); if nnb[i] <= max_nb,
 * trip[i*max_nb + k] for k < nnb[i] = the triplets of its bonds packed as
 * (n_cn << 20) | (n_b << 10) | n_lcb, sorted ascending (entries k >= nnb[i]
 * are not written), exact whatever the bond counts of its neighbours (the
 * bonds among its neighbours are tested directly); if nnb[i] > max_nb, no
 * triplets are written.  label[i] = 0 other, 1 fcc, 2 hcp, 3 bcc; every
 * reference signature has 12 or 14 bonds, so labels are exact for all
 * particles whenever max_nb >= 14.  max_count (device, nullable) receives
 * the largest bond count of any particle, so that a caller can see that
 * max_nb covered every particle or repeat with a larger one. */
mdpl_status mdpl_cna(const double* x, const double* y, const double* z, int64_t n,
                     const double* box_host, double rc, int32_t max_nb, uint32_t* trip,
                     int32_t* nnb, uint8_t* label, int32_t* max_count, void* workspace,
                     size_t workspace_bytes, void* stream);


/* ------------------------------------------------------- learned potential
 * (An extension; not in the paper.)  Descriptors of the particles of
 * the last mdpl_build with cutoff rc: 16 radial Gaussians
 * exp(-eta_r (r - R_k)^2) fc(r), R_k = 0.85 + 0.11 k, eta_r = 1/(2*0.11^2),
 * and 8 angular sums 2^(1-zeta) sum_{j != k} (1 + lam cos t_jik)^zeta w_j w_k,
 * w = exp(-eta r^2) fc(r), (zeta, lam, eta) in {1,4} x {+1,-1} x {0.5, 2}
 * (index 16 + 4 zi + 2 li + ei), fc(r) = (cos(pi r / rc) + 1) / 2.
 * G: n x 24 floats (caller order); mom: n x 50 floats (nullable), the
 * spherical-harmonic moments that mdpl_desc_bwd needs. */
mdpl_status mdpl_desc_fwd(mdpl_sim* sim, const double* x, const double* y, const double* z,
                          float* G, float* mom);

/* Forces F_i = -dE/dr_i of E = sum_i E_i(G_i), from dEdG (n x 24, dE_i/dG_i)
 * and mom of mdpl_desc_fwd at the same positions.  fx, fy, fz: float,
 * caller order, overwritten.  The pair terms are summed per tile in 64-bit
 * fixed point and then added to the outputs with FP32 device atomics, so
 * the last bits of the forces may differ between runs (the sum of all
 * forces stays zero to rounding). */
mdpl_status mdpl_desc_bwd(mdpl_sim* sim, const double* x, const double* y, const double* z,
                          const float* dEdG, const float* mom, float* fx, float* fy, float* fz);

/* Network 24 -> 64 -> 64 -> 1 with SiLU: inputs g = (G - mu) / sd padded
 * to 32, E = e_mean + e_sd (w3 . silu(W2 silu(W1 g + b1) + b2) + b3).
 * Weights are bfloat16 bit patterns, row-major [out][in]: w1 64 x 32
 * (columns 24..31 must be zero), w2 64 x 64, w3 64; biases float. */
typedef struct {
  const uint16_t* w1;
  const float* b1;
  const uint16_t* w2;
  const float* b2;
  const uint16_t* w3;
  const float* b3;
  const float* mu;  /* 24 */
  const float* sd;  /* 24 */
  float e_mean, e_sd;
} mdpl_mlp_weights;

/* Number of trainable parameters in the packed FP32 vector used by
 * training: W1 [64][32] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3. */
#define MDPL_MLP_PARAMS 6337

/* Per-atom energies (n floats, nullable) and, if dEdG is not NULL, dE/dG
 * (n x 24 floats) for features G (n x 24), on the BF16 matrix cores. */
mdpl_status mdpl_mlp_fwd(const mdpl_mlp_weights* w, const float* G, int64_t n, float* energy,
                         float* dEdG, void* stream);

/* One force evaluation of the learned potential at positions x, y, z (caller
 * order) already built in sim (mdpl_build): mdpl_desc_fwd, mdpl_mlp_fwd and
 * mdpl_desc_bwd in one call that gathers the positions once and clears the
 * force outputs inside the descriptor pass (no separate clearing launch).
 * ws: device workspace of mdpl_mlp_run_floats(n) floats (features, moments,
 * energies, dE/dG; contents undefined afterwards).  energy: per-atom
 * energies (n floats, nullable); fx, fy, fz: float, caller order,
 * overwritten, with the run-to-run last-bit variation of mdpl_desc_bwd.
 * The sim must use full neighbour lists (not half lists or the list-free
 * loop).  Errors: MDPL_EINVAL (null argument, unsupported list mode),
 * MDPL_ESTATE (no mdpl_build), MDPL_EWORKSPACE (ws too small). */
mdpl_status mdpl_mlp_forces(mdpl_sim* sim, const mdpl_mlp_weights* w, const double* x,
                            const double* y, const double* z, float* ws, int64_t ws_floats,
                            float* energy, float* fx, float* fy, float* fz);

/* Floats of scratch mdpl_mlp_train_grad needs for a batch of `batch` rows. */
mdpl_status mdpl_mlp_train_floats(int64_t batch, int64_t* floats_host);

/* Loss L = sum_b (y_b - t_b)^2 / batch (y as above without e_mean/e_sd)
 * over the rows a = index[0..batch) of G, with the standardised target
 * t_b = (energy[a] - e_mean) / e_sd (energy: per-atom FP64 energies indexed
 * like G), and dL/dparams.  grad: MDPL_MLP_PARAMS + 1 floats receiving the
 * packed gradient and, last, L.  index: nullable (rows 0..batch).
 * scratch: mdpl_mlp_train_floats. */
mdpl_status mdpl_mlp_train_grad(const mdpl_mlp_weights* w, const float* G, const int32_t* index,
                                int64_t batch, const double* energy, float* scratch,
                                int64_t scratch_floats, float* grad, void* stream);

/* Standardisation of a training set (n rows of features G, n x 24 floats,
 * and per-atom energies e, FP64): mu[c] = mean of feature c, sd[c] = its
 * population standard deviation + 1e-6 (24 floats each), e_stats[0] = mean
 * energy, e_stats[1] = its population standard deviation + 1e-12 (FP64).
 * Sums in FP64 in a fixed order (two passes); device outputs.  scratch:
 * MDPL_MLP_STD_SCRATCH doubles. */
#define MDPL_MLP_STD_SCRATCH (256 * 25 + 50)
mdpl_status mdpl_mlp_standardise(const float* G, const double* e, int64_t n, float* mu,
                                 float* sd, double* e_stats, double* scratch, void* stream);

/* The bf16 copies w1, w2, w3 (layouts as in mdpl_mlp_weights) of the packed
 * FP32 parameters, rounded to nearest even (mdpl_adam_step refreshes them
 * after every step; this sets them for the initial parameters). */
mdpl_status mdpl_mlp_bf16(const float* params, uint16_t* w1, uint16_t* w2, uint16_t* w3,
                          void* stream);

/* One bias-corrected Adam step (step t >= 1) on the packed FP32 parameters
 * with moments m, v; then writes the bf16 copies w1, w2, w3 (layouts as in
 * mdpl_mlp_weights).  Padding columns of W1 are kept at zero. */
mdpl_status mdpl_adam_step(float* params, const float* grad, float* m, float* v, float lr,
                           float beta1, float beta2, float eps, int32_t step, uint16_t* w1,
                           uint16_t* w2, uint16_t* w3, void* stream);

/* v *= factor for n particles (used to hold a temperature while generating
 * training configurations). */
mdpl_status mdpl_scale_velocities(double* vx, double* vy, double* vz, int64_t n, double factor,
                                  void* stream);

/* Floats of caller workspace mdpl_run_mlp needs for n particles (99 n:
 * features, moments, energies, dE/dG). */
mdpl_status mdpl_mlp_run_floats(int64_t n, int64_t* floats_host);

/* mdpl_run with the learned potential as the force field (Alg.
 * VelocityVerlet with list reuse, Sec. 3.5; forces F = -grad sum_i E_i).
 * Same state arrays, in-place reordering, ids, flags and rebuild rule as
 * mdpl_run; the sim must have precision MDPL_FP32 (forces are float) and
 * its rc is the descriptor cutoff.  thermo rows: KE, sum_i E_i (FP64 sum
 * of the FP32 per-atom energies), 0 (no virial), max displacement.  ws:
 * mdpl_mlp_run_floats floats (MDPL_EWORKSPACE if fewer); its contents are
 * scratch.  Force-pass timing (mdpl_set_timing) is recorded as for LJ. */
mdpl_status mdpl_run_mlp(mdpl_sim* sim, const mdpl_mlp_weights* w, float* ws, int64_t ws_floats,
                         double* x, double* y, double* z, double* vx, double* vy, double* vz,
                         float* fx, float* fy, float* fz, int32_t* ids, int64_t nsteps,
                         int32_t sample_every, double* thermo, int32_t start);

/* out[0] = sum_i |f_i - g_i|^2, out[1] = sum_i |g_i|^2 over the sim's n
 * particles (FP64, fixed order): the force error of one force field (f,
 * float) against another (g, FP64) at the same positions.  out: 2 doubles
 * on the device; uses the sim's partials and stream. */
mdpl_status mdpl_force_error(mdpl_sim* sim, const float* fx, const float* fy, const float* fz,
                             const double* gx, const double* gy, const double* gz, double* out);

#ifdef __cplusplus
}
#endif

#endif /* MDPL_H */
