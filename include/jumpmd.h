/*
 * jumpmd.h — C ABI of libjumpmd.so, the MI355X (gfx950) implementation of the
 * hot path of the JUMP integrator of "Velocity Jumps for Molecular Dynamics"
 * (Gouraud, Lagardere, Adjoua, Ple, Monmarche, Piquemal; arXiv 2412.15073).
 *
 * Every step runs in HIP kernels on the caller's stream. Host pointers passed
 * in are read during the call and never retained (the caller keeps
 * ownership). Device memory of a context comes from the caller's allocator
 * (md_allocator, e.g. PyTorch's caching allocator, which then owns its
 * lifetime) or, without one, from hipMalloc; md_destroy returns all of it.
 * No call throws: every function returns MD_OK (0) or a negative MD_ERR_*
 * code, and md_last_error() gives a message for the last failure.
 *
 * Stepping calls are asynchronous on the context's stream. md_observables,
 * md_get_*, md_sync and md_profile_read synchronise the stream and report
 * device-side error flags (bound violations in strict mode, list
 * invalidation, non-finite state) raised by earlier steps. A neighbour row
 * that outgrew its capacity is not an error: the synchronising call restores
 * the state of the last good synchronisation, regrows the rows and replays
 * the stepping calls made since, so results are those of a run with enough
 * capacity from the start. One context per host thread; contexts are
 * independent.
 *
 * Units are the caller's: lengths, times, masses, energies and charges must
 * be consistent, with accel_factor converting force/mass to length/time^2
 * (1 for reduced units; 100 for kJ/mol, A, ps, amu) and coulomb_k the
 * Coulomb constant in energy*length/charge^2.
 */
#ifndef JUMPMD_H
#define JUMPMD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MD_OK 0
#define MD_ERR_ARG (-1)       /* invalid argument or unsupported combination */
#define MD_ERR_HIP (-2)       /* a HIP runtime call failed */
#define MD_ERR_BOUND (-3)     /* strict mode: an acceptance probability exceeded 1 */
#define MD_ERR_LIST (-4)      /* displacement beyond skin/2 on a fixed rebuild period */
#define MD_ERR_UNSTABLE (-5)  /* non-finite kinetic energy */
#define MD_ERR_OOM (-6)       /* device allocation failed */
#define MD_ERR_CAPACITY (-7)  /* rows would exceed the row builder's limits (8192 candidates, 4096 short
                                 entries per atom) even after regrowing; the state is then that of the
                                 last good synchronisation (the stepping calls since are not applied) */
#define MD_ERR_EVENTS (-8)    /* md_get_events: more accepted jumps were logged than the log holds
                                 (md_params.event_capacity); the events kept are an unspecified subset */

/* jump kinds (Sec. 2.2 of the paper) */
#define MD_JUMP_NONE 0
#define MD_JUMP_BPS 1          /* bouncy-particle rate beta (v.F)_+ and reflection, Eqs. (tauxbps),(reflexion) */
#define MD_JUMP_MRZ_CONST 2    /* rate/kernel of Eqs. (tauxsaut),(majvitesse), constant eps (Alg. 4) */
#define MD_JUMP_MRZ_ADAPTIVE 3 /* same with eps(x) = eps0 |F_ij(x)| */
#define MD_JUMP_BOUNCE 4       /* jump_coul only: the BOUNCE scheme of Sec. 3, B J A O A J B, with BPS
                                  bounces on the Coulomb long part in the (J) step together with the LJ
                                  ones (one chain over the whole long part, no acceleration between
                                  jumps); the (C) steps reduce to plain kicks */
#define MD_JUMP_IN_C 5         /* jump_lj only: the LJ long part jumps in the (C) step together with the
                                  Coulomb one, with jump_coul's kernel (one chain over the whole long
                                  part, bounds summed; Sec. 2.2 with F_ij the whole long-part force),
                                  no (J) step; needs jump_coul MRZ_CONST, MRZ_ADAPTIVE or BPS */

/* arithmetic of the pair terms */
#define MD_FP64 0
#define MD_FP32_MIXED 1        /* pair forces and jump rates in FP32; positions, velocities, sums in FP64 */

/* md_observables flags */
#define MD_OBS_PE 1u           /* also evaluate the potential energies (extra kernels) */

/* The system. Arrays are host pointers with the given lengths; atoms of
 * replica r are [replica_offset[r], replica_offset[r+1]). Bond, angle and
 * exclusion indices are global atom indices and must stay inside one
 * replica. Exclusions (CSR, symmetric, may be NULL) remove a pair from both
 * the force and the jump candidates. Velocities may not be NULL. */
typedef struct {
  int32_t n_atoms;
  int32_t n_types;
  int32_t n_replicas;             /* >= 1 */
  const double *pos;              /* [3N] unwrapped positions */
  const double *vel;              /* [3N] */
  const double *mass;             /* [N]  */
  const double *charge;           /* [N]  (may be NULL: all zero) */
  const int32_t *type;            /* [N]  in [0, n_types) */
  const double *lj_eps;           /* [n_types^2] 4*eps*((s/r)^12-(s/r)^6); 0 = no LJ */
  const double *lj_sigma;         /* [n_types^2] */
  const double *box;              /* [3*n_replicas] orthorhombic edges */
  const int32_t *replica_offset;  /* [n_replicas+1] (may be NULL when n_replicas == 1) */
  int32_t n_bonds;                /* harmonic bonds (k/2)(b-b0)^2 */
  const int32_t *bond_ij;         /* [2*n_bonds] */
  const double *bond_k, *bond_r0;
  int32_t n_angles;               /* harmonic angles (k/2)(theta-theta0)^2, vertex = middle index */
  const int32_t *angle_ijk;       /* [3*n_angles] */
  const double *angle_k, *angle_t0;
  const int32_t *excl_ptr;        /* [N+1] */
  const int32_t *excl_j;          /* [excl_ptr[N]] */
  double coulomb_k;
  double accel_factor;
  double kB;                      /* energy per kelvin, for the reported temperature */
} md_system;

/* The short/long split of every pair potential (Sec. 3.1, 3.2): chi = 1 below
 * r_s - switch_width, 0 above r_s (C2 quintic); forces from chi*U every step,
 * (1-chi)*U out to r_c drives the jumps. Pair terms are truncated at r_c
 * (LJ energy-shifted, Coulomb damped-shifted-force with coulomb_alpha).
 * skin: Verlet skin of all neighbour rows. n_rings/ring_width: jump
 * candidates are binned by build-time distance in rings of ring_width
 * starting at r_s - switch_width - skin, each with its own bound (ring
 * technique of Sec. 3.1.1; n_rings = 1 is the uniform per-atom bound of
 * Alg. 4/5). Requires every box edge > r_c + skin and r_s - w >= 1.25 sigma
 * of every LJ pair. Where an edge is below 2 (r_c + skin) (at most 8192 atoms
 * in such a replica), a partner can lie within the cutoff in two images:
 * rows then hold every image within the cutoff, each its own pair term and
 * jump candidate; elsewhere the nearest image is the only one. */
typedef struct {
  double r_s, r_c, switch_width, skin, coulomb_alpha;
  int32_t n_rings;
  double ring_width;
  int32_t coulomb_kind;  /* MD_COUL_DSF, MD_COUL_EWALD or MD_COUL_SPME */
  int32_t ewald_kmax;    /* Ewald: lattice vectors n with 0 < |n|^2 <= kmax^2 in the reciprocal sum */
  int32_t pme_grid[3];   /* SPME: grid points per box edge, powers of two in [8, 256], >= pme_order */
  int32_t pme_order;     /* SPME: cardinal B-spline order, 4, 6 or 8 */
} md_split;

/* electrostatics (md_split.coulomb_kind) */
#define MD_COUL_DSF 0    /* damped shifted-force Coulomb out to r_c, nothing beyond */
#define MD_COUL_EWALD 1  /* Ewald (Sec. 3.1): the same real-space term with coulomb_alpha, plus the
                            reciprocal-space sum over ewald_kmax (with the self term and the excluded
                            pairs taken back); one replica only; schemes md_step_baoab and
                            md_step_jump (reciprocal forces in every kick or C' acceleration) and the
                            three-level md_step_jump_respa1 and md_step_baoab_respa1 */
#define MD_COUL_SPME 2   /* as MD_COUL_EWALD, with the reciprocal sum by smooth particle-mesh Ewald
                            (Essmann et al. 1995; the paper's Tinker runs use it): charges spread
                            with order-pme_order B-splines on the pme_grid mesh, three-dimensional
                            transforms, the B-spline-corrected influence function, forces gathered
                            with the B-spline derivatives; spreading sums with atomics, so results
                            agree between runs to rounding, not bit for bit */

/* Device memory for a context (md_create): alloc returns `bytes` of device
 * memory usable on `stream` (NULL on failure), release gives it back. Both
 * are called only inside md_create, the synchronising calls (when rows are
 * regrown), md_rdf (first use of a histogram size) and md_destroy, never
 * during stepping or graph capture. ctx is passed through unchanged. */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*release)(void *ctx, void *ptr, size_t bytes, void *stream);
} md_allocator;

typedef struct {
  double dt;            /* time step (inner step for the RESPA schemes) */
  double gamma;         /* friction */
  double kT;            /* energy */
  uint64_t seed;        /* counter-based Philox4x32-10 key: (low 32 bits of seed, high 32 bits of
                           seed xor replica index); counters (step, local atom, phase tag, draw) */
  int32_t jump_lj;      /* MD_JUMP_NONE, MD_JUMP_BPS (J step, Alg. 5) or MD_JUMP_IN_C */
  int32_t jump_coul;    /* MD_JUMP_NONE, MD_JUMP_MRZ_CONST or MD_JUMP_MRZ_ADAPTIVE (C step, Alg. 4),
                           or MD_JUMP_BPS: bounces of Sec. 3.2 in the C step (the eps -> infinity
                           end of the MRZ family, Sec. 2.2), or MD_JUMP_BOUNCE: bounces in the J step */
  double eps;           /* eps (constant) or eps0 (adaptive, 1/force units); unused with BPS */
  int32_t precision;    /* MD_FP64 or MD_FP32_MIXED */
  int32_t rebuild_every;/* 0: rebuild when max displacement > skin/2; k>0: every k steps */
  int32_t respa_inner;  /* inner steps per outer step of the RESPA schemes (>= 1) */
  int32_t log_events;   /* 1: record every accepted jump for md_get_events */
  int32_t strict_bounds;/* 1: an acceptance probability > 1 makes the next sync fail with MD_ERR_BOUND */
  int32_t chain_lanes;  /* lanes per atom in the jump chains: 0 = automatic, or 1, 2, 4, 8, 16
                           (results do not depend on it) */
  int32_t graph_steps;  /* 0: launch kernels step by step; K > 0 (even): md_step_jump and
                           md_step_baoab replay a captured HIP graph of K steps (needs
                           rebuild_every == 0; results do not depend on it) */
  double bound_scale;   /* every jump-rate bound multiplied by this (0 or 1: the bounds as derived).
                           Thinning is exact for any valid bound (Sec. 2.4): > 1 leaves the law
                           unchanged; < 1 makes bounds invalid (counted; MD_ERR_BOUND in strict mode) */
  double row_capacity;  /* initial row capacity as a multiple of the density estimate (0: 1.5);
                           rows regrow on demand, so this only trades memory for early regrows */
  int64_t event_capacity; /* accepted jumps the event log holds (log_events = 1); 0: 2^22 */
  int32_t chain_order;  /* wave order of the jump chains: 0 or 1 by atom type (heaviest chains first),
                           2 replica by replica (each by type); results do not depend on it */
  int32_t respa_outer;  /* middle steps per outer step of the three-level RESPA schemes (>= 1) */
} md_params;

typedef struct {
  int64_t step;
  double time;
  double ke, temperature;
  double pe_short, pe_long, pe_bonded;  /* filled when MD_OBS_PE is set */
  int64_t n_prop, n_acc, n_bound_viol, n_rebuilds, n_zsampler_overflow, n_list_errors;
  uint64_t event_hash;  /* FNV-1a over the per-atom event hashes, atom order */
  int64_t n_regrows;    /* times the rows were regrown and the steps replayed */
  double pe_recip;      /* MD_OBS_PE with Ewald: reciprocal sum + self term + excluded-pair correction */
} md_obs;

typedef struct {          /* one accepted jump */
  int64_t step;
  int32_t phase;          /* 2/3: J first/second half, 4/5: C first/second half */
  int32_t atom;           /* global index */
  int32_t partner;        /* global index */
  int32_t proposal;       /* index of the proposal within the atom's chain */
} md_event;

typedef struct md_ctx md_ctx;

/* Create a context for the JUMP integrator (Sec. 2.3 step composition,
 * Sec. 3.1 short/long split, Alg. 4/5 jump chains): validates the input
 * (MD_ERR_ARG: shapes, ranges, indices outside [0, N) or outside their
 * replica, non-monotone replica or exclusion offsets), computes the rate
 * bounds of the ring technique (Sec. 3.1.1), uploads the system and sets up
 * the jump-chain layout on `stream` (a hipStream_t; NULL: a private
 * non-blocking stream). alloc may be NULL (hipMalloc). On failure *out is
 * NULL and the code says why (message via md_last_error(NULL)); MD_ERR_OOM
 * when an allocation failed. Rows and forces are built at the first step. */
int md_create(const md_system *sys, const md_split *split, const md_params *par,
              void *stream, const md_allocator *alloc, md_ctx **out);
void md_destroy(md_ctx *ctx);
const char *md_last_error(const md_ctx *ctx);

/* BAOAB with full-range forces (r < r_c): B A O A B (Sec. 2.3 without J). */
int md_step_baoab(md_ctx *ctx, int64_t nsteps);
/* JUMP: C' J' A O A J' C' (Sec. 2.3, 3.3): C' = short forces + Coulomb jumps
 * (plain B kick if jump_coul is NONE), J' = LJ jumps (skipped if NONE). With
 * Ewald electrostatics the jumps act on the damped real-space long part and
 * the C' acceleration also carries the reciprocal-space forces, evaluated
 * every step (Sec. 3.1: everything not jumped is in the acceleration). */
int md_step_jump(md_ctx *ctx, int64_t nsteps);
/* JUMP-RESPA (Sec. 2.3.2, 3.3): bonded forces at dt, short non-bonded forces
 * and all jumps at respa_inner*dt. */
int md_step_jump_respa(md_ctx *ctx, int64_t n_outer);
/* BAOAB-RESPA comparator: full-range non-bonded kick at the outer step. */
int md_step_baoab_respa(md_ctx *ctx, int64_t n_outer);
/* JUMP-RESPA1 (Sec. 2.3.2, Sec. 3.3, Table 2; needs MD_COUL_EWALD or MD_COUL_SPME): three
 * levels, bonded forces at dt, short non-bonded forces and all jumps at
 * respa_inner*dt (the JUMP-RESPA step), reciprocal-space forces at
 * respa_outer*respa_inner*dt. n_outer outer steps. */
int md_step_jump_respa1(md_ctx *ctx, int64_t n_outer);
/* BAOAB-RESPA1 comparator (needs MD_COUL_EWALD or MD_COUL_SPME): bonded forces at dt, short
 * non-bonded chi U at respa_inner*dt, the long real-space part (1 - chi) U and
 * the reciprocal-space forces at respa_outer*respa_inner*dt. */
int md_step_baoab_respa1(md_ctx *ctx, int64_t n_outer);

/* Synchronise and report the observables of Sec. 4: kinetic energy and
 * temperature 2 KE / (3 N kB) (no centre-of-mass constraint), jump
 * statistics, and with MD_OBS_PE the potential energies of the split
 * (Sec. 3.1): short part chi U, long part (1 - chi) U (pairs r < r_c,
 * each once) and bonded. Returns the first pending error (above). */
int md_observables(md_ctx *ctx, uint32_t flags, md_obs *out);
int md_sync(md_ctx *ctx);

/* Host copies of the state (x, v of Sec. 2.1; [3N] each, either may be
 * NULL; positions unwrapped). md_set_state rebuilds the neighbour rows and
 * forces at the new positions at the next step; step < 0 keeps the step
 * counter. Both synchronise. */
int md_get_state(md_ctx *ctx, double *pos, double *vel);
int md_set_state(md_ctx *ctx, const double *pos, const double *vel, int64_t step);
/* Current accelerations [3N]: kind 0 = short non-bonded, 1 = full non-bonded,
 * 2 = bonded, 3 = long real-space part (1 - chi) U, 4 = Ewald reciprocal
 * space with the excluded-pair correction (evaluated at the current
 * positions). */
int md_get_accel(md_ctx *ctx, int32_t kind, double *acc);
/* Per-atom jump statistics [N] each (any may be NULL). */
int md_get_atom_stats(md_ctx *ctx, int64_t *n_prop, int64_t *n_acc, int64_t *n_viol, uint64_t *hash);
/* Accepted-jump log (log_events = 1), sorted by (step, phase, atom,
 * proposal); the log holds event_capacity events since creation. buf may be NULL to
 * query *n. MD_ERR_EVENTS when events were lost (*n = those kept). */
int md_get_events(md_ctx *ctx, md_event *buf, int64_t cap, int64_t *n);
/* Pair histogram of types (ta, tb) over [0, r_max) in n_bins bins, pairs
 * inside each replica (minimum image), unordered when ta == tb. */
int md_rdf(md_ctx *ctx, int32_t ta, int32_t tb, double r_max, int32_t n_bins, double *hist);
/* Velocity trace for autocorrelation spectra (Sec. 4, Figs. 3-4: spectra at
 * the level of the smallest time step). From this call on, every O update
 * (once per smallest step in every scheme: mid-step of BAOAB and JUMP, every
 * inner step of the RESPA schemes) records the velocities of atoms
 * [0, n_atoms) into a ring of `capacity` records on the device (memory from
 * the context's allocator); steps then run without HIP-graph replay.
 * n_atoms = 0 stops tracing and frees the ring. Records count from 0 at each
 * call. MD_ERR_ARG for n_atoms outside [0, N] or capacity < 1 with
 * n_atoms > 0; MD_ERR_OOM when the ring cannot be allocated. */
int md_trace_velocities(md_ctx *ctx, int32_t n_atoms, int64_t capacity);
/* The last min(recorded, capacity, max_records) records in time order, as
 * [records][n_atoms][3] doubles in out (host); *n_out = records copied,
 * *n_recorded = records taken since md_trace_velocities. MD_ERR_ARG when no
 * trace is active. */
int md_get_trace(md_ctx *ctx, double *out, int64_t max_records, int64_t *n_out, int64_t *n_recorded);

/* Allocation-free variant of md_rdf, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments and result as md_rdf; n_bins at most
 * 16384 (MD_ERR_ARG above). The counts live in a static device array of the
 * library (256 KiB per device, held until the process ends), set up once per
 * device at md_create; the call allocates nothing and synchronises the
 * stream. All calls on one device share that array: calls that overlap on
 * one device (other host threads or streams) race. Rows that outgrew their
 * capacity since the last synchronisation are not regrown here (regrowing
 * allocates): the call then returns MD_ERR_CAPACITY and changes nothing, and
 * md_sync must run first. Other pending device-side errors are reported as by
 * md_sync. */
int md_rdf_noalloc(md_ctx *ctx, int32_t ta, int32_t tb, double r_max, int32_t n_bins, double *hist);

/* Neighbour rows as last built (for checks): candidate row of atom i (global
 * j indices, sorted by (type of j, ring, j, image)) and its S+1 segment
 * starts, S = n_types*n_rings. *n receives the row length; j, img and
 * seg_start may be NULL. In a replica with an edge below 2 (r_c + skin) a
 * candidate is one periodic image x_j + n L of j (n an integer vector fixed
 * at the row build) and img[k] = (n_x mod 8) | (n_y mod 8) << 3 |
 * (n_z mod 8) << 6; elsewhere candidates are nearest images and img[k] = -1. */
int md_get_cand_row(md_ctx *ctx, int32_t i, int32_t *j, int32_t *img, int32_t cap, int32_t *n,
                    int32_t *seg_start);
/* Number of (i,j) entries in the short rows (r < r_s + skin at build), both directions. */
int md_get_row_counts(md_ctx *ctx, int32_t which, int32_t *counts);

/* Run one phase at the current state (for kernel-level checks): 'C' or 'J'
 * with the given phase tag and half-step h, 'O' with step h. */
int md_run_phase(md_ctx *ctx, int32_t which, int32_t phase, double h);

/* Per-kernel timing with HIP events on the context's stream. enable = 1
 * starts recording (resets the sums); md_profile_read synchronises and
 * returns the total milliseconds and launch count of kernel `kid`
 * (MD_K_* below). */
#define MD_K_LOCAL 0      /* per-atom B/A/O updates and displacement check */
#define MD_K_FORCE 1      /* non-bonded pair forces (with the bonded forces when both are due) */
#define MD_K_BONDED 2
#define MD_K_REBUILD 3    /* all neighbour-row kernels of a step */
#define MD_K_CHAIN 4      /* jump chains (J and C ops, with the kicks between them) */
#define MD_K_RECIP 5      /* Ewald reciprocal-space forces */
#define MD_K_COUNT 6
int md_profile(md_ctx *ctx, int32_t enable);
int md_profile_read(md_ctx *ctx, int32_t kid, double *total_ms, int64_t *launches);

/* Work counters for throughput reporting: unordered pairs inside the cutoff
 * of the last force evaluation (r < r_s for the JUMP schemes, r < r_c for
 * BAOAB; -1 if no force is current), and the jump proposals evaluated since
 * creation. Synchronises. */
int md_counters(md_ctx *ctx, int64_t *pairs_last, int64_t *proposals_total);

/* Autotuner of the launch and list settings that leave the method's law
 * unchanged: lanes per atom of the jump chains (results do not depend on
 * them), the Verlet skin and the ring count of the rate bounds (exact thinning
 * for any valid bound, Sec. 2.4, Sec. 3.1.1: they change the random proposals
 * drawn, not the law of the process), and HIP-graph replay. Each trial creates
 * a context for `sys` with one setting (device memory from alloc, as
 * md_create), runs untimed warm-up steps of `scheme` and times `steps` steps
 * with HIP events on `stream`; a coordinate descent over lanes {auto, 1, 2, 4,
 * 8, 16}, the wave order of the chains (several replicas: by type, by
 * replica), skin x {0.6, 0.8, 1.2, 1.5, 2} (edges must stay above
 * r_c + skin), rings x {1/2, 3/2, 2} (n_types * n_rings <= 32) and graph
 * steps {0, 10, 20, 50}, then lanes again. *split_out / *params_out receive the caller's split
 * and parameters with the fastest setting, *ms_out its ms per step; trials
 * (may be NULL) receives up to cap of the settings timed, *n_trials their
 * number. The result is cached per process (same system shape, split,
 * parameters, scheme and steps: no trials). Synchronous. */
#define MD_SCHEME_BAOAB 0
#define MD_SCHEME_JUMP 1
#define MD_SCHEME_JUMP_RESPA 2
#define MD_SCHEME_BAOAB_RESPA 3
typedef struct {
  int32_t chain_lanes;
  double skin;
  int32_t n_rings;
  int32_t graph_steps;
  int32_t chain_order;
  double ms_per_step;
} md_tune_trial;
int md_tune(const md_system *sys, const md_split *split, const md_params *params, void *stream,
            const md_allocator *alloc, int32_t scheme, int32_t steps, md_split *split_out,
            md_params *params_out, double *ms_out, md_tune_trial *trials, int32_t cap, int32_t *n_trials);

/* Diagnostic of the float screen of Theta (Sec. 2.2, Theta(eta) = eta Phi(eta)
 * + phi(eta)) that the FP64 jump chains use to take most acceptance decisions
 * without FP64 Theta: the largest relative error of the screen against FP64
 * Theta over n >= 2 points evenly spaced in [eta_lo, eta_hi], computed on the
 * current device (a few hundred bytes of scratch, freed on return).
 * *max_rel_err receives it. Synchronous. MD_ERR_ARG for n < 2 or
 * eta_lo >= eta_hi; the message is then in md_last_error(NULL). */
int md_theta_screen_error(double eta_lo, double eta_hi, int32_t n, double *max_rel_err);

#ifdef __cplusplus
}
#endif
#endif
