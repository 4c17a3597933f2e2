/*
 * jumpmd_oracle.h — API of the CPU FP64 oracle for the JUMP integrator.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the plain, slow, obviously-correct
 * reference that the GPU library is checked against. Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. It shares
 * no code, header, table or helper with the GPU library.
 *
 * Paper: "Velocity Jumps for Molecular Dynamics" (Gouraud et al., arXiv 2412.15073).
 * Citations below name the paper section / equation / algorithm.
 */
#ifndef JUMPMD_ORACLE_H
#define JUMPMD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* jump kinds */
#define ORC_JUMP_NONE 0
#define ORC_JUMP_BPS 1          /* Sec. 2.2 Eqs. (tauxbps),(reflexion); Sec. 3.2 */
#define ORC_JUMP_MRZ_CONST 2    /* Sec. 2.2 Eqs. (tauxsaut),(majvitesse), constant eps; Alg. 4 */
#define ORC_JUMP_MRZ_ADAPTIVE 3 /* same with eps(x) = eps0 |F_ij(x)| (Sec. 2.2, Sec. 3.1) */
#define ORC_JUMP_BOUNCE 4       /* Coulomb: BPS bounces in the (J) step together with the LJ ones, no
                                   acceleration between jumps (the BOUNCE scheme B J A O A J B, Sec. 3) */
#define ORC_JUMP_IN_C 5         /* LJ: the long part jumps in the (C) step with the Coulomb one, with the
                                   Coulomb kernel (Sec. 2.2 with F_ij the whole long-part force) */

/* random-stream phase tags (counter word 2, low byte) */
#define ORC_PH_O 1
#define ORC_PH_J1 2
#define ORC_PH_J2 3
#define ORC_PH_C1 4
#define ORC_PH_C2 5

/* force kinds for orc_accel */
#define ORC_F_SHORT 0   /* -grad of chi*U over r < r_s (non-bonded) */
#define ORC_F_FULL 1    /* -grad of U over r < r_c (non-bonded) */
#define ORC_F_BONDED 2  /* -grad of bonds + angles */
#define ORC_F_LONG 3    /* -grad of (1-chi)*U over r < r_c (non-bonded) */
#define ORC_F_RECIP 4   /* Ewald: -grad of the reciprocal-space energy and the excluded-pair correction */

/* electrostatics */
#define ORC_COUL_DSF 0    /* damped shifted-force Coulomb out to r_c, nothing beyond */
#define ORC_COUL_EWALD 1  /* the same real-space term plus the Ewald reciprocal sum (Sec. 3.1) */
#define ORC_COUL_SPME 2   /* the same, the reciprocal sum by smooth particle-mesh Ewald (Sec. 3.1) */

typedef struct {
  int32_t n_atoms, n_types;
  const double *pos, *vel;      /* [3N] */
  const double *mass, *charge;  /* [N] */
  const int32_t *type;          /* [N] in [0, n_types) */
  const double *lj_eps, *lj_sigma; /* [n_types^2] */
  double box[3];
  int32_t n_bonds;
  const int32_t *bond_ij;       /* [2*n_bonds] */
  const double *bond_k, *bond_r0;
  int32_t n_angles;
  const int32_t *angle_ijk;     /* [3*n_angles], j = vertex */
  const double *angle_k, *angle_t0;
  const int32_t *excl_ptr, *excl_j; /* CSR [N+1], symmetric; may be NULL */
  double coulomb_k;             /* energy*length/charge^2 */
  double accel_factor;          /* (energy/length)/mass -> length/time^2 */
  double kB;                    /* energy per kelvin (reduced units: 1) */
} orc_system;

typedef struct {
  double r_s, r_c, switch_width, skin, coulomb_alpha;
  int32_t n_rings;
  double ring_width;
  int32_t coulomb_kind;         /* ORC_COUL_DSF, ORC_COUL_EWALD or ORC_COUL_SPME */
  int32_t ewald_kmax;           /* Ewald: lattice vectors n with 0 < |n|^2 <= kmax^2 */
  int32_t pme_grid[3];          /* SPME: grid points per box edge */
  int32_t pme_order;            /* SPME: B-spline order (even, 4..8) */
} orc_split;

typedef struct {
  double dt, gamma, kT;
  uint64_t seed, replica;
  int32_t jump_lj, jump_coul;
  double eps;                   /* constant eps, or eps0 for the adaptive kind */
  int32_t respa_inner;
  int32_t rebuild_every;        /* 0: displacement-triggered */
  int32_t log_events;
  int32_t respa_outer;          /* middle steps per outer step of the three-level schemes */
} orc_params;

typedef struct orc_sim orc_sim;

/* primitives */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
uint64_t orc_event_mix(uint64_t h, int64_t step, int32_t phase, int32_t j);
double orc_theta(double eta);
double orc_zsample(double eta, uint64_t seed, uint64_t replica, int64_t step,
                   int64_t atom, int32_t phase, int64_t k, int32_t *iters);
void orc_pair_terms(double r, double eps, double sigma, double qq, double coulomb_k,
                    double alpha, double r_s, double w, double r_c, double out[6]);

/* simulation object */
orc_sim *orc_create(const orc_system *sys, const orc_split *split, const orc_params *par,
                    char *err, int errlen);
void orc_destroy(orc_sim *s);
int orc_step_baoab(orc_sim *s, int64_t n);
int orc_step_jump(orc_sim *s, int64_t n);
int orc_step_jump_respa(orc_sim *s, int64_t n_outer);
int orc_step_baoab_respa(orc_sim *s, int64_t n_outer);
int orc_step_jump_respa1(orc_sim *s, int64_t n_outer);   /* Ewald: three levels, Sec. 2.3.2 */
int orc_step_baoab_respa1(orc_sim *s, int64_t n_outer);
void orc_get_state(const orc_sim *s, double *pos, double *vel);
void orc_set_state(orc_sim *s, const double *pos, const double *vel, int64_t step);
int64_t orc_step_index(const orc_sim *s);
int64_t orc_n_rebuilds(const orc_sim *s);
int64_t orc_n_zsampler_overflow(const orc_sim *s);
int64_t orc_n_list_errors(const orc_sim *s);
/* accepted MRZ jumps by Z-sampler regime (Sec. 2.4): eta < -1, -1 <= eta <= 0, eta > 0 */
void orc_zsampler_regimes(const orc_sim *s, int64_t out[3]);
void orc_atom_stats(const orc_sim *s, int64_t *nprop, int64_t *nacc, int64_t *nviol, uint64_t *hash);
uint64_t orc_event_hash(const orc_sim *s);
int64_t orc_n_events(const orc_sim *s);
void orc_get_events(const orc_sim *s, int64_t *buf); /* 5 int64 per event: step, phase, i, j, k */
void orc_energies(const orc_sim *s, double out[7]);  /* ke, T, pe_short, pe_long, pe_bonded, pe_full,
                                                        pe_recip (Ewald: reciprocal + self + excluded-pair
                                                        correction; 0 otherwise; included in pe_full) */
void orc_accel(const orc_sim *s, int kind, double *acc); /* [3N], length/time^2 */
void orc_rdf(const orc_sim *s, int ta, int tb, double r_max, int n_bins, double *hist);

/* lists and bounds (rebuilt at the current positions by orc_build_lists) */
void orc_build_lists(orc_sim *s);
int32_t orc_n_segments(const orc_sim *s);
int64_t orc_cand_count(const orc_sim *s, int32_t i);
void orc_cand_row(const orc_sim *s, int32_t i, int32_t *j, int32_t *n); /* n: [3*len] image vectors, may be NULL */
void orc_seg_start(const orc_sim *s, int32_t i, int32_t *starts); /* [S+1] */
int64_t orc_pairs_within(const orc_sim *s, double rcut, int32_t *ij, int64_t cap);
void orc_bounds(const orc_sim *s, double *ell_lj, double *ell_coul_unit, double *qmax);
void orc_set_bound_scale(orc_sim *s, double scale);

/* single phases at the current state, for kernel-level parity */
void orc_phase_c(orc_sim *s, int32_t phase, double h, int a_kind);
void orc_phase_j(orc_sim *s, int32_t phase, double h);
void orc_phase_o(orc_sim *s, double h, int32_t substep);

#ifdef __cplusplus
}
#endif
#endif
