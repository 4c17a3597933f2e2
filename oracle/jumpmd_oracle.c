/*
 * jumpmd_oracle.c — plain CPU FP64 oracle of the JUMP integrator.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library. It shares no
 * code with the GPU path. Everything here is written for being checked by eye
 * against the paper, not for speed: all pair sums are brute force over every
 * pair of atoms and every periodic image within the cutoff, candidate rows are
 * built by brute force and sorted with qsort, every jump chain is a sequential
 * loop.
 *
 * Paper: Gouraud, Lagardere, Adjoua, Ple, Monmarche, Piquemal,
 * "Velocity Jumps for Molecular Dynamics", arXiv 2412.15073.
 *
 * Readings of the paper that this file adopts (the supporting information
 * that would fix them is not part of the paper text):
 *  - switching function chi: C2 quintic smoothstep, chi = 1 for r <= r_s - w,
 *    chi = 0 for r >= r_s (Sec. 3.1 only says it goes smoothly from 1 to 0);
 *  - F_ij is a gradient (Sec. 2.1: grad U = sum F_i; Sec. 3.1: F_ij = grad_{x_i}
 *    of the long part), so the force on atom i is -F_ij;
 *  - jump candidates of atom i are the entries of a neighbour row built with a
 *    skin (Remark in Sec. 3.1.1) rather than all N atoms (Alg. 4, Alg. 5);
 *    candidates whose long-range gradient is exactly zero have rate zero;
 *  - thinning uses the exponential clock of Alg. 1/2 for the J step as well
 *    (equivalent in law to the Poisson count of Alg. 3/5, Sec. 2.4);
 *  - in the C step the local rate bound is re-evaluated after each accepted
 *    jump (Sec. 2.4) rather than after each proposal (Alg. 4); both are exact;
 *  - in Alg. 1/2/4 the overflow branch ends the half step;
 *  - adaptive eps: eps = eps0 |F_ij| (Sec. 2.2) inserted in Eqs.
 *    (tauxsaut),(majvitesse), per-candidate bound beta*B_v*l_j + sqrt(beta/(2 pi m))/eps0;
 *  - BPS kernel for the Coulomb long part runs in the C step (acceleration
 *    between bounces), the eps -> infinity end of the MRZ family (Sec. 2.2);
 *  - Z = eta + G~ is drawn by exact rejection from the density
 *    z exp(-(z-eta)^2/2) on z > 0 with the regimes of Sec. 2.4
 *    (Gamma(2) for eta < -1, Rayleigh for -1 <= eta <= 0, mixed
 *    Rayleigh-Gaussian for eta > 0).
 */
#include "jumpmd_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Planted mistakes for the mutation tests (tests/test_oracle_mutants.py):
 * a build with -DORC_PLANT=k > 0 plants mistake k, which at least one pin of
 * tests/test_oracle_pins.py must catch. The default build plants nothing. */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

#define PI 3.14159265358979323846
#define ZS_MAXIT 64
#define MAX_PROPOSALS (1ll << 22) /* per chain and half step */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of a
 * multiply-based bijection on four 32-bit words, keyed by a Weyl sequence
 * on two 32-bit key words. */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in the open interval (0,1): (word + 1/2) / 2^32, exact */
double orc_u01(uint32_t w) {
  return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* One block of four uniforms. Counter words: step, local atom index,
 * tag = phase | substep << 8 | Z-iteration << 24, proposal index k (each
 * taken modulo 2^32); key words: low and high halves of the seed, the
 * high half xor the replica index. */
static void draw4(uint64_t seed, uint64_t replica, int64_t step, int64_t atom,
                  uint64_t tag, int64_t k, double u[4]) {
  uint32_t ctr[4] = {(uint32_t)step, (uint32_t)atom, (uint32_t)tag, (uint32_t)k};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)replica};
  uint32_t w[4];
  orc_philox4x32(ctr, key, w);
  for (int q = 0; q < 4; q++) u[q] = orc_u01(w[q]);
}

/* ------------------------------------------------------------------------ */
/* Theta(eta) = E[(eta + G)_+], G ~ N(0,1)  (Sec. 2.2, Eq. (tauxsaut)).
 * Closed form eta*Phi(eta) + phi(eta). */
double orc_theta(double eta) {
  double Phi = 0.5 * erfc(-eta / sqrt(2.0));
  double phi = exp(-0.5 * eta * eta) / sqrt(2.0 * PI);
  return eta * Phi + phi;
}

/* Z = eta + G~ where G~ has density (eta+y)_+ exp(-y^2/2) / (Theta sqrt(2 pi))
 * (Sec. 2.2, Eq. (majvitesse)); rejection sampling as in Sec. 2.4.
 * Iteration r draws one Philox block with counter word 2 = phase | (r+1)<<24. */
double orc_zsample(double eta, uint64_t seed, uint64_t replica, int64_t step,
                   int64_t atom, int32_t phase, int64_t k, int32_t *iters) {
  for (int r = 0; r < ZS_MAXIT; r++) {
    double u[4];
    uint64_t tag = (uint64_t)(uint32_t)phase | ((uint64_t)(r + 1) << 24);
    draw4(seed, replica, step, atom, tag, k, u);
    if (iters) *iters = r + 1;
    if (eta > 0.0) {
      /* proposal density on y: eta*exp(-y^2/2) (Gaussian part, mass eta*sqrt(2 pi))
       * plus y_+ exp(-y^2/2) (Rayleigh part, mass 1) */
      double p_ray = 1.0 / (1.0 + eta * sqrt(2.0 * PI));
      double y;
      if (u[0] < p_ray) {
        y = sqrt(-2.0 * log(u[1]));
      } else {
        y = sqrt(-2.0 * log(u[1])) * cos(2.0 * PI * u[2]);
      }
      double z = eta + y;
      if (y >= 0.0) return z;          /* target/proposal ratio 1 */
      if (z <= 0.0) continue;          /* ratio 0 */
      if (u[3] <= z / eta) return z;   /* ratio (eta+y)/eta */
    } else if (eta >= -1.0) {
      /* Rayleigh proposal z exp(-z^2/2); ratio exp(eta z) <= 1 */
      double z = sqrt(-2.0 * log(u[0]));
      if (u[1] <= exp(eta * z)) return z;
    } else {
      /* Gamma(2, rate |eta|) proposal z exp(-|eta| z); ratio exp(-z^2/2) */
      double z = -(log(u[0]) + log(u[1])) / (-eta);
      if (u[2] <= exp(-0.5 * z * z)) return z;
    }
  }
  if (iters) *iters = -1;
  return 0.5 * (eta + sqrt(eta * eta + 4.0)); /* mode; only after ZS_MAXIT rejections */
}

/* ------------------------------------------------------------------------ */
/* Pair potential pieces (Sec. 3.1 direct electrostatics, Sec. 3.2 LJ):
 *  LJ truncated and energy-shifted at r_c: 4 eps [(s/r)^12 - (s/r)^6] - (same at r_c)
 *  damped shifted-force Coulomb (Fennell-Gezelter) with damping alpha, cut at r_c
 *  switch chi(r) on [r_s - w, r_s].
 * out = {U_lj, dU_lj/dr, U_c, dU_c/dr, chi, dchi/dr} */
static void lj_terms(double r, double eps, double sig, double rc, double *U, double *dU) {
  *U = 0.0; *dU = 0.0;
  if (eps == 0.0 || r >= rc) return;
  double sr6 = pow(sig / r, 6.0);
  double sc6 = pow(sig / rc, 6.0);
  *U = 4.0 * eps * (sr6 * sr6 - sr6) - 4.0 * eps * (sc6 * sc6 - sc6);
  *dU = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
}

static void dsf_terms(double r, double qq, double ke, double alpha, double rc, double *U, double *dU) {
  *U = 0.0; *dU = 0.0;
  if (qq == 0.0 || r >= rc) return;
  double two_a_sqpi = 2.0 * alpha / sqrt(PI);
  double erfc_rc = erfc(alpha * rc);
  double fc = erfc_rc / (rc * rc) + two_a_sqpi * exp(-alpha * alpha * rc * rc) / rc;
  double erfc_r = erfc(alpha * r);
  *U = ke * qq * (erfc_r / r - erfc_rc / rc + fc * (r - rc));
  *dU = ke * qq * (-(erfc_r / (r * r) + two_a_sqpi * exp(-alpha * alpha * r * r) / r) + fc);
}

static void switch_terms(double r, double rs, double w, double *chi, double *dchi) {
  double rlo = rs - w;
  if (r <= rlo) { *chi = 1.0; *dchi = 0.0; return; }
  if (r >= rs) { *chi = 0.0; *dchi = 0.0; return; }
  double t = (r - rlo) / w;
  *chi = 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
  *dchi = -30.0 * t * t * (1.0 - t) * (1.0 - t) / w;
}

void orc_pair_terms(double r, double eps, double sigma, double qq, double coulomb_k,
                    double alpha, double r_s, double w, double r_c, double out[6]) {
  lj_terms(r, eps, sigma, r_c, &out[0], &out[1]);
  dsf_terms(r, qq, coulomb_k, alpha, r_c, &out[2], &out[3]);
  switch_terms(r, r_s, w, &out[4], &out[5]);
}

/* ------------------------------------------------------------------------ */
/* A jump candidate of atom i is one periodic image of atom j: the image at
 * x_j + n L (n an integer vector fixed when the row is built), so that its
 * displacement is d = x_i - x_j - n L. img = (s_x+1) + 3 (s_y+1) + 9 (s_z+1)
 * numbers the image by its offset s = n - m from the nearest image m at the
 * build (the order of images of one j inside a row). */
typedef struct { int32_t seg, j, img; int32_t n[3]; } cand_t;

struct orc_sim {
  int n, nt;
  double *x, *v, *mass, *me, *q;
  int32_t *type;
  double *eps, *sig;
  double L[3];
  int nb; int32_t *bij; double *bk, *br0;
  int na; int32_t *aijk; double *ak, *at0;
  int32_t *xptr, *xj;
  double ke_c, accel, kB;
  double rs, rc, w, skin, alpha, rlo; int nr; double rw;
  double dt, gamma, kT, beta; uint64_t seed, replica;
  int jlj, jc; double eps0; int respa_inner, rebuild_every, log_events, respa_outer;
  int coul_kind, kmax;  /* electrostatics: DSF, or DSF real part + Ewald reciprocal sum */
  int pme_K[3], pme_p;  /* SPME grid and B-spline order */
  double *frec;         /* Ewald reciprocal-space forces (-grad), with the excluded-pair correction */
  int frec_valid;
  /* state */
  int64_t step;
  double *xref;
  int64_t steps_since_build;
  double *fnb, *fb;   /* forces (-grad) */
  int fkind;          /* -1: stale, ORC_F_SHORT or ORC_F_FULL */
  int fb_valid;
  /* candidate rows */
  int S;
  int64_t *cptr; cand_t *cand; int32_t *segst;
  int lists_valid;
  /* bounds */
  double *ell_lj, *ell_cu, *qmax;
  double bound_scale;  /* test knob: every bound multiplied by this (1 by default) */
  /* statistics */
  int64_t *nprop, *nacc, *nviol; uint64_t *hash;
  int64_t *knext;   /* per atom: first unused proposal of the last closing C' stream */
  int64_t n_rebuilds, n_zs_overflow, n_list_err;
  int64_t zs_regime[3];   /* accepted MRZ jumps by Z-sampler regime: eta < -1, -1 <= eta <= 0, eta > 0 */
  int64_t nev, evcap; int64_t *ev;
};

static void *xmalloc(size_t n) { void *p = calloc(1, n ? n : 1); return p; }

static double min_image(double d, double L) { return d - L * rint(d / L); }

static double pair_vec(const orc_sim *s, int i, int j, double d[3]) {
  for (int c = 0; c < 3; c++) d[c] = min_image(s->x[3 * i + c] - s->x[3 * j + c], s->L[c]);
  return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* displacement from the image x_j + n L of atom j to atom i */
static double pair_vec_n(const orc_sim *s, int i, int j, const int32_t n[3], double d[3]) {
  for (int c = 0; c < 3; c++) d[c] = (s->x[3 * i + c] - s->x[3 * j + c]) - (double)n[c] * s->L[c];
  return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Images of j that can lie within `cut` of i: the nearest image m plus, along
 * every edge shorter than 2 cut, the neighbouring images m - 1 and m + 1
 * (edges are longer than cut, so images two or more edges away from the
 * nearest are farther than cut). *nimg receives their count (1 ... 27); n
 * receives the lattice vectors and code the offset numbers (s+1) + 3 (s+1) + 9 (s+1),
 * in increasing order of code. */
static void images_within(const orc_sim *s, int i, int j, double cut, int *nimg, int32_t n[27][3],
                          int32_t code[27]) {
  int32_t m[3], lo[3], hi[3];
  for (int c = 0; c < 3; c++) {
    m[c] = (int32_t)rint((s->x[3 * i + c] - s->x[3 * j + c]) / s->L[c]);
    lo[c] = s->L[c] < 2.0 * cut ? -1 : 0;
    hi[c] = -lo[c];
  }
  int q = 0;
  for (int sz = lo[2]; sz <= hi[2]; sz++)
    for (int sy = lo[1]; sy <= hi[1]; sy++)
      for (int sx = lo[0]; sx <= hi[0]; sx++) {
        n[q][0] = m[0] + sx; n[q][1] = m[1] + sy; n[q][2] = m[2] + sz;
        code[q] = (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1);
        q++;
      }
  *nimg = q;
}

static int excluded(const orc_sim *s, int i, int j) {
  if (!s->xptr) return 0;
  for (int e = s->xptr[i]; e < s->xptr[i + 1]; e++)
    if (s->xj[e] == j) return 1;
  return 0;
}

/* ---------------------------------------------------------------- bounds */
/* Analytic bounds on |F_ij| (Sec. 3.1 end, Sec. 3.1.1 ring technique).
 * For r >= r_a >= r_s - w, |U| and |U'| of both LJ (r_a >= 1.25 sigma) and DSF
 * are non-increasing, so sup |(1-chi) U' - chi' U| <= |U'(r_a)| + max|chi'| |U(r_a)|
 * with max|chi'| = 15/(8w); the chi' term vanishes when r_a >= r_s. Ring k holds
 * candidates whose build-time distance is in [e_k, e_k + ring_width), e_k =
 * r_s - w - skin + k*ring_width; their current distance is at least e_k - skin. */
static double ring_ra(const orc_sim *s, int k) {
  double ek = (s->rlo - s->skin) + k * s->rw;
  double ra = ek - s->skin;
  return ra > s->rlo ? ra : s->rlo;
}

static void compute_bounds(orc_sim *s) {
  int nt = s->nt, nr = s->nr;
  for (int a = 0; a < nt; a++)
    for (int b = 0; b < nt; b++)
      for (int k = 0; k < nr; k++) {
        double ra = ring_ra(s, k);
        double Ul, dUl, Uc, dUc;
        double lj = 0.0, cu = 0.0;
        if (ra < s->rc) {
          lj_terms(ra, s->eps[a * nt + b], s->sig[a * nt + b], s->rc, &Ul, &dUl);
          dsf_terms(ra, 1.0, s->ke_c, s->alpha, s->rc, &Uc, &dUc);
          lj = fabs(dUl);
          cu = fabs(dUc);
          if (ra < s->rs) {
            lj += 15.0 / (8.0 * s->w) * fabs(Ul);
            cu += 15.0 / (8.0 * s->w) * fabs(Uc);
          }
        }
        s->ell_lj[(a * nt + b) * nr + k] = lj;
        s->ell_cu[(a * nt + b) * nr + k] = cu;
      }
  for (int t = 0; t < nt; t++) s->qmax[t] = 0.0;
  for (int i = 0; i < s->n; i++)
    if (fabs(s->q[i]) > s->qmax[s->type[i]]) s->qmax[s->type[i]] = fabs(s->q[i]);
}

/* bound of candidates of atom i in segment sg (class = type of j, ring) for
 * one jump component: 0 the LJ long part, 1 the Coulomb long part, 2 both
 * (their sum bounds the gradient of the whole long part) */
static double seg_bound(const orc_sim *s, int i, int sg, int coulomb) {
  int b = sg / s->nr, k = sg % s->nr, a = s->type[i];
  int idx = (a * s->nt + b) * s->nr + k;
  double lj = s->ell_lj[idx], cu = (fabs(s->q[i]) * s->qmax[b]) * s->ell_cu[idx];
  double ell = coulomb == 2 ? lj + cu : (coulomb ? cu : lj);
  return s->bound_scale == 1.0 ? ell : ell * s->bound_scale;
}

/* thinning is exact for any valid bound: larger bounds only add rejected
 * proposals (Sec. 2.4); tests use this to check that the law is unchanged */
void orc_set_bound_scale(orc_sim *s, double scale) { s->bound_scale = scale; }

/* ----------------------------------------------------------------- lists */
static int cand_cmp(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (a->seg != b->seg) return a->seg < b->seg ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  if (a->img != b->img) return a->img < b->img ? -1 : 1;
  return 0;
}

/* Candidate rows (Remark of Sec. 3.1.1): for each i, every image of every
 * j != i, not excluded, with r_s - w - skin <= r < r_c + skin at the build
 * positions, keyed by (type of j, ring) and sorted by (segment, j, image).
 * An exclusion removes every image of the pair. */
void orc_build_lists(orc_sim *s) {
  int n = s->n;
  int64_t total = 0;
  double rin = s->rlo - s->skin, rout = s->rc + s->skin;
  int nimg;
  int32_t nv[27][3], code[27];
  /* count */
  for (int i = 0; i < n; i++) {
    int64_t c = 0;
    for (int j = 0; j < n; j++) {
      if (j == i || excluded(s, i, j)) continue;
      images_within(s, i, j, rout, &nimg, nv, code);
      for (int q = 0; q < nimg; q++) {
        double d[3], r = pair_vec_n(s, i, j, nv[q], d);
        if (r >= rin && r < rout) c++;
      }
    }
    s->cptr[i + 1] = s->cptr[i] + c;
    total += c;
  }
  free(s->cand);
  s->cand = (cand_t *)xmalloc(sizeof(cand_t) * (size_t)total);
  for (int i = 0; i < n; i++) {
    int64_t p = s->cptr[i];
    for (int j = 0; j < n; j++) {
      if (j == i || excluded(s, i, j)) continue;
      images_within(s, i, j, rout, &nimg, nv, code);
      for (int q = 0; q < nimg; q++) {
        double d[3], r = pair_vec_n(s, i, j, nv[q], d);
        if (!(r >= rin && r < rout)) continue;
        int k = (int)floor((r - rin) / s->rw);
        if (k < 0) k = 0;
        if (k > s->nr - 1) k = s->nr - 1;
        s->cand[p].seg = s->type[j] * s->nr + k;
        s->cand[p].j = j;
        s->cand[p].img = code[q];
        for (int c = 0; c < 3; c++) s->cand[p].n[c] = nv[q][c];
        p++;
      }
    }
    qsort(s->cand + s->cptr[i], (size_t)(s->cptr[i + 1] - s->cptr[i]), sizeof(cand_t), cand_cmp);
    /* segment starts, relative to the row start */
    int64_t len = s->cptr[i + 1] - s->cptr[i];
    int64_t e = 0;
    for (int sg = 0; sg <= s->S; sg++) {
      while (e < len && s->cand[s->cptr[i] + e].seg < sg) e++;
      s->segst[(int64_t)i * (s->S + 1) + sg] = (int32_t)e;
    }
  }
  memcpy(s->xref, s->x, sizeof(double) * 3 * (size_t)n);
  s->steps_since_build = 0;
  s->lists_valid = 1;
}

/* Rebuild when some atom moved more than skin/2 since the last build
 * (or on the fixed period; then a larger displacement is a list error). */
static void maybe_rebuild(orc_sim *s) {
  double maxd2 = 0.0;
  for (int i = 0; i < s->n; i++) {
    double d2 = 0.0;
    for (int c = 0; c < 3; c++) {
      double d = s->x[3 * i + c] - s->xref[3 * i + c];
      d2 += d * d;
    }
    if (d2 > maxd2) maxd2 = d2;
  }
  double half = 0.5 * s->skin;
  int exceed = maxd2 > half * half;
  s->steps_since_build++;
  if (s->rebuild_every > 0) {
    if (s->steps_since_build >= s->rebuild_every) {
      orc_build_lists(s); s->n_rebuilds++;
    } else if (exceed) {
      s->n_list_err++;
    }
  } else if (exceed) {
    orc_build_lists(s); s->n_rebuilds++;
  }
}

/* ---------------------------------------------------------------- forces */
/* Non-bonded forces by brute force over all pairs and all their periodic
 * images within r_c (every box edge exceeds r_c + skin, so an atom never
 * meets its own image). kind SHORT: U_short = chi U for r < r_s; kind FULL:
 * U for r < r_c. */
static void nb_forces(const orc_sim *s, int kind, double *f, double *pe_s, double *pe_l) {
  int n = s->n;
  memset(f, 0, sizeof(double) * 3 * (size_t)n);
  double es = 0.0, el = 0.0;
  int nimg;
  int32_t nv[27][3], code[27];
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++) {
      if (excluded(s, i, j)) continue;
      images_within(s, i, j, s->rc, &nimg, nv, code);
      for (int q = 0; q < nimg; q++) {
      double d[3], r = pair_vec_n(s, i, j, nv[q], d);
      if (r >= s->rc) continue;
      int a = s->type[i], b = s->type[j];
      double Ul, dUl, Uc, dUc, chi, dchi;
      lj_terms(r, s->eps[a * s->nt + b], s->sig[a * s->nt + b], s->rc, &Ul, &dUl);
      dsf_terms(r, s->q[i] * s->q[j], s->ke_c, s->alpha, s->rc, &Uc, &dUc);
      switch_terms(r, s->rs, s->w, &chi, &dchi);
      double U = Ul + Uc, dU = dUl + dUc;
      es += chi * U;
      el += (1.0 - chi) * U;
      double g;
      if (kind == ORC_F_SHORT) {
        if (r >= s->rs) continue;
        g = chi * dU + dchi * U;
      } else if (kind == ORC_F_LONG) {
        g = (1.0 - chi) * dU - dchi * U;
      } else {
        g = dU;
      }
      for (int c = 0; c < 3; c++) {
        double fc = -g * d[c] / r;
        f[3 * i + c] += fc;
        f[3 * j + c] -= fc;
      }
      }
    }
  if (pe_s) *pe_s = es;
  if (pe_l) *pe_l = el;
}

/* Harmonic bonds (k/2)(b-b0)^2 and angles (k/2)(theta-theta0)^2 */
static double bonded_forces(const orc_sim *s, double *f) {
  memset(f, 0, sizeof(double) * 3 * (size_t)s->n);
  double e = 0.0;
  for (int t = 0; t < s->nb; t++) {
    int i = s->bij[2 * t], j = s->bij[2 * t + 1];
    double d[3], b = pair_vec(s, i, j, d);
    double db = b - s->br0[t];
    e += 0.5 * s->bk[t] * db * db;
    for (int c = 0; c < 3; c++) {
      double fc = -s->bk[t] * db * d[c] / b;
      f[3 * i + c] += fc;
      f[3 * j + c] -= fc;
    }
  }
  for (int t = 0; t < s->na; t++) {
    int i = s->aijk[3 * t], j = s->aijk[3 * t + 1], k = s->aijk[3 * t + 2];
    double u[3], w[3];
    double ru = pair_vec(s, i, j, u), rw = pair_vec(s, k, j, w);
    double cs = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / (ru * rw);
    if (cs > 1.0) cs = 1.0;
    if (cs < -1.0) cs = -1.0;
    double th = acos(cs), sn = sqrt(1.0 - cs * cs);
    double dth = th - s->at0[t];
    e += 0.5 * s->ak[t] * dth * dth;
    double dUdth = s->ak[t] * dth;
    /* d theta / d x_i = -(1/sin) d cos / d x_i ; d cos/d x_i = w/(ru rw) - cos u/ru^2 */
    for (int c = 0; c < 3; c++) {
      double dci = w[c] / (ru * rw) - cs * u[c] / (ru * ru);
      double dck = u[c] / (ru * rw) - cs * w[c] / (rw * rw);
      double fi = dUdth * dci / sn;  /* -dU/dx_i = dU/dth * dcos/dx_i / sin */
      double fk = dUdth * dck / sn;
      f[3 * i + c] += fi;
      f[3 * k + c] += fk;
      f[3 * j + c] -= fi + fk;
    }
  }
  return e;
}

/* ------------------------------------------------------------- Ewald */
/* Reciprocal-space part of the Ewald sum (Sec. 3.1: the paper's electrostatics
 * are Ewald direct space plus a reciprocal part), written out plainly: for
 * every lattice vector n with 0 < |n|^2 <= kmax^2, k = 2 pi (n_x/L_x, n_y/L_y,
 * n_z/L_z) and the structure factor S(k) = sum_j q_j exp(i k.x_j),
 *   E_k = (2 pi k_e / V) sum_k exp(-|k|^2 / (4 alpha^2)) / |k|^2 |S(k)|^2,
 * whose gradient gives the force on atom i
 *   f_i = (4 pi k_e q_i / V) sum_k exp(-|k|^2/(4 alpha^2)) / |k|^2 k (Re S sin(k.x_i) - Im S cos(k.x_i)).
 * The self term E_self = -k_e alpha / sqrt(pi) sum_i q_i^2 removes each
 * charge's interaction with its own screening cloud, and the excluded pairs,
 * whose real-space term is left out, lose their reciprocal-space
 * interaction by E_excl = -k_e q_i q_j erf(alpha r) / r (each pair once).
 * The real-space part is the damped shifted-force term with the same alpha.
 * Returns E_k + E_self + E_excl; f (may be NULL) receives the forces. */
static double spme_sum(const orc_sim *s, double *f);

static double recip_part(const orc_sim *s, double *f) {
  int n = s->n, K = s->kmax;
  double V = s->L[0] * s->L[1] * s->L[2], a = s->alpha, ke = s->ke_c;
  if (f) memset(f, 0, sizeof(double) * 3 * (size_t)n);
  double ek = 0.0;
  if (s->coul_kind == ORC_COUL_SPME) {
    ek = spme_sum(s, f);
    K = 0;   /* no plain sum */
  }
  for (int nx = -K; nx <= K; nx++)
    for (int ny = -K; ny <= K; ny++)
      for (int nz = -K; nz <= K; nz++) {
        int n2 = nx * nx + ny * ny + nz * nz;
        if (n2 == 0 || n2 > K * K) continue;
        double k[3] = {2.0 * PI * nx / s->L[0], 2.0 * PI * ny / s->L[1], 2.0 * PI * nz / s->L[2]};
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double w = exp(-k2 / (4.0 * a * a)) / k2;
        double sre = 0.0, sim = 0.0;
        for (int j = 0; j < n; j++) {
          double ph = k[0] * s->x[3 * j] + k[1] * s->x[3 * j + 1] + k[2] * s->x[3 * j + 2];
          sre += s->q[j] * cos(ph);
          sim += s->q[j] * sin(ph);
        }
        ek += w * (sre * sre + sim * sim);
        if (f)
          for (int i = 0; i < n; i++) {
            double ph = k[0] * s->x[3 * i] + k[1] * s->x[3 * i + 1] + k[2] * s->x[3 * i + 2];
            double c = 4.0 * PI * ke * s->q[i] / V * w * (sre * sin(ph) - sim * cos(ph));
            for (int q = 0; q < 3; q++) f[3 * i + q] += c * k[q];
          }
      }
  if (s->coul_kind != ORC_COUL_SPME) ek *= 2.0 * PI * ke / V;
  double eself = 0.0;
  for (int i = 0; i < n; i++) eself += s->q[i] * s->q[i];
  eself *= -ke * a / sqrt(PI);
  double eexcl = 0.0;
#if ORC_PLANT == 7   /* planted mistake: no excluded-pair correction (energy and forces alike) */
  if (0)
#else
  if (s->xptr)
#endif
    for (int i = 0; i < n; i++)
      for (int e = s->xptr[i]; e < s->xptr[i + 1]; e++) {
        int j = s->xj[e];
        if (j <= i) continue;
        double d[3], r = pair_vec(s, i, j, d);
        double qq = ke * s->q[i] * s->q[j];
        eexcl -= qq * erf(a * r) / r;
        if (f) {
          /* dE/dr of -qq erf(a r)/r, then f_i = -dE/dr d/r */
          double dEdr = -qq * (2.0 * a / sqrt(PI) * exp(-a * a * r * r) / r - erf(a * r) / (r * r));
          for (int q = 0; q < 3; q++) {
            double fc = -dEdr * d[q] / r;
            f[3 * i + q] += fc;
            f[3 * j + q] -= fc;
          }
        }
      }
  return ek + eself + eexcl;
}

/* Smooth particle-mesh Ewald (Essmann et al., J. Chem. Phys. 103, 8577
 * (1995)), the reciprocal sum the paper's Tinker runs use. Charges are
 * spread on a K1 x K2 x K3 grid with cardinal B-splines of order p,
 *   Q(k) = sum_i q_i M_p(u_i1 - k1) M_p(u_i2 - k2) M_p(u_i3 - k3),  u_id = K_d x_id / L_d
 * (periodically), and with F(m) = sum_k Q(k) exp(2 pi i m.k / K) the energy is
 *   E = (k_e / (2 pi V)) sum_{m != 0} exp(-pi^2 |m~|^2 / alpha^2) / |m~|^2 B(m) |F(m)|^2,
 * m~_d = m'_d / L_d with m'_d the index centred on zero, B(m) = prod_d |b_d(m_d)|^2,
 *   1 / b_d(m) = sum_{k=0}^{p-2} M_p(k + 1) exp(2 pi i m k / K_d)   (up to a phase).
 * With Psi(k) = sum_m G(m) conj(F(m)) exp(2 pi i m.k / K), G the factor of
 * |F|^2 above, the force is
 *   f_id = -2 q_i (K_d / L_d) sum_k Psi(k) M_p'(u_id - k_d) prod_{d' != d} M_p(u_id' - k_d').
 * Written out plainly: the B-splines by their recursion, the transforms as
 * separable discrete Fourier sums. Returns E; f (may be NULL) gets the forces. */
static double bspl(int p, double u) {
  if (u <= 0.0 || u >= p) return 0.0;
  if (p == 2) return 1.0 - fabs(u - 1.0);
  return (u * bspl(p - 1, u) + (p - u) * bspl(p - 1, u - 1.0)) / (p - 1);
}
static double dbspl(int p, double u) { return bspl(p - 1, u) - bspl(p - 1, u - 1.0); }

/* in-place discrete Fourier sum with exp(+2 pi i m k / K) along one axis of a
 * K0 x K1 x K2 complex grid (re, im separate) */
static void dft_axis(double *re, double *im, const int *K, int axis) {
  int Ka = K[axis];
  int st = axis == 0 ? K[1] * K[2] : (axis == 1 ? K[2] : 1);
  double *tr = (double *)xmalloc(sizeof(double) * Ka), *ti = (double *)xmalloc(sizeof(double) * Ka);
  for (int a = 0; a < K[0]; a++)
    for (int b = 0; b < K[1]; b++)
      for (int c = 0; c < K[2]; c++) {
        int idx[3] = {a, b, c};
        if (idx[axis] != 0) continue;   /* one line per start point */
        int base = (a * K[1] + b) * K[2] + c;
        for (int m = 0; m < Ka; m++) {
          double sr = 0.0, si = 0.0;
          for (int k = 0; k < Ka; k++) {
            double ph = 2.0 * PI * (double)((long)m * k % Ka) / Ka;
            double xr = re[base + k * st], xi = im[base + k * st];
            sr += xr * cos(ph) - xi * sin(ph);
            si += xr * sin(ph) + xi * cos(ph);
          }
          tr[m] = sr; ti[m] = si;
        }
        for (int m = 0; m < Ka; m++) { re[base + m * st] = tr[m]; im[base + m * st] = ti[m]; }
      }
  free(tr); free(ti);
}

static double spme_sum(const orc_sim *s, double *f) {
  const int *K = s->pme_K, p = s->pme_p, n = s->n;
  const int NG = K[0] * K[1] * K[2];
  const double V = s->L[0] * s->L[1] * s->L[2], a = s->alpha, ke = s->ke_c;
  double *qr = (double *)xmalloc(sizeof(double) * (size_t)NG), *qi = (double *)xmalloc(sizeof(double) * (size_t)NG);
  /* spread */
  for (int i = 0; i < n; i++) {
    double u[3]; long k0[3];
    for (int d = 0; d < 3; d++) { u[d] = K[d] * s->x[3 * i + d] / s->L[d]; k0[d] = (long)floor(u[d]); }
    for (int j0 = 0; j0 < p; j0++)
      for (int j1 = 0; j1 < p; j1++)
        for (int j2 = 0; j2 < p; j2++) {
          long kk[3] = {k0[0] - j0, k0[1] - j1, k0[2] - j2};
          double w = s->q[i];
          int g[3];
          for (int d = 0; d < 3; d++) {
            w *= bspl(p, u[d] - (double)kk[d]);
            g[d] = (int)(((kk[d] % K[d]) + K[d]) % K[d]);
          }
          qr[(g[0] * K[1] + g[1]) * K[2] + g[2]] += w;
        }
  }
  for (int d = 0; d < 3; d++) dft_axis(qr, qi, K, d);
  /* influence function and energy; the grid then holds G conj(F) */
  double e = 0.0;
  for (int m0 = 0; m0 < K[0]; m0++)
    for (int m1 = 0; m1 < K[1]; m1++)
      for (int m2 = 0; m2 < K[2]; m2++) {
        int m[3] = {m0, m1, m2}, idx = (m0 * K[1] + m1) * K[2] + m2;
        double G = 0.0;
        if (m0 || m1 || m2) {
          double mm = 0.0, B = 1.0;
          for (int d = 0; d < 3; d++) {
            int mc = m[d] <= K[d] / 2 ? m[d] : m[d] - K[d];
            mm += ((double)mc / s->L[d]) * ((double)mc / s->L[d]);
            double br = 0.0, bi = 0.0;
            for (int k = 0; k <= p - 2; k++) {
              double ph = 2.0 * PI * (double)((long)m[d] * k % K[d]) / K[d];
              br += bspl(p, k + 1.0) * cos(ph);
              bi += bspl(p, k + 1.0) * sin(ph);
            }
#if ORC_PLANT == 8   /* planted mistake: no B-spline correction B(m) in the influence function */
            (void)br; (void)bi;
#else
            B /= br * br + bi * bi;
#endif
          }
          G = ke / (2.0 * PI * V) * exp(-PI * PI * mm / (a * a)) / mm * B;
        }
        e += G * (qr[idx] * qr[idx] + qi[idx] * qi[idx]);
        qr[idx] *= G;
        qi[idx] *= -G;
      }
  if (f) {
    for (int d = 0; d < 3; d++) dft_axis(qr, qi, K, d);   /* qr = Psi */
    for (int i = 0; i < n; i++) {
      double u[3]; long k0[3];
      for (int d = 0; d < 3; d++) { u[d] = K[d] * s->x[3 * i + d] / s->L[d]; k0[d] = (long)floor(u[d]); }
      double fi[3] = {0.0, 0.0, 0.0};
      for (int j0 = 0; j0 < p; j0++)
        for (int j1 = 0; j1 < p; j1++)
          for (int j2 = 0; j2 < p; j2++) {
            long kk[3] = {k0[0] - j0, k0[1] - j1, k0[2] - j2};
            double M[3], dM[3];
            int g[3];
            for (int d = 0; d < 3; d++) {
              M[d] = bspl(p, u[d] - (double)kk[d]);
              dM[d] = dbspl(p, u[d] - (double)kk[d]);
              g[d] = (int)(((kk[d] % K[d]) + K[d]) % K[d]);
            }
            double psi = qr[(g[0] * K[1] + g[1]) * K[2] + g[2]];
            fi[0] += psi * dM[0] * M[1] * M[2];
#if ORC_PLANT == 9   /* planted mistake: the y force from the B-spline values instead of their derivative */
            fi[1] += psi * M[0] * M[1] * M[2];
#else
            fi[1] += psi * M[0] * dM[1] * M[2];
#endif
            fi[2] += psi * M[0] * M[1] * dM[2];
          }
      for (int d = 0; d < 3; d++) f[3 * i + d] = -2.0 * s->q[i] * (K[d] / s->L[d]) * fi[d];
    }
  }
  free(qr); free(qi);
  return e;
}

static int has_recip(const orc_sim *s) { return s->coul_kind == ORC_COUL_EWALD || s->coul_kind == ORC_COUL_SPME; }

static void ensure_recip(orc_sim *s) {
  if (!has_recip(s) || s->frec_valid) return;
  recip_part(s, s->frec);
  s->frec_valid = 1;
}

static void ensure_forces(orc_sim *s, int kind) {
  if (s->fkind != kind) {
    nb_forces(s, kind, s->fnb, NULL, NULL);
    s->fkind = kind;
  }
  if (!s->fb_valid) {
    bonded_forces(s, s->fb);
    s->fb_valid = 1;
  }
}

static void positions_moved(orc_sim *s) { s->fkind = -1; s->fb_valid = 0; s->frec_valid = 0; }

/* Long-range gradient F_ij = grad_{x_i} (1 - chi) U_ij (Sec. 3.1, Sec. 3.2)
 * for the candidate image (j, n); coulomb selects the DSF part, otherwise the
 * LJ part. Zero when r <= r_s - w or r >= r_c. */
static double long_grad(const orc_sim *s, int i, const cand_t *cj, int coulomb, double F[3]) {
  const int j = cj->j;
  double d[3], r = pair_vec_n(s, i, j, cj->n, d);
  int a = s->type[i], b = s->type[j];
  double U, dU, chi, dchi;
  if (coulomb == 1) {
    dsf_terms(r, s->q[i] * s->q[j], s->ke_c, s->alpha, s->rc, &U, &dU);
  } else if (coulomb == 0) {
    lj_terms(r, s->eps[a * s->nt + b], s->sig[a * s->nt + b], s->rc, &U, &dU);
  } else {   /* both parts: the long part of the whole pair potential */
    double Uc, dUc;
    lj_terms(r, s->eps[a * s->nt + b], s->sig[a * s->nt + b], s->rc, &U, &dU);
    dsf_terms(r, s->q[i] * s->q[j], s->ke_c, s->alpha, s->rc, &Uc, &dUc);
#if ORC_PLANT == 5   /* planted mistake: the BOUNCE gradient keeps the LJ part only */
    Uc = 0.0; dUc = 0.0;
#endif
    U += Uc;
    dU += dUc;
  }
  switch_terms(r, s->rs, s->w, &chi, &dchi);
  double g = (1.0 - chi) * dU - dchi * U;
  for (int c = 0; c < 3; c++) F[c] = g * d[c] / r;
  return F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
}

/* ------------------------------------------------------------ event log */
/* Per-atom fingerprint of the accepted jumps (not part of the method): each
 * event (step, phase, partner) is folded in with one multiply-xorshift. */
uint64_t orc_event_mix(uint64_t h, int64_t step, int32_t phase, int32_t j) {
  uint64_t key = (uint64_t)step * 0x9E3779B97F4A7C15ULL + (uint64_t)(uint32_t)phase * 0xC2B2AE3D27D4EB4FULL +
                 (uint64_t)(uint32_t)j;
  h = (h ^ key) * 0xFF51AFD7ED558CCDULL;
  return h ^ (h >> 29);
}

static uint64_t fnv1a_bytes(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t q = 0; q < n; q++) {
    h ^= (uint64_t)b[q];
    h *= 0x100000001b3ULL;
  }
  return h;
}

static void log_event(orc_sim *s, int32_t phase, int i, int j, int64_t k) {
  s->hash[i] = orc_event_mix(s->hash[i], s->step, phase, j);
  s->nacc[i]++;
  if (!s->log_events) return;
  if (s->nev == s->evcap) {
    s->evcap = s->evcap ? 2 * s->evcap : 1024;
    s->ev = (int64_t *)realloc(s->ev, sizeof(int64_t) * 5 * (size_t)s->evcap);
  }
  int64_t *e = s->ev + 5 * s->nev++;
  e[0] = s->step; e[1] = phase; e[2] = i; e[3] = j; e[4] = k;
}

/* Segment tables of atom i for one jump component: counts n_s, bounds l_s,
 * cumulative weights cumW_s = sum_{q<=s} n_q l_q and cumulative counts of the
 * segments with a nonzero bound cumN_s (the candidates whose rate can be > 0). */
typedef struct {
  int S;
  int64_t n[64], st[64];
  double ell[64], cumW[64], cumN[64];
  double W, nf;
} segtab_t;

static void seg_table(const orc_sim *s, int i, int coulomb, segtab_t *T) {
  const int32_t *st = s->segst + (int64_t)i * (s->S + 1);
  T->S = s->S;
  double cw = 0.0, cn = 0.0;
  for (int q = 0; q < s->S; q++) {
    T->st[q] = st[q];
    T->n[q] = st[q + 1] - st[q];
    T->ell[q] = seg_bound(s, i, q, coulomb);
    cw += (double)T->n[q] * T->ell[q];
    if (T->ell[q] > 0.0) cn += (double)T->n[q];
    T->cumW[q] = cw;
    T->cumN[q] = cn;
  }
  T->W = cw;
  T->nf = cn;
}

/* Candidate drawn with probability proportional to the bound (ring technique,
 * Sec. 3.1.1: choose the ring/segment in proportion to N l, then j uniformly
 * inside it). u picks the segment; its residual inside the segment picks j. */
static int64_t pick_by_bound(const segtab_t *T, double u, int *seg) {
  double target = u * T->W;
  int s = -1, last = -1;
  for (int q = 0; q < T->S; q++) {
    if (T->n[q] > 0 && T->ell[q] > 0.0) last = q;
    if (target < T->cumW[q] && T->n[q] > 0 && T->ell[q] > 0.0) { s = q; break; }
  }
  if (s < 0) s = last;
  double below = s > 0 ? T->cumW[s - 1] : 0.0;
  int64_t idx = (int64_t)floor((target - below) / T->ell[s]);
  if (idx < 0) idx = 0;
  if (idx > T->n[s] - 1) idx = T->n[s] - 1;
  *seg = s;
  return T->st[s] + idx;
}

/* Candidate drawn uniformly among the candidates of segments with l > 0. */
static int64_t pick_uniform(const segtab_t *T, double u, int *seg) {
  double target = u * T->nf;
  int s = -1, last = -1;
  for (int q = 0; q < T->S; q++) {
    if (T->n[q] > 0 && T->ell[q] > 0.0) last = q;
    if (target < T->cumN[q] && T->n[q] > 0 && T->ell[q] > 0.0) { s = q; break; }
  }
  if (s < 0) s = last;
  double below = s > 0 ? T->cumN[s - 1] : 0.0;
  int64_t idx = (int64_t)floor(target - below);
  if (idx < 0) idx = 0;
  if (idx > T->n[s] - 1) idx = T->n[s] - 1;
  *seg = s;
  return T->st[s] + idx;
}

/* ------------------------------------------------------------- J step */
/* Step (J) with BPS jumps for the LJ long part (Sec. 3.2, Alg. 5), one
 * independent chain per atom (Sec. 3.1), in the exponential-clock form of
 * Alg. 2. The bound beta |v_i| l_s per candidate is constant over the half
 * step (|v_i| is preserved), so proposal k happens at (E_0 + ... + E_k)/Lambda.
 * Proposal k uses Philox block (step, i, phase, k): u0 -> E_k, u2 -> candidate,
 * u3 -> acceptance (u1 unused). In the BOUNCE scheme (Sec. 3: bounces on the
 * Coulomb part as well, in (J)) one chain covers the long part of the whole
 * pair potential: bounds l_LJ + l_Coulomb, F_ij the gradient of both. */
static void jstep_atom(orc_sim *s, int i, int32_t phase, double h) {
  double *v = s->v + 3 * i;
  const int comp = s->jc == ORC_JUMP_BOUNCE ? 2 : 0;
  segtab_t T;
  seg_table(s, i, comp, &T);
  double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double Lam = s->beta * vn * T.W;
  if (!(Lam > 0.0) || !isfinite(Lam)) return;
  double sumE = 0.0;
  for (int64_t k = 0; k < MAX_PROPOSALS; k++) {
    double u[4];
    draw4(s->seed, s->replica, s->step, i, (uint64_t)phase, k, u);
    sumE += -log(u[0]);
    if (sumE / Lam > h) break;
    int sg;
    int64_t pos = pick_by_bound(&T, u[2], &sg);
    const cand_t *cj = &s->cand[s->cptr[i] + pos];
    int j = cj->j;
    double F[3];
    double F2 = long_grad(s, i, cj, comp, F);
    s->nprop[i]++;
    double vF = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
    double p = (vF > 0.0 ? vF : 0.0) / (vn * T.ell[sg]);
    if (p > 1.0) s->nviol[i]++;
    if (p > 0.0 && u[3] <= p) {
      /* reflection R_ij (Sec. 3.2): v - 2 (v.F)/|F|^2 F */
      double c = 2.0 * vF / F2;
      for (int q = 0; q < 3; q++) v[q] -= c * F[q];
      log_event(s, phase, i, j, k);
    }
  }
}

/* ------------------------------------------------------------- C step */
/* Step (C) (Sec. 2.3, Alg. 1, Alg. 4): constant acceleration a_i between
 * jumps plus MRZ jumps for the Coulomb long part. The rate bound is local and
 * re-evaluated after each jump (Sec. 2.4): from a jump (or the start) at
 * time t_e with velocity v_e, v(t) = v_e + (t - t_e) a_i and
 *   B_v = sqrt(|v_e|^2 + tau^2 |a|^2 + 2 tau (v_e.a)_+),  tau = h - t_e
 * bounds |v(t)| up to the end of the half step (Alg. 4). Per-candidate bound
 *   adaptive eps:  c_j = beta B_v l_s + f,   f = sqrt(beta/(2 pi m_i))/eps0
 *   constant eps:  c_j = l_s (beta B_v + sqrt(beta/(2 pi m_i))/eps)
 *   BPS kernel:    c_j = beta B_v l_s
 * and Lambda = sum_j c_j. Proposal k (Philox block (step, i, phase, k)):
 * u0 -> E_k (time t_e + (E_first + ... + E_k)/Lambda), u1 -> which part of
 * c_j proposes (the beta B_v l part or the f part, adaptive only), u2 -> the
 * candidate (by bound, or uniform over candidates with l > 0), u3 ->
 * acceptance lambda_ij / c_j.
 * With the BPS kernel on the Coulomb long part (the bounces of Sec. 3.2 in
 * place of Eqs. (tauxsaut),(majvitesse), i.e. the eps -> infinity end of the
 * MRZ family, Sec. 2.2) the rate is beta (v.F_ij)_+ and an accepted jump
 * reflects v about the plane orthogonal to F_ij; the acceleration between
 * jumps and the bound B_v are those of the MRZ case.
 * The proposals come from the stream (rstep, rphase) starting at index k0;
 * the return value is the first index the chain did not use (the one after
 * the proposal past the end of the half step). Events keep the op's own
 * (step, phase) labels. */
static int64_t cstep_atom(orc_sim *s, int i, int32_t phase, double h, const double a[3], int64_t rstep,
                          int32_t rphase, int64_t k0) {
  double *v = s->v + 3 * i;
  segtab_t T;
  const int comp = s->jlj == ORC_JUMP_IN_C ? 2 : 1;   /* Coulomb long part, or LJ and Coulomb together */
  seg_table(s, i, comp, &T);
  double me = s->me[i], beta = s->beta, eps0 = s->eps0;
  int adaptive = (s->jc == ORC_JUMP_MRZ_ADAPTIVE);
  int bps = (s->jc == ORC_JUMP_BPS);
  double f = bps ? 0.0 : sqrt(beta / (2.0 * PI * me)) / eps0;
  double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
  double ve[3] = {v[0], v[1], v[2]};
  double te = 0.0;
  int64_t k = k0;
  int done = 0;
  while (!done) {
    /* epoch: bound from (t_e, v_e) */
    double tau = h - te;
    double vv = ve[0] * ve[0] + ve[1] * ve[1] + ve[2] * ve[2];
    double va = ve[0] * a[0] + ve[1] * a[1] + ve[2] * a[2];
    double Bv = sqrt(vv + tau * tau * aa + 2.0 * tau * (va > 0.0 ? va : 0.0));
    double bBv = beta * Bv;
    double Wb = bBv * T.W;
    double Lam = adaptive ? Wb + f * T.nf : (bps ? Wb : (bBv + f) * T.W);
    if (!(Lam > 0.0) || !isfinite(Lam)) {
      for (int q = 0; q < 3; q++) v[q] = ve[q] + tau * a[q];
      break;
    }
    double sumE = 0.0;
    for (;; k++) {
      if (k >= MAX_PROPOSALS) { done = 1; for (int q = 0; q < 3; q++) v[q] = ve[q] + tau * a[q]; break; }
      double u[4];
      draw4(s->seed, s->replica, rstep, i, (uint64_t)rphase, k, u);
      sumE += -log(u[0]);
      double tk = te + sumE / Lam;
      if (tk > h) {
        for (int q = 0; q < 3; q++) v[q] = ve[q] + tau * a[q];
        done = 1;
        k++;   /* this proposal's clock decided the end */
        break;
      }
      double vk[3];
      for (int q = 0; q < 3; q++) vk[q] = ve[q] + (tk - te) * a[q];
      int sg;
      int64_t pos;
      if (adaptive && !(u[1] * Lam < Wb)) pos = pick_uniform(&T, u[2], &sg);
      else pos = pick_by_bound(&T, u[2], &sg);
      const cand_t *cj = &s->cand[s->cptr[i] + pos];
      int j = cj->j;
      double F[3];
#if ORC_PLANT == 10   /* planted mistake: LJ in C bounded for both parts, but jumping on the Coulomb one */
      double F2 = long_grad(s, i, cj, 1, F);
#else
      double F2 = long_grad(s, i, cj, comp, F);
#endif
      s->nprop[i]++;
      double ell = T.ell[sg];
      double c = adaptive ? bBv * ell + f : (bps ? bBv * ell : ell * (bBv + f));
      double lam = 0.0, eta = 0.0;
      double vF = vk[0] * F[0] + vk[1] * F[1] + vk[2] * F[2];
      if (bps) {
        lam = vF > 0.0 ? beta * vF : 0.0;
        double p = lam / c;
        if (p > 1.0) s->nviol[i]++;
        if (p > 0.0 && u[3] <= p) {
          double cr = 2.0 * vF / F2;   /* reflection R_ij at the jump time */
          for (int q = 0; q < 3; q++) ve[q] = vk[q] - cr * F[q];
          te = tk;
          log_event(s, phase, i, j, k);
          k++;
          break; /* new epoch */
        }
        continue;
      }
      if (F2 > 0.0) {
        if (adaptive) {
          /* eps = eps0 |F|: lambda = sqrt(beta/m)/eps0 Theta(eps0 sqrt(beta m) v.F) */
          eta = eps0 * sqrt(beta * me) * vF;
          lam = sqrt(beta / me) / eps0 * orc_theta(eta);
        } else {
          double Fn = sqrt(F2);
          eta = eps0 * sqrt(beta * me) * vF / Fn;
          lam = sqrt(beta) / (eps0 * sqrt(me)) * Fn * orc_theta(eta);
        }
      }
      double p = lam / c;
      if (p > 1.0) s->nviol[i]++;
      if (p > 0.0 && u[3] <= p) {
        int32_t it;
        double Z = orc_zsample(eta, s->seed, s->replica, rstep, i, rphase, k, &it);
        if (it < 0) s->n_zs_overflow++;
        s->zs_regime[eta < -1.0 ? 0 : (eta <= 0.0 ? 1 : 2)]++;
        /* Eq. (majvitesse) restricted to atom i (Sec. 3.1) */
        double coef;
        if (adaptive) coef = 2.0 * eps0 * Z / ((1.0 + eps0 * eps0 * F2) * sqrt(beta * me));
        else coef = 2.0 * eps0 * Z / ((1.0 + eps0 * eps0) * sqrt(beta * me) * sqrt(F2));
        for (int q = 0; q < 3; q++) ve[q] = vk[q] - coef * F[q];
        te = tk;
        log_event(s, phase, i, j, k);
        k++;
        break; /* new epoch */
      }
    }
  }
  return k;
}

/* ------------------------------------------------------------- B, A, O */
static void kick(orc_sim *s, double h, int with_nb, int with_b) {
  for (int i = 0; i < s->n; i++)
    for (int c = 0; c < 3; c++) {
      double fc = (with_nb ? s->fnb[3 * i + c] : 0.0) + (with_b ? s->fb[3 * i + c] : 0.0);
      s->v[3 * i + c] += h * fc / s->me[i];
    }
}

/* v += h f / m for a force array f */
static void kick_with(orc_sim *s, double h, const double *f) {
  for (int i = 0; i < s->n; i++)
    for (int c = 0; c < 3; c++) s->v[3 * i + c] += h * f[3 * i + c] / s->me[i];
}

static void drift(orc_sim *s, double h) {
  for (int i = 0; i < 3 * s->n; i++) s->x[i] += h * s->v[i];
  positions_moved(s);
}

/* (O): v <- e^{-gamma dt} v + sqrt((1 - e^{-2 gamma dt}) kT/m) G  (Sec. 2.3).
 * Normals by Box-Muller from one Philox block per atom. */
void orc_phase_o(orc_sim *s, double h, int32_t substep) {
  double c1 = exp(-s->gamma * h);
  double c2 = sqrt(1.0 - c1 * c1);
  uint64_t tag = (uint64_t)ORC_PH_O | ((uint64_t)(uint32_t)substep << 8);
  for (int i = 0; i < s->n; i++) {
    double u[4];
    draw4(s->seed, s->replica, s->step, i, tag, 0, u);
    double r1 = sqrt(-2.0 * log(u[0])), r2 = sqrt(-2.0 * log(u[2]));
    double g[3] = {r1 * cos(2.0 * PI * u[1]), r1 * sin(2.0 * PI * u[1]), r2 * cos(2.0 * PI * u[3])};
    double sd = sqrt(s->kT / s->me[i]);
    for (int c = 0; c < 3; c++) s->v[3 * i + c] = c1 * s->v[3 * i + c] + c2 * sd * g[c];
  }
}

void orc_phase_j(orc_sim *s, int32_t phase, double h) {
  if (!s->lists_valid) orc_build_lists(s);
  for (int i = 0; i < s->n; i++) jstep_atom(s, i, phase, h);
}

/* C for every atom. stream 0: own stream (step, phase) from index 0;
 * STREAM_SAVE: the same, and the first unused index is kept per atom;
 * STREAM_CONTINUE: the stream (step - 1, ORC_PH_C2) from the kept index.
 * a_kind 0: acceleration from short non-bonded + bonded, 1: short non-bonded */
#define STREAM_SAVE 1
#define STREAM_CONTINUE 2
/* a_kind 0: the acceleration is everything not jumped (short non-bonded,
 * bonded and, with Ewald electrostatics, reciprocal-space forces); 1: the
 * short non-bonded forces only (the RESPA schemes) */
static void phase_c(orc_sim *s, int32_t phase, double h, int a_kind, int stream) {
  if (!s->lists_valid) orc_build_lists(s);
  ensure_forces(s, ORC_F_SHORT);
#if ORC_PLANT == 6   /* planted mistake: the reciprocal forces are left out of the C' acceleration */
  const int rec = 0;
#else
  const int rec = a_kind == 0 && has_recip(s);
#endif
  if (rec) ensure_recip(s);
  for (int i = 0; i < s->n; i++) {
    double a[3];
    for (int c = 0; c < 3; c++) {
      double fc = s->fnb[3 * i + c] + (a_kind == 0 ? s->fb[3 * i + c] : 0.0) + (rec ? s->frec[3 * i + c] : 0.0);
      a[c] = fc / s->me[i];
    }
    if (stream == STREAM_CONTINUE) {
      cstep_atom(s, i, phase, h, a, s->step - 1, ORC_PH_C2, s->knext[i]);
    } else {
      const int64_t kend = cstep_atom(s, i, phase, h, a, s->step, phase, 0);
      if (stream == STREAM_SAVE) s->knext[i] = kend;
    }
  }
}

void orc_phase_c(orc_sim *s, int32_t phase, double h, int a_kind) { phase_c(s, phase, h, a_kind, 0); }

/* (C') or plain (B) depending on whether Coulomb jumps are on */
static void c_or_b(orc_sim *s, int32_t phase, double h, int a_kind, int stream) {
  if (s->jc != ORC_JUMP_NONE && s->jc != ORC_JUMP_BOUNCE) {
    phase_c(s, phase, h, a_kind, stream);
  } else {
    kick(s, h, 1, a_kind == 0);
    if (a_kind == 0 && has_recip(s)) { ensure_recip(s); kick_with(s, h, s->frec); }
  }
}

/* whether the scheme has (J) steps: LJ bounces, or the BOUNCE scheme */
static int has_j(const orc_sim *s) { return s->jlj == ORC_JUMP_BPS || s->jc == ORC_JUMP_BOUNCE; }

/* ------------------------------------------------------------- schemes */
/* BAOAB with full-range forces (Sec. 2.3 without J); with Ewald
 * electrostatics the reciprocal-space forces are part of every kick. */
int orc_step_baoab(orc_sim *s, int64_t n) {
  double h = 0.5 * s->dt;
  int ew = has_recip(s);
  ensure_forces(s, ORC_F_FULL);
  ensure_recip(s);
  for (int64_t it = 0; it < n; it++) {
    kick(s, h, 1, 1);
    if (ew) kick_with(s, h, s->frec);
    drift(s, h);
    orc_phase_o(s, s->dt, 0);
    drift(s, h);
    maybe_rebuild(s);
    ensure_forces(s, ORC_F_FULL);
    ensure_recip(s);
    kick(s, h, 1, 1);
    if (ew) kick_with(s, h, s->frec);
    s->step++;
  }
  return 0;
}

/* JUMP: B J A O A J B, or C' J' A O A J' C' (Sec. 2.3, Sec. 3.3); with
 * Ewald electrostatics the C' acceleration (or the B kick) also carries the
 * reciprocal-space forces, re-evaluated every step. The
 * closing C' of a step and the opening C' of the next act at the same
 * positions; the opening one draws its proposals from the closing one's
 * stream, from the proposal after the one that ended it. Those proposals
 * were never used, so they are fresh draws and the law is unchanged. */
int orc_step_jump(orc_sim *s, int64_t n) {
  double h = 0.5 * s->dt;
  if (!s->lists_valid) orc_build_lists(s);
  ensure_forces(s, ORC_F_SHORT);
  for (int64_t it = 0; it < n; it++) {
    c_or_b(s, ORC_PH_C1, h, 0, STREAM_CONTINUE);
    if (has_j(s)) orc_phase_j(s, ORC_PH_J1, h);
    drift(s, h);
    orc_phase_o(s, s->dt, 0);
    drift(s, h);
    maybe_rebuild(s);
    ensure_forces(s, ORC_F_SHORT);
    if (has_j(s)) orc_phase_j(s, ORC_PH_J2, h);
    c_or_b(s, ORC_PH_C2, h, 0, STREAM_SAVE);
    s->step++;
  }
  return 0;
}

/* The inner loop shared by JUMP-RESPA and BAOAB-RESPA (Sec. 2.3.2): m
 * steps B_b A O A B_b of length dt = 2h with the bonded forces only, the
 * bonded forces re-evaluated after each pair of drifts; the O draw of inner
 * step `sub` carries `sub` in its counter. */
static void respa_inner_steps(orc_sim *s, int m, double h) {
  for (int sub = 0; sub < m; sub++) {
#if ORC_PLANT == 1   /* planted mistake: the opening inner kick of the first inner step is dropped */
    if (sub > 0) kick(s, h, 0, 1);
#elif ORC_PLANT == 2 /* planted mistake: inner kicks last the outer half step m*h */
    kick(s, m * h, 0, 1);
#else
    kick(s, h, 0, 1);
#endif
    drift(s, h);
    orc_phase_o(s, s->dt, sub);
    drift(s, h);
#if ORC_PLANT == 3   /* planted mistake: the bonded forces are not re-evaluated after the drifts */
    if (sub == m - 1) bonded_forces(s, s->fb);
#else
    bonded_forces(s, s->fb);
#endif
    s->fb_valid = 1;
#if ORC_PLANT == 2
    kick(s, m * h, 0, 1);
#else
    kick(s, h, 0, 1);
#endif
  }
}

/* JUMP-RESPA (Sec. 2.3.2 and Sec. 3.3): bonded forces at the inner step dt,
 * short non-bonded forces and all jumps at the outer step n*dt. Inner steps
 * are B_b A O A B_b; the O draw carries the inner index. As in JUMP, the
 * opening C' continues the stream of the closing C' of the outer step before
 * (both act at the same positions). */
int orc_step_jump_respa(orc_sim *s, int64_t n_outer) {
  if (has_recip(s)) return -1;
  int m = s->respa_inner > 0 ? s->respa_inner : 1;
  double H = 0.5 * s->dt * m, h = 0.5 * s->dt;
  if (!s->lists_valid) orc_build_lists(s);
  ensure_forces(s, ORC_F_SHORT);
  for (int64_t it = 0; it < n_outer; it++) {
    c_or_b(s, ORC_PH_C1, H, 1, STREAM_CONTINUE);
    if (has_j(s)) orc_phase_j(s, ORC_PH_J1, H);
    respa_inner_steps(s, m, h);
    maybe_rebuild(s);
    ensure_forces(s, ORC_F_SHORT);
    if (has_j(s)) orc_phase_j(s, ORC_PH_J2, H);
    c_or_b(s, ORC_PH_C2, H, 1, STREAM_SAVE);
    s->step++;
  }
  return 0;
}

/* BAOAB-RESPA comparator: full-range non-bonded kick at the outer step. */
int orc_step_baoab_respa(orc_sim *s, int64_t n_outer) {
  if (has_recip(s)) return -1;
  int m = s->respa_inner > 0 ? s->respa_inner : 1;
  double H = 0.5 * s->dt * m, h = 0.5 * s->dt;
  ensure_forces(s, ORC_F_FULL);
  for (int64_t it = 0; it < n_outer; it++) {
    kick(s, H, 1, 0);
    respa_inner_steps(s, m, h);
    maybe_rebuild(s);
    ensure_forces(s, ORC_F_FULL);
    kick(s, H, 1, 0);
    s->step++;
  }
  return 0;
}

/* JUMP-RESPA1 (Sec. 2.3.2, Sec. 3.3, Table 2): three levels. Bonded forces
 * at the inner step dt (m inner steps per middle step), short non-bonded
 * forces and all jumps at the middle step m dt (the JUMP-RESPA step above,
 * with its C' streams continued from middle step to middle step), and the
 * Ewald reciprocal-space forces at the outer step p m dt, as kicks of half
 * an outer step around the p middle steps. */
int orc_step_jump_respa1(orc_sim *s, int64_t n_outer) {
  if (!has_recip(s)) return -1;
  int m = s->respa_inner > 0 ? s->respa_inner : 1, p = s->respa_outer > 0 ? s->respa_outer : 1;
  double h = 0.5 * s->dt, H = 0.5 * s->dt * m, HH = 0.5 * s->dt * m * p;
  if (!s->lists_valid) orc_build_lists(s);
  ensure_forces(s, ORC_F_SHORT);
  ensure_recip(s);
  for (int64_t it = 0; it < n_outer; it++) {
    kick_with(s, HH, s->frec);
    for (int q = 0; q < p; q++) {
      c_or_b(s, ORC_PH_C1, H, 1, STREAM_CONTINUE);
      if (has_j(s)) orc_phase_j(s, ORC_PH_J1, H);
      respa_inner_steps(s, m, h);
      maybe_rebuild(s);
      ensure_forces(s, ORC_F_SHORT);
      if (has_j(s)) orc_phase_j(s, ORC_PH_J2, H);
      c_or_b(s, ORC_PH_C2, H, 1, STREAM_SAVE);
      s->step++;
    }
    ensure_recip(s);
    kick_with(s, HH, s->frec);
  }
  return 0;
}

/* BAOAB-RESPA1 comparator (Sec. 2.3.2, Table 2): bonded forces at dt, the
 * short non-bonded forces chi U at m dt, the long real-space part (1 - chi) U
 * and the reciprocal-space forces at p m dt. */
int orc_step_baoab_respa1(orc_sim *s, int64_t n_outer) {
  if (!has_recip(s)) return -1;
  int m = s->respa_inner > 0 ? s->respa_inner : 1, p = s->respa_outer > 0 ? s->respa_outer : 1;
  double h = 0.5 * s->dt, H = 0.5 * s->dt * m, HH = 0.5 * s->dt * m * p;
  double *fl = (double *)xmalloc(sizeof(double) * 3 * (size_t)s->n);
  nb_forces(s, ORC_F_LONG, fl, NULL, NULL);
  ensure_recip(s);
  ensure_forces(s, ORC_F_SHORT);
  for (int64_t it = 0; it < n_outer; it++) {
    kick_with(s, HH, fl);
    kick_with(s, HH, s->frec);
    for (int q = 0; q < p; q++) {
      kick(s, H, 1, 0);
      respa_inner_steps(s, m, h);
      maybe_rebuild(s);
      ensure_forces(s, ORC_F_SHORT);
      kick(s, H, 1, 0);
      s->step++;
    }
    nb_forces(s, ORC_F_LONG, fl, NULL, NULL);
    ensure_recip(s);
    kick_with(s, HH, fl);
    kick_with(s, HH, s->frec);
  }
  free(fl);
  return 0;
}

/* ------------------------------------------------------------ create */
orc_sim *orc_create(const orc_system *sy, const orc_split *sp, const orc_params *pa,
                    char *err, int errlen) {
#define FAIL(msg) do { if (err) snprintf(err, (size_t)errlen, "%s", msg); orc_destroy(s); return NULL; } while (0)
  orc_sim *s = (orc_sim *)xmalloc(sizeof(orc_sim));
  int n = sy->n_atoms, nt = sy->n_types;
  s->n = n; s->nt = nt;
  if (n <= 0 || nt <= 0) FAIL("n_atoms and n_types must be positive");
  s->x = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  s->v = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  s->xref = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  s->fnb = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  s->fb = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  s->mass = (double *)xmalloc(sizeof(double) * (size_t)n);
  s->me = (double *)xmalloc(sizeof(double) * (size_t)n);
  s->q = (double *)xmalloc(sizeof(double) * (size_t)n);
  s->type = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  s->eps = (double *)xmalloc(sizeof(double) * (size_t)(nt * nt));
  s->sig = (double *)xmalloc(sizeof(double) * (size_t)(nt * nt));
  memcpy(s->x, sy->pos, sizeof(double) * 3 * (size_t)n);
  memcpy(s->v, sy->vel, sizeof(double) * 3 * (size_t)n);
  memcpy(s->mass, sy->mass, sizeof(double) * (size_t)n);
  for (int i = 0; i < n; i++) s->q[i] = sy->charge ? sy->charge[i] : 0.0;
  memcpy(s->type, sy->type, sizeof(int32_t) * (size_t)n);
  memcpy(s->eps, sy->lj_eps, sizeof(double) * (size_t)(nt * nt));
  memcpy(s->sig, sy->lj_sigma, sizeof(double) * (size_t)(nt * nt));
  for (int c = 0; c < 3; c++) s->L[c] = sy->box[c];
  s->nb = sy->n_bonds; s->na = sy->n_angles;
  s->bij = (int32_t *)xmalloc(sizeof(int32_t) * 2 * (size_t)s->nb);
  s->bk = (double *)xmalloc(sizeof(double) * (size_t)s->nb);
  s->br0 = (double *)xmalloc(sizeof(double) * (size_t)s->nb);
  if (s->nb) {
    memcpy(s->bij, sy->bond_ij, sizeof(int32_t) * 2 * (size_t)s->nb);
    memcpy(s->bk, sy->bond_k, sizeof(double) * (size_t)s->nb);
    memcpy(s->br0, sy->bond_r0, sizeof(double) * (size_t)s->nb);
  }
  s->aijk = (int32_t *)xmalloc(sizeof(int32_t) * 3 * (size_t)s->na);
  s->ak = (double *)xmalloc(sizeof(double) * (size_t)s->na);
  s->at0 = (double *)xmalloc(sizeof(double) * (size_t)s->na);
  if (s->na) {
    memcpy(s->aijk, sy->angle_ijk, sizeof(int32_t) * 3 * (size_t)s->na);
    memcpy(s->ak, sy->angle_k, sizeof(double) * (size_t)s->na);
    memcpy(s->at0, sy->angle_t0, sizeof(double) * (size_t)s->na);
  }
  if (sy->excl_ptr) {
    s->xptr = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    memcpy(s->xptr, sy->excl_ptr, sizeof(int32_t) * (size_t)(n + 1));
    s->xj = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)s->xptr[n]);
    memcpy(s->xj, sy->excl_j, sizeof(int32_t) * (size_t)s->xptr[n]);
  }
  s->ke_c = sy->coulomb_k; s->accel = sy->accel_factor; s->kB = sy->kB;
  for (int i = 0; i < n; i++) s->me[i] = s->mass[i] / s->accel;
  s->rs = sp->r_s; s->rc = sp->r_c; s->w = sp->switch_width; s->skin = sp->skin;
  s->alpha = sp->coulomb_alpha; s->nr = sp->n_rings > 0 ? sp->n_rings : 1;
  s->rw = sp->ring_width;
  s->rlo = s->rs - s->w;
  if (s->nr == 1) s->rw = (s->rc + s->skin) - (s->rlo - s->skin);
  if (!(s->w > 0.0) || !(s->rs <= s->rc) || s->skin < 0.0 || !(s->rw > 0.0)) FAIL("bad split");
  for (int c = 0; c < 3; c++)
    if (!(s->L[c] > s->rc + s->skin)) FAIL("every box edge must exceed r_c + skin");
  s->dt = pa->dt; s->gamma = pa->gamma; s->kT = pa->kT; s->beta = 1.0 / pa->kT;
  s->seed = pa->seed; s->replica = pa->replica;
  s->jlj = pa->jump_lj; s->jc = pa->jump_coul; s->eps0 = pa->eps;
  s->respa_inner = pa->respa_inner; s->rebuild_every = pa->rebuild_every;
  s->log_events = pa->log_events; s->respa_outer = pa->respa_outer;
  s->coul_kind = sp->coulomb_kind; s->kmax = sp->ewald_kmax;
  for (int d = 0; d < 3; d++) s->pme_K[d] = sp->pme_grid[d];
  s->pme_p = sp->pme_order;
  if (s->coul_kind != ORC_COUL_DSF && s->coul_kind != ORC_COUL_EWALD && s->coul_kind != ORC_COUL_SPME)
    FAIL("coulomb_kind: DSF, EWALD or SPME");
  if (s->coul_kind == ORC_COUL_EWALD && (s->kmax < 1 || !(s->alpha > 0.0))) FAIL("Ewald needs kmax >= 1 and alpha > 0");
  if (s->coul_kind == ORC_COUL_SPME &&
      (!(s->alpha > 0.0) || s->pme_p < 4 || s->pme_p > 8 || (s->pme_p & 1) || s->pme_K[0] < s->pme_p ||
       s->pme_K[1] < s->pme_p || s->pme_K[2] < s->pme_p))
    FAIL("SPME needs alpha > 0, an even order 4..8 and at least `order` grid points per edge");
  s->frec = (double *)xmalloc(sizeof(double) * 3 * (size_t)n);
  if (s->jlj != ORC_JUMP_NONE && s->jlj != ORC_JUMP_BPS && s->jlj != ORC_JUMP_IN_C) FAIL("LJ jumps: NONE, BPS or IN_C");
  if (s->jlj == ORC_JUMP_IN_C && s->jc != ORC_JUMP_BPS && s->jc != ORC_JUMP_MRZ_CONST && s->jc != ORC_JUMP_MRZ_ADAPTIVE)
    FAIL("LJ jumps in the C step need Coulomb jumps in the C step (BPS or MRZ)");
  if (s->jc != ORC_JUMP_NONE && s->jc != ORC_JUMP_BPS && s->jc != ORC_JUMP_MRZ_CONST &&
      s->jc != ORC_JUMP_MRZ_ADAPTIVE && s->jc != ORC_JUMP_BOUNCE)
    FAIL("Coulomb jumps: NONE, BPS, MRZ_CONST, MRZ_ADAPTIVE or BOUNCE");
  if ((s->jc == ORC_JUMP_MRZ_CONST || s->jc == ORC_JUMP_MRZ_ADAPTIVE) && !(s->eps0 > 0.0))
    FAIL("eps must be positive");
  /* the LJ bound needs |U|, |U'| non-increasing beyond r_s - w */
  for (int ab = 0; ab < nt * nt; ab++)
    if (s->eps[ab] != 0.0 && s->rlo < 1.25 * s->sig[ab]) FAIL("r_s - w must be >= 1.25 sigma");
  s->S = nt * s->nr;
  if (s->S > 64) FAIL("too many segments (n_types * n_rings > 64)");
  s->cptr = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
  s->segst = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n * (size_t)(s->S + 1));
  s->ell_lj = (double *)xmalloc(sizeof(double) * (size_t)(nt * nt * s->nr));
  s->ell_cu = (double *)xmalloc(sizeof(double) * (size_t)(nt * nt * s->nr));
  s->qmax = (double *)xmalloc(sizeof(double) * (size_t)nt);
  s->nprop = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  s->knext = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  s->nacc = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  s->nviol = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  s->hash = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)n);
  for (int i = 0; i < n; i++) s->hash[i] = 0xcbf29ce484222325ULL;
  compute_bounds(s);
  s->bound_scale = 1.0;
  s->fkind = -1;
  s->fb_valid = 0;
  s->lists_valid = 0;
  memcpy(s->xref, s->x, sizeof(double) * 3 * (size_t)n);
  return s;
#undef FAIL
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->xref); free(s->fnb); free(s->fb); free(s->mass);
  free(s->me); free(s->q); free(s->type); free(s->eps); free(s->sig); free(s->bij);
  free(s->bk); free(s->br0); free(s->aijk); free(s->ak); free(s->at0); free(s->xptr);
  free(s->xj); free(s->cptr); free(s->cand); free(s->segst); free(s->ell_lj);
  free(s->ell_cu); free(s->qmax); free(s->nprop); free(s->knext); free(s->nacc); free(s->nviol);
  free(s->hash); free(s->ev); free(s->frec); free(s);
}

/* ------------------------------------------------------------ accessors */
void orc_get_state(const orc_sim *s, double *pos, double *vel) {
  if (pos) memcpy(pos, s->x, sizeof(double) * 3 * (size_t)s->n);
  if (vel) memcpy(vel, s->v, sizeof(double) * 3 * (size_t)s->n);
}

void orc_set_state(orc_sim *s, const double *pos, const double *vel, int64_t step) {
  if (pos) { memcpy(s->x, pos, sizeof(double) * 3 * (size_t)s->n); positions_moved(s); s->lists_valid = 0; }
  if (vel) memcpy(s->v, vel, sizeof(double) * 3 * (size_t)s->n);
  if (step >= 0) s->step = step;
}

int64_t orc_step_index(const orc_sim *s) { return s->step; }
int64_t orc_n_rebuilds(const orc_sim *s) { return s->n_rebuilds; }
int64_t orc_n_zsampler_overflow(const orc_sim *s) { return s->n_zs_overflow; }
int64_t orc_n_list_errors(const orc_sim *s) { return s->n_list_err; }
void orc_zsampler_regimes(const orc_sim *s, int64_t out[3]) {
  for (int q = 0; q < 3; q++) out[q] = s->zs_regime[q];
}

void orc_atom_stats(const orc_sim *s, int64_t *nprop, int64_t *nacc, int64_t *nviol, uint64_t *hash) {
  size_t n = (size_t)s->n;
  if (nprop) memcpy(nprop, s->nprop, 8 * n);
  if (nacc) memcpy(nacc, s->nacc, 8 * n);
  if (nviol) memcpy(nviol, s->nviol, 8 * n);
  if (hash) memcpy(hash, s->hash, 8 * n);
}

/* run hash: FNV-1a over the per-atom hashes in atom order */
uint64_t orc_event_hash(const orc_sim *s) {
  uint64_t h = 0xcbf29ce484222325ULL;
  for (int i = 0; i < s->n; i++) h = fnv1a_bytes(h, &s->hash[i], 8);
  return h;
}

int64_t orc_n_events(const orc_sim *s) { return s->nev; }
void orc_get_events(const orc_sim *s, int64_t *buf) {
  memcpy(buf, s->ev, sizeof(int64_t) * 5 * (size_t)s->nev);
}

void orc_energies(const orc_sim *s, double out[7]) {
  double ke = 0.0;
  for (int i = 0; i < s->n; i++)
    for (int c = 0; c < 3; c++) ke += 0.5 * s->me[i] * s->v[3 * i + c] * s->v[3 * i + c];
  double *tmp = (double *)xmalloc(sizeof(double) * 3 * (size_t)s->n);
  double es, el;
  nb_forces(s, ORC_F_FULL, tmp, &es, &el);
  double eb = bonded_forces(s, tmp);
  free(tmp);
  double er = has_recip(s) ? recip_part(s, NULL) : 0.0;
  out[0] = ke;
  out[1] = 2.0 * ke / (3.0 * s->n * s->kB);
  out[2] = es; out[3] = el; out[4] = eb; out[5] = es + el + eb + er; out[6] = er;
}

void orc_accel(const orc_sim *s, int kind, double *acc) {
  double *f = (double *)xmalloc(sizeof(double) * 3 * (size_t)s->n);
  if (kind == ORC_F_BONDED) bonded_forces(s, f);
  else if (kind == ORC_F_RECIP) { if (has_recip(s)) recip_part(s, f); }
  else nb_forces(s, kind, f, NULL, NULL);
  for (int i = 0; i < s->n; i++)
    for (int c = 0; c < 3; c++) acc[3 * i + c] = f[3 * i + c] / s->me[i];
  free(f);
}

/* pair-count histogram of (ta, tb) pairs (unordered if ta == tb) with r < r_max */
void orc_rdf(const orc_sim *s, int ta, int tb, double r_max, int n_bins, double *hist) {
  for (int b = 0; b < n_bins; b++) hist[b] = 0.0;
  double dr = r_max / n_bins;
  for (int i = 0; i < s->n; i++)
    for (int j = i + 1; j < s->n; j++) {
      int a = s->type[i], b = s->type[j];
      if (!((a == ta && b == tb) || (a == tb && b == ta))) continue;
      double d[3], r = pair_vec(s, i, j, d);
      if (r >= r_max) continue;
#if ORC_PLANT == 4   /* planted mistake: bins rounded to the nearest edge */
      int bin = (int)(r / dr + 0.5);
#else
      int bin = (int)(r / dr);
#endif
      if (bin < n_bins) hist[bin] += 1.0;
    }
}

int32_t orc_n_segments(const orc_sim *s) { return s->S; }
int64_t orc_cand_count(const orc_sim *s, int32_t i) { return s->cptr[i + 1] - s->cptr[i]; }
void orc_cand_row(const orc_sim *s, int32_t i, int32_t *j, int32_t *n) {
  for (int64_t p = s->cptr[i]; p < s->cptr[i + 1]; p++) {
    j[p - s->cptr[i]] = s->cand[p].j;
    if (n)
      for (int c = 0; c < 3; c++) n[3 * (p - s->cptr[i]) + c] = s->cand[p].n[c];
  }
}
void orc_seg_start(const orc_sim *s, int32_t i, int32_t *starts) {
  memcpy(starts, s->segst + (int64_t)i * (s->S + 1), sizeof(int32_t) * (size_t)(s->S + 1));
}

/* unordered non-excluded pairs (i<j, each periodic image once) with r < rcut
 * at the current positions */
int64_t orc_pairs_within(const orc_sim *s, double rcut, int32_t *ij, int64_t cap) {
  int64_t c = 0;
  int nimg;
  int32_t nv[27][3], code[27];
  for (int i = 0; i < s->n; i++)
    for (int j = i + 1; j < s->n; j++) {
      if (excluded(s, i, j)) continue;
      images_within(s, i, j, rcut, &nimg, nv, code);
      for (int q = 0; q < nimg; q++) {
        double d[3], r = pair_vec_n(s, i, j, nv[q], d);
        if (r < rcut) {
          if (c < cap) { ij[2 * c] = i; ij[2 * c + 1] = j; }
          c++;
        }
      }
    }
  return c;
}

void orc_bounds(const orc_sim *s, double *ell_lj, double *ell_coul_unit, double *qmax) {
  size_t m = (size_t)(s->nt * s->nt * s->nr);
  if (ell_lj) memcpy(ell_lj, s->ell_lj, sizeof(double) * m);
  if (ell_coul_unit) memcpy(ell_coul_unit, s->ell_cu, sizeof(double) * m);
  if (qmax) memcpy(qmax, s->qmax, sizeof(double) * (size_t)s->nt);
}
