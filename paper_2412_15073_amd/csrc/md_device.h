// md_device.h — device-side building blocks of libjumpmd (gfx950):
// counter-based random numbers, pair terms, the MRZ helper functions and the
// per-context device view shared by all kernels.
//
// Paper: Gouraud et al., "Velocity Jumps for Molecular Dynamics", arXiv 2412.15073.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MD_MAX_OPS 12
#define MD_ZS_MAXIT 64
#define MD_MAX_PROPOSALS (1ll << 22)  // per chain and half step; reaching it flags the run as unstable
#define MD_CHAIN_MAX_BLOCK_WAVES 8     // waves per k_chain block at most (two per SIMD of a CU)
#define MD_PI 3.14159265358979323846
#define MD_INV_SQRT_2PI 0.3989422804014327

// ----------------------------------------------------------------- random
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). Counter words: step,
// local atom index, tag = phase | substep << 8 | Z iteration << 24, proposal
// index k (each modulo 2^32); key words: low half of the seed, high half of
// the seed xor the replica index.
struct u32x4 { uint32_t w[4]; };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // one 32x32 -> 64 multiply gives both halves (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  u32x4 o; o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// uniform in (0,1): (w + 1/2) * 2^-32, exact in FP64
__device__ __forceinline__ double u01(uint32_t w) {
  return ((double)w + 0.5) * 2.3283064365386962890625e-10;
}

struct Uni4 { double u[4]; };

// the four raw words of block (step, atom, tag, k) under key (seed, replica)
__device__ __forceinline__ u32x4 draw4w(uint64_t seed, uint64_t rep, int64_t step, int64_t atom,
                                        uint64_t tag, int64_t k) {
  return philox4x32_10((uint32_t)step, (uint32_t)atom, (uint32_t)tag, (uint32_t)k,
                       (uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)rep);
}

__device__ __forceinline__ Uni4 draw4(uint64_t seed, uint64_t rep, int64_t step, int64_t atom,
                                      uint64_t tag, int64_t k) {
  const u32x4 r = draw4w(seed, rep, step, atom, tag, k);
  Uni4 o;
#pragma unroll
  for (int q = 0; q < 4; ++q) o.u[q] = u01(r.w[q]);
  return o;
}

// ------------------------------------------------------------ event hash
// Per-atom fingerprint of the accepted jumps (step, phase, partner), one
// multiply-xorshift per event.
__device__ __forceinline__ uint64_t event_mix(uint64_t h, int64_t step, int phase, int j) {
  const uint64_t key = (uint64_t)step * 0x9E3779B97F4A7C15ull + (uint64_t)(uint32_t)phase * 0xC2B2AE3D27D4EB4Full +
                       (uint64_t)(uint32_t)j;
  h = (h ^ key) * 0xFF51AFD7ED558CCDull;
  return h ^ (h >> 29);
}

// ------------------------------------------------------- context view
struct MDOp {
  int kind;      // OP_*
  int phase;     // random-stream phase tag (J/C/O)
  int substep;   // O: inner index of the RESPA schemes
  int flags;     // B: bit0 non-bonded, bit1 bonded, bit2 reciprocal, bit3 long real part;
                 // C: 0 -> a from nb+bonded, 1 -> nb only, 4 -> nb+bonded+reciprocal
  double h;      // duration
  double c1, c2; // O: exp(-gamma h), sqrt(1 - c1^2)
                 // (an O op carries its velocity-trace record index in rstep, -1: none)
  int64_t step;  // random-stream step word (and the label of logged events)
  // J/C proposal stream: words (rstep, rphase); stream 0: from index 0,
  // 1 (MD_STREAM_SAVE): from 0, first unused index kept per atom,
  // 2 (MD_STREAM_CONTINUE): from the kept index
  int64_t rstep;
  int rphase, stream;
};
#define MD_STREAM_SAVE 1
#define MD_STREAM_CONTINUE 2

enum { OP_B = 1, OP_A = 2, OP_O = 3, OP_J = 4, OP_C = 5, OP_DISP = 6 };

struct MDProg {
  int nops;
  int disp_slot;   // slot written by OP_DISP
  int reset_slot;  // slot cleared by thread 0 (-1: none)
  int dev_step;    // 1: op.step is an offset from ctl->step_base (graph replays)
  MDOp ops[MD_MAX_OPS];
};

struct MDCtl {                       // device-side control words
  int do_rebuild;
  int ovf_short;                     // longest short row requested beyond its capacity (0: none)
  int ovf_long;                      // longest full or candidate row requested beyond its capacity
  int ovf_queue;                     // longest stencil queue of the row builder beyond its LDS slots
  unsigned long long n_rebuilds;
  unsigned long long n_list_err;
  unsigned long long n_zs_overflow;
  unsigned long long n_events;
  unsigned long long nonfinite;
  long long step_base;               // random-stream step of offset 0 in graph replays
};

struct MDEventDev { long long step; int phase, atom, partner, proposal; };

// All device pointers and run constants; passed by value to every kernel.
struct MDView {
  int n, nt, nrep, nr, S;
  // state (positions double-buffered: chains read one buffer while drift writes the other)
  double4 *x0, *x1;      // xyz + charge
  double4 *v;            // velocity + mass in energy units (mass / accel_factor)
  double4 *fnb, *fb;     // forces (-grad): non-bonded, bonded
  double4 *frec, *flong; // Ewald: reciprocal-space forces (with the excluded-pair correction), and the
                         // long real-space part (1 - chi) U of the three-level BAOAB comparator
  double4 *xref;         // positions at the last row build
  const int *type, *rep, *loc;
  const double *box;     // [3*nrep]
  // per-type tables
  const double *c12, *c6, *ljshift;     // [nt*nt]
  const double *ell_lj, *ell_cu;        // [nt*nt*nr] bound per unit (Coulomb: per unit charge product)
  const double *qmax;                   // [nt]
  const double *qseg;                   // [nt*nr] qmax of the type of segment sg
  const int *type_active;               // [2*nt] type has a nonzero LJ / Coulomb segment bound
  // exclusions and bonded incidence
  const int *xptr, *xj;
  const int *bptr, *bterm;              // per atom: term code (idx << 1 | is_angle)
  const int *bond_ij; const double *bond_k, *bond_r0;
  const int *angle_ijk; const double *angle_k, *angle_t0;
  // cells
  const int *rep_cell_off;              // [nrep+1]
  const int *rep_cdim;                  // [3*nrep]
  int *cell_count, *cell_start, *cell_atoms, *atom_cell, *atom_slot;
  double4 *xcell;                       // [n] build positions in cell order
  float4 *xcellf;                       // [n] the same wrapped into the box, float (row prefilter)
  const int *cell_rep;                  // [ncell] replica of each cell
  const int *rep_off;                   // [nrep+1] first atom of each replica
  unsigned long long *rep_maxd2;        // [2*nrep] max |x - x_ref|^2 (double bits) per step parity and replica
  int ncell_total;
  int qimg;                             // row builder queue slots of replicas with explicit images (0: none)
  // Ewald reciprocal sum (one replica): k-vectors of the half space, w = exp(-k^2/(4 alpha^2)) / k^2
  const double4 *kvec;                  // [nk] (kx, ky, kz, w), ordered by (nx, ny, nz)
  const int4 *kint;                     // [nk] (nx, ny, nz, 1 if the first of its (nx, ny) column)
  int nk, kmax;
  int ew_ranges, ew_apb, ew_ta;         // structure factor: atom ranges of ew_apb atoms (partials per range), tiles of ew_ta
  int ew_krange;                        // reciprocal forces: k-vectors per range (partials per range)
  // smooth particle-mesh Ewald (one replica): K0 x K1 x K2 complex grid, influence
  // function G(m) (zero at m = 0), twiddles exp(2 pi i k / ptw_n) for k < ptw_n / 2
  int spme, porder;
  int pk[3];
  double2 *pgrid;
  const double *pinf;
  const double2 *ptw;
  int ptw_n;
  // velocity trace: O ops with rstep >= 0 record v of atoms [0, ntrace) into slot rstep % trace_cap
  double4 *trace;
  int ntrace;
  long long trace_cap;
  double ew_fcoef;                      // force prefactor 2 * 4 pi k_e / V (k and -k together)
  // neighbour rows (row-major, fixed capacity)
  int cap_s, cap_f, cap_c;
  int *srow, *scnt, *frow, *fcnt, *crow, *ccnt, *segst;
  // statistics
  long long *nprop, *nacc, *nviol;
  unsigned long long *hash;
  int *knext;            // [n] first unused proposal index of the last saved C stream
  MDCtl *ctl;
  MDEventDev *ev; long long ev_cap;
  // constants
  double rs, rc, w, inv_w, rlo, skin, rin, rout, rw, alpha, ke;
  double dsf_erfc_rc_over_rc, dsf_fc, two_a_sqpi;
  double beta, kT, eps0;
  int jlj, jc, log_events, precision;
  int chain_lanes;       // lanes cooperating on one atom's jump chain (1, 2, 4, 8, 16)
  int chain_block_waves; // waves per k_chain block
  int chain_groups;      // length of chain_perm (>= n)
  int chain_order;       // wave order of chain_perm: 1 type-major, 2 replica-major
  const int *chain_perm; // [chain_groups] atom whose chain group g runs, -1: idle group
  uint64_t seed;
};

// force of a B kick with these flags (see MDOp), atom i
__device__ __forceinline__ double3 kick_force(const MDView &V, int flags, int i, double4 fn, double4 fb) {
  double3 f = make_double3(0.0, 0.0, 0.0);
  if (flags & 1) { f.x += fn.x; f.y += fn.y; f.z += fn.z; }
  if (flags & 2) { f.x += fb.x; f.y += fb.y; f.z += fb.z; }
  if (flags & 4) { const double4 r = V.frec[i]; f.x += r.x; f.y += r.y; f.z += r.z; }
  if (flags & 8) { const double4 l = V.flong[i]; f.x += l.x; f.y += l.y; f.z += l.z; }
  return f;
}

// wave-scope ordering of LDS writes by some lanes before reads by others
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// -------------------------------------------------------------- geometry
__device__ __forceinline__ double min_img(double d, double L, double iL) {
  return d - L * rint(d * iL);
}

// Row entries: bits 0-22 hold the partner j (global index); in replicas with
// an edge shorter than 2 (r_c + skin), where a partner can have several
// images within the cutoff, bits 23-31 hold the image: the lattice vector n
// of the image x_j + n L, each component modulo 8 (3 bits each, x lowest).
// Between two row builds no atom moves by half an edge, so the nearest
// image m of the current displacement is within 1 of the build's, and n
// (within 1 of the build's nearest) is within 2 of m: n mod 8 fixes n.
#define MD_ROW_J_MASK 0x7fffff
#define MD_ROW_IMG_SHIFT 23

__device__ __forceinline__ int row_j(int e) { return e & MD_ROW_J_MASK; }

// whether the replica's rows carry explicit images (some edge < 2 (r_c + skin))
__device__ __forceinline__ bool rep_images(const double *L, double rout) {
  return L[0] < 2.0 * rout || L[1] < 2.0 * rout || L[2] < 2.0 * rout;
}

// d - n L for the image whose lattice component is congruent to c3 mod 8
__device__ __forceinline__ double img_comp(double d, double L, double iL, int c3) {
  const int m = (int)rint(d * iL);
  int dd = (c3 - m) & 7;
  dd = dd >= 4 ? dd - 8 : dd;
  return d - L * (double)(m + dd);
}

// displacement x_i - (image of x_j) of row entry e
__device__ __forceinline__ void row_disp(double4 xi, double4 xj, const double *L, const double *iL, bool img,
                                         int e, double &dx, double &dy, double &dz) {
  dx = xi.x - xj.x; dy = xi.y - xj.y; dz = xi.z - xj.z;
  if (!img) {
    dx = min_img(dx, L[0], iL[0]); dy = min_img(dy, L[1], iL[1]); dz = min_img(dz, L[2], iL[2]);
  } else {
    const unsigned c = (unsigned)e >> MD_ROW_IMG_SHIFT;
    dx = img_comp(dx, L[0], iL[0], (int)(c & 7u));
    dy = img_comp(dy, L[1], iL[1], (int)((c >> 3) & 7u));
    dz = img_comp(dz, L[2], iL[2], (int)((c >> 6) & 7u));
  }
}

// --------------------------------------------------------- pair terms (FP64)
// LJ energy-shifted at r_c: U = c12/r^12 - c6/r^6 - shift; Sec. 3.2.
// ir = 1/r (one reciprocal per pair serves every term).
__device__ __forceinline__ void lj_pair(double ir, double c12, double c6, double shift, double &U, double &dU) {
  const double ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
  U = ir6 * (c12 * ir6 - c6) - shift;
  dU = (-12.0 * c12 * ir6 * ir6 + 6.0 * c6 * ir6) * ir;
}

// Damped shifted-force Coulomb (Fennell-Gezelter 2006), zero value and slope at r_c.
__device__ __forceinline__ void dsf_pair(double r, double ir, double kqq, const MDView &V, double &U, double &dU) {
  const double e = erfc(V.alpha * r);
  const double g = exp(-V.alpha * V.alpha * r * r);
  U = kqq * (e * ir - V.dsf_erfc_rc_over_rc + V.dsf_fc * (r - V.rc));
  dU = kqq * (-(e * ir * ir + V.two_a_sqpi * g * ir) + V.dsf_fc);
}

// C2 quintic switch, 1 below r_s - w, 0 above r_s.
__device__ __forceinline__ void switch_fn(double r, const MDView &V, double &chi, double &dchi) {
  if (r <= V.rlo) { chi = 1.0; dchi = 0.0; return; }
  if (r >= V.rs) { chi = 0.0; dchi = 0.0; return; }
  const double t = (r - V.rlo) * V.inv_w;
  chi = 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
  dchi = -30.0 * t * t * (1.0 - t) * (1.0 - t) * V.inv_w;
}

// FP32 variants (mixed-precision path): pair arithmetic in float, with the
// constants of the run rounded once; accumulation stays in FP64.
__device__ __forceinline__ void lj_pair_f(float ir, float c12, float c6, float shift, float &U, float &dU) {
  const float ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
  U = ir6 * (c12 * ir6 - c6) - shift;
  dU = (-12.0f * c12 * ir6 * ir6 + 6.0f * c6 * ir6) * ir;
}

__device__ __forceinline__ void dsf_pair_f(float r, float ir, float kqq, const MDView &V, float &U, float &dU) {
  const float alpha = (float)V.alpha;
  const float e = erfcf(alpha * r);
  const float g = __expf(-alpha * alpha * r * r);
  U = kqq * (e * ir - (float)V.dsf_erfc_rc_over_rc + (float)V.dsf_fc * (r - (float)V.rc));
  dU = kqq * (-(e * ir * ir + (float)V.two_a_sqpi * g * ir) + (float)V.dsf_fc);
}

__device__ __forceinline__ void switch_fn_f(float r, const MDView &V, float &chi, float &dchi) {
  const float rlo = (float)V.rlo, rs = (float)V.rs, iw = (float)V.inv_w;
  if (r <= rlo) { chi = 1.0f; dchi = 0.0f; return; }
  if (r >= rs) { chi = 0.0f; dchi = 0.0f; return; }
  const float t = (r - rlo) * iw;
  chi = 1.0f - t * t * t * (10.0f - 15.0f * t + 6.0f * t * t);
  dchi = -30.0f * t * t * (1.0f - t) * (1.0f - t) * iw;
}

__device__ __forceinline__ float theta_fn_f(float eta) {
  return eta * (0.5f * erfcf(-eta * 0.70710678f)) + __expf(-0.5f * eta * eta) * 0.39894228f;
}

// Screen of Theta in float with the accurate erfcf and expf: relative error
// below MD_THETA_SCREEN_TOL / 4 against theta_fn for eta >= MD_THETA_SCREEN_LO
// (there the cancellation between the two terms amplifies rounding by less
// than 2 eta^2 = 50; the bound is checked on the device by a test).
#define MD_THETA_SCREEN_LO (-5.0)
#define MD_THETA_SCREEN_TOL 2.44140625e-4   // 2^-12
__device__ __forceinline__ float theta_screen(float eta) {
  return eta * (0.5f * erfcf(-eta * 0.70710678f)) + expf(-0.5f * eta * eta) * 0.39894228f;
}

// Theta(eta) = E[(eta+G)_+] = eta Phi(eta) + phi(eta)  (Sec. 2.2)
__device__ __forceinline__ double theta_fn(double eta) {
  return eta * (0.5 * erfc(-eta * 0.70710678118654752440)) + exp(-0.5 * eta * eta) * MD_INV_SQRT_2PI;
}

// Z = eta + G~ by exact rejection sampling (Sec. 2.4 regimes); one Philox
// block per iteration, counter word 2 = phase | (iteration+1) << 24.
__device__ double zsample(double eta, uint64_t seed, uint64_t rep, int64_t step, int64_t atom,
                          int phase, int64_t k, int &iters) {
  for (int r = 0; r < MD_ZS_MAXIT; ++r) {
    uint64_t tag = (uint64_t)(uint32_t)phase | ((uint64_t)(r + 1) << 24);
    Uni4 u = draw4(seed, rep, step, atom, tag, k);
    iters = r + 1;
    if (eta > 0.0) {
      double p_ray = 1.0 / (1.0 + eta * 2.5066282746310002);
      double rad = sqrt(-2.0 * log(u.u[1]));
      double y = (u.u[0] < p_ray) ? rad : rad * cos(2.0 * MD_PI * u.u[2]);
      double z = eta + y;
      if (y >= 0.0) return z;
      if (z <= 0.0) continue;
      if (u.u[3] <= z / eta) return z;
    } else if (eta >= -1.0) {
      double z = sqrt(-2.0 * log(u.u[0]));
      if (u.u[1] <= exp(eta * z)) return z;
    } else {
      double z = -(log(u.u[0]) + log(u.u[1])) / (-eta);
      if (u.u[2] <= exp(-0.5 * z * z)) return z;
    }
  }
  iters = -1;
  return 0.5 * (eta + sqrt(eta * eta + 4.0));
}
