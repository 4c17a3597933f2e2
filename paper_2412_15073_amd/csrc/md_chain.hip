// md_chain.hip — the jump-chain kernel of libjumpmd for gfx950 (CDNA4, wave64).
//
//  k_chain     the position-preserving prefix of a step program: B kicks,
//              J chains (BPS jumps, Sec. 3.2, Alg. 5 in exponential-clock
//              form) and C chains (acceleration + MRZ jumps, Sec. 2.4,
//              Alg. 4); G lanes per atom, proposal rings in LDS.
//  k_theta_screen_err  device check of the float screen of Theta.
#include "md_device.h"
#include "md_internal.h"

// ------------------------------------------------------------- helpers
// bound of segment sg = (type b, ring k) for an atom of type a; the table
// index (a * nt + b) * nr + k equals a * S + sg. Component coul: 0 the LJ
// long part, 1 the Coulomb long part, 2 both (the BOUNCE chain: their sum
// bounds the gradient of the whole long part)
__device__ __forceinline__ double seg_ell(const MDView &V, int a, int sg, int coul, double absq) {
  const int idx = a * V.S + sg;
  if (coul == 0) return V.ell_lj[idx];
  const double cu = (absq * V.qseg[sg]) * V.ell_cu[idx];
  return coul == 1 ? cu : V.ell_lj[idx] + cu;
}

// Damped shifted-force Coulomb in float for the jump gradients of the mixed
// path, with erfc(x) from the rational approximation of Abramowitz and Stegun
// (Handbook of Mathematical Functions, 1964, eq. 7.1.26; absolute error below
// 1.5e-7 for x >= 0), which reuses the Gaussian factor the force needs anyway.
__device__ __forceinline__ void dsf_pair_fa(float r, float ir, float kqq, const MDView &V, float &U, float &dU) {
  const float x = (float)V.alpha * r;
  const float g = __expf(-x * x);
  const float t = 1.0f / (1.0f + 0.3275911f * x);
  const float e = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f)))) * g;
  U = kqq * (e * ir - (float)V.dsf_erfc_rc_over_rc + (float)V.dsf_fc * (r - (float)V.rc));
  dU = kqq * (-(e * ir * ir + (float)V.two_a_sqpi * g * ir) + (float)V.dsf_fc);
}

// long-range gradient in FP32 (mixed-precision path) for the candidate image
// of row entry e: displacement in FP64,
// pair arithmetic in float, gradient returned in FP64
__device__ __forceinline__ double long_grad_f(const MDView &V, double4 xi, double4 xj, int a, int b, int coul,
                                              const double *L, const double *iL, bool img, int e, double &Fx,
                                              double &Fy, double &Fz) {
  double ddx, ddy, ddz;
  row_disp(xi, xj, L, iL, img, e, ddx, ddy, ddz);
  const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float r = sqrtf(r2);
  const float ir = 1.0f / r;
  float U = 0.0f, dU = 0.0f;
  if (r < (float)V.rc) {
    if (coul != 1) {
      const int ab = a * V.nt + b;
      const float c12 = (float)V.c12[ab], c6 = (float)V.c6[ab];
      if (c12 != 0.0f || c6 != 0.0f) lj_pair_f(ir, c12, c6, (float)V.ljshift[ab], U, dU);
    }
    if (coul != 0) {
      const float qq = (float)(xi.w * xj.w);
      if (qq != 0.0f) {
        float Uc, dUc;
        dsf_pair_fa(r, ir, (float)V.ke * qq, V, Uc, dUc);
        U += Uc; dU += dUc;
      }
    }
  }
  float chi, dchi;
  switch_fn_f(r, V, chi, dchi);
  const float g = ((1.0f - chi) * dU - dchi * U) * ir;
  Fx = (double)(g * dx); Fy = (double)(g * dy); Fz = (double)(g * dz);
  return Fx * Fx + Fy * Fy + Fz * Fz;
}

// long-range gradient F_ij = grad_i (1 - chi) U_ij of component coul (0 LJ,
// 1 Coulomb, 2 both; Sec. 3.1, 3.2)
__device__ __forceinline__ double long_grad_d(const MDView &V, double4 xi, double4 xj, int a, int b,
                                            int coul, const double *L, const double *iL, bool img, int e,
                                            double &Fx, double &Fy, double &Fz) {
  double dx, dy, dz;
  row_disp(xi, xj, L, iL, img, e, dx, dy, dz);
  double r2 = dx * dx + dy * dy + dz * dz;
  double r = sqrt(r2);
  const double ir = 1.0 / r;
  double U = 0.0, dU = 0.0;
  if (r < V.rc) {
    if (coul != 1) {
      int ab = a * V.nt + b;
      double c12 = V.c12[ab], c6 = V.c6[ab];
      if (c12 != 0.0 || c6 != 0.0) lj_pair(ir, c12, c6, V.ljshift[ab], U, dU);
    }
    if (coul != 0) {
      double qq = xi.w * xj.w;
      if (qq != 0.0) {
        double Uc, dUc;
        dsf_pair(r, ir, V.ke * qq, V, Uc, dUc);
        U += Uc; dU += dUc;
      }
    }
  }
  double chi, dchi;
  switch_fn(r, V, chi, dchi);
  const double g = ((1.0 - chi) * dU - dchi * U) * ir;
  Fx = g * dx; Fy = g * dy; Fz = g * dz;
  return Fx * Fx + Fy * Fy + Fz * Fz;
}

// PREC: MD_FP64 or MD_FP32_MIXED (pair arithmetic and Theta in float)
template <int PREC>
__device__ __forceinline__ double long_grad(const MDView &V, double4 xi, double4 xj, int a, int b, int coul,
                                            const double *L, const double *iL, bool img, int e, double &Fx,
                                            double &Fy, double &Fz) {
  if (PREC == MD_FP32_MIXED) return long_grad_f(V, xi, xj, a, b, coul, L, iL, img, e, Fx, Fy, Fz);
  return long_grad_d(V, xi, xj, a, b, coul, L, iL, img, e, Fx, Fy, Fz);
}

// uniform in (0, 1) in the chain's real type: in FP64 (w + 1/2) 2^-32 (u01),
// in the mixed path (w >> 9 + 1/2) 2^-23 from the top 23 bits, exact in float
__device__ __forceinline__ double u01r(uint32_t w, double) { return u01(w); }
__device__ __forceinline__ float u01r(uint32_t w, float) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// Theta in the chain's real type (float in the mixed path)
__device__ __forceinline__ double theta_r(double eta) { return theta_fn(eta); }
// mixed path: Theta(eta) = eta Phi(eta) + phi(eta) with Phi from the same
// erfc approximation (eq. 7.1.26) and the Gaussian factor shared with phi;
// absolute error below 1e-7 (1 + |eta|)
__device__ __forceinline__ float theta_r(float eta) {
  const float x = fabsf(eta) * 0.70710678f;
  const float g = __expf(-x * x);
  const float t = 1.0f / (1.0f + 0.3275911f * x);
  const float ec = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f)))) * g;
  const float Phi = eta >= 0.0f ? 1.0f - 0.5f * ec : 0.5f * ec;
  return eta * Phi + 0.39894228f * g;
}

// per-atom statistics of one launch: counts since its start (added to the
// stored totals at its end) and the running event fingerprint
struct AtomStats { int nprop, nacc, nviol; uint64_t hash; };

// accepted jump of atom i with partner lj (index within the replica)
__device__ __forceinline__ void log_jump(const MDView &V, AtomStats &st, int64_t step, int phase,
                                         int i, int lj, int64_t k) {
  st.hash = event_mix(st.hash, step, phase, lj);
  st.nacc++;
  if (V.log_events) {
    unsigned long long e = atomicAdd(&V.ctl->n_events, 1ull);
    if ((long long)e < V.ev_cap) {
      MDEventDev ev; ev.step = step; ev.phase = phase; ev.atom = i; ev.partner = V.rep_off[V.rep[i]] + lj;
      ev.proposal = (int)k;
      V.ev[e] = ev;
    }
  }
}

// the part of log_jump every lane of a group repeats (replicated statistics)
__device__ __forceinline__ void log_jump_hash_only(AtomStats &st, int64_t step, int phase, int lj) {
  st.hash = event_mix(st.hash, step, phase, lj);
  st.nacc++;
}

// ------------------------------------------------------- jump chains
// G lanes cooperate on one atom's chain; a wave holds 64/G atoms. The
// velocity-independent part of every proposal (Philox block, candidate of
// each branch, gathered position, long-range gradient, the uniforms of the
// first Z iteration) is computed into a per-atom ring of M slots in LDS, one
// proposal per lane. Refills are wave-synchronous: when any atom of the wave
// runs low, every atom with room takes G more proposals in the same pass, so
// the wave pays for one refill where desynchronised atoms would pay for each.
// The sequential part evaluates windows of G proposals: proposal times are
// left folds of the exponential clocks in proposal order, acceptance uses the
// velocity at the proposal time, and the first event (acceptance or end of
// the half step) is found with a group minimum. Every decision is the one the
// one-proposal-at-a-time chain takes.

// ring fields (chain real type R, field-major: field f of slot s at f*M + s):
// clock E, gradient and bound of each branch, and the first Z iteration's
// velocity-independent part (log u0, log u1, cospi(2 u2), u2; with G < 4 the
// uniforms u0, u1, -, u2 instead). Then, per slot,
// the raw words (u1, u3) of the proposal block and (u0, u3) of the Z block
// (uint2 each), and the candidate pair (by-bound, uniform) as int2.
enum { RF_E = 0, RF_BX, RF_BY, RF_BZ, RF_BL, RF_FX, RF_FY, RF_FZ, RF_FL,
       RF_ZL0, RF_ZL1, RF_ZCP, RF_ZU2, RF_N };

// real type of the chain arithmetic: FP64, or float in the mixed path
template <int PREC> struct ChainReal { using T = double; };
template <> struct ChainReal<MD_FP32_MIXED> { using T = float; };

__host__ __device__ constexpr int ring_slots(int G) { return G == 1 ? 3 : (5 * G) / 2; }

// LDS bytes of one atom's ring: R fields (8-byte aligned), then the two
// uint2 word pairs and the int2 candidate pair of every slot
__host__ __device__ constexpr int ring_rbytes(int G, int rsize) { return ((RF_N * ring_slots(G) * rsize + 7) / 8) * 8; }
__host__ __device__ constexpr int ring_bytes(int G, int rsize) { return ring_rbytes(G, rsize) + 24 * ring_slots(G); }

// LDS doubles per atom of the segment table for S segments: cumulative
// weights (S), cumulative counts (S, plus one spare: last usable segment)
// and starts (S + 1 ints)
// (with_el: the per-segment bounds too; kept in LDS when G >= 4 lanes share an atom)
// cw, [el,] then cn and st (32-bit with G >= 4; 16-bit below, where 64 / G
// tables per wave bound occupancy; row positions stay below 8192)
__host__ __device__ constexpr int seg_count_bytes(int G) { return G >= 4 ? 4 : 2; }
__host__ __device__ constexpr int seg_lds_doubles(int S, int G) {
  return (G >= 4 ? 2 * S : S) + (2 * seg_count_bytes(G) * (S + 1) + 7) / 8;
}
__host__ __device__ constexpr bool seg_el_in_lds(int G) { return G >= 4; }
template <int G> struct SegCount { using T = int; };
template <> struct SegCount<1> { using T = unsigned short; };
template <> struct SegCount<2> { using T = unsigned short; };

// Reductions over the G lanes of a group (G <= 16, groups aligned in the
// wave) with DPP lane permutations: swap neighbours, swap pairs, mirror
// within 8 lanes, mirror within 16 lanes. Every lane of the group must be
// active (group control flow is uniform).
template <int G, typename Op>
__device__ __forceinline__ int group_reduce(int x, Op op) {
  if (G >= 2) x = op(x, __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  if (G >= 4) x = op(x, __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  if (G >= 8) x = op(x, __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  if (G >= 16) x = op(x, __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false)); // row_mirror
  return x;
}
template <int G>
__device__ __forceinline__ int group_min(int x) {
  return group_reduce<G>(x, [](int a, int b) { return a < b ? a : b; });
}
template <int G>
__device__ __forceinline__ int group_sum(int x) {
  return group_reduce<G>(x, [](int a, int b) { return a + b; });
}

// |F|^2 evaluated the same way wherever it is needed
template <typename R>
__device__ __forceinline__ R norm2_nc(R x, R y, R z) {
#pragma clang fp contract(off)
  return x * x + y * y + z * z;
}

// Segment table of one atom for one jump component: cumulative weights
// sum n_q l_q and cumulative counts of the candidates whose bound is nonzero.
// The first segment whose cumulative value exceeds a target always has
// n_q l_q > 0, so the searches need no validity test.
// Per-atom segment table in LDS: cumulative weights cw[S], bounds el[S] (or
// read from the global table with fewer than 4 lanes per atom, where 64 / G
// tables per wave would cost occupancy), cumulative usable counts cn[S] (+
// spare slot: last usable segment + 1) and segment starts st[S + 1], of
// integer type CT (rows hold at most 8192 candidates).
template <typename CT>
struct SegL {
  double *cw, *el;
  CT *cn, *st;
  int S, top, last, a, coul;   // top: largest power of two <= S
  double W, nf, absq;

  __device__ __forceinline__ void attach(double *base, int S_, bool with_el) {
    S = S_;
    top = 1 << (31 - __clz(S_));
    cw = base;
    el = with_el ? base + S : nullptr;
    cn = (CT *)(base + (with_el ? 2 * S : S));
    st = cn + S + 1;
  }
  // bound of segment sg (the value seg_ell gives); EL: the table holds el
  template <bool EL>
  __device__ __forceinline__ double bound(const MDView &V, int sg) const {
    return EL ? el[sg] : seg_ell(V, a, sg, coul, absq);
  }
  // a table with no usable segment (no proposals), left untouched in LDS
  __device__ __forceinline__ void set_empty(int a_, int coul_, double absq_) {
    a = a_; coul = coul_; absq = absq_;
    W = 0.0; nf = 0.0; last = -1;
  }
  // The group's G lanes gather the segment starts and bounds in parallel;
  // lane r == 0 then forms the running sums in segment order from LDS, and
  // every lane reads back the totals.
  template <int G>
  __device__ __forceinline__ void build(const MDView &V, int i, int a_, int coul_, double absq_, int r) {
    a = a_; coul = coul_; absq = absq_;
    wave_lds_sync();   // earlier reads of the table by the group are complete
    const int *sst = V.segst + (size_t)i * (S + 1);
    for (int q = r; q <= S; q += G) st[q] = (CT)sst[q];
    for (int q = r; q < S; q += G) cw[q] = seg_ell(V, a, q, coul, absq);   // bound; running sum below
    wave_lds_sync();
    if (r == 0) {
      double w = 0.0;
      int c = 0, lst = -1;
#pragma unroll 4
      for (int q = 0; q < S; ++q) {
        const double l = cw[q];
        const int nq = (int)st[q + 1] - (int)st[q];
        w += (double)nq * l;
        if (l > 0.0) c += nq;
        if (nq > 0 && l > 0.0) lst = q;
        cw[q] = w; cn[q] = (CT)c;
        if (el) el[q] = l;
      }
      cn[S] = (CT)(lst + 1);   // spare slot: last usable segment + 1
    }
    wave_lds_sync();
    W = cw[S - 1];
    nf = (double)cn[S - 1];
    last = (int)cn[S] - 1;
  }
  // Candidates of both branches for one uniform u (the second only if
  // both): by bound (segment by n_q l_q, then uniform inside from the
  // residual) and uniform among those with a nonzero bound. Each segment is
  // the first whose cumulative value exceeds the target (the last usable one
  // past the end), found by two interleaved fixed-step bisections.
  template <bool EL>
  __device__ __forceinline__ void pick2(const MDView &V, double u, bool both, int &pb, double &ellb, int &segb,
                                        int &pf, double &ellf, int &segf) const {
    const double tb = u * W, tf = u * nf;
    int qb = 0, qf = 0;
    for (int step = top; step > 0; step >>= 1) {
      const int xb = qb + step, xf = qf + step;
      const double cb = cw[(xb <= S ? xb : S) - 1], cf = (double)cn[(xf <= S ? xf : S) - 1];
      if (xb <= S && cb <= tb) qb = xb;
      if (xf <= S && cf <= tf) qf = xf;
    }
    {
      const int sg = qb < S ? qb : last;
      const double below = sg > 0 ? cw[sg - 1] : 0.0;
      const double el_s = bound<EL>(V, sg);
      const int base = st[sg], n = st[sg + 1] - base;
      long long idx = (long long)floor((tb - below) / el_s);
      idx = idx < 0 ? 0 : (idx > n - 1 ? n - 1 : idx);
      pb = base + (int)idx; ellb = el_s; segb = sg;
    }
    pf = pb; ellf = 0.0; segf = segb;
    if (both) {
      const int sg = qf < S ? qf : last;
      const double below = sg > 0 ? (double)cn[sg - 1] : 0.0;
      const int base = st[sg], n = st[sg + 1] - base;
      long long idx = (long long)floor(tf - below);
      idx = idx < 0 ? 0 : (idx > n - 1 ? n - 1 : idx);
      pf = base + (int)idx; ellf = bound<EL>(V, sg); segf = sg;
    }
  }
};

// One Z iteration (Sec. 2.4 regimes) from the block's four uniforms. Both
// logarithms and the square root are shared by the regimes (lanes of a wave
// often sit in different regimes), and the acceptance tests of the first two
// regimes are taken in log space or without division.
// The iteration splits into its velocity-independent part (two logarithms
// and a cosine of the uniforms) and the eta-dependent rest.
template <typename R> struct ZPre { R l0, l1, cp; };

__device__ __forceinline__ double cospi_r(double x) { return cospi(x); }
__device__ __forceinline__ float cospi_r(float x) { return cospif(x); }

template <typename R>
__device__ __forceinline__ ZPre<R> z_pre(R u0, R u1, R u2) {
  return ZPre<R>{log(u0), log(u1), cospi_r(R(2) * u2)};
}

template <typename R>
__device__ __forceinline__ bool z_accept(R eta, const ZPre<R> &p, R u0, R u2, R u3, R &z) {
  const R rad = sqrt(R(-2) * (eta > R(0) ? p.l1 : p.l0));
  if (eta > R(0)) {
    // Rayleigh part with probability 1 / (1 + eta sqrt(2 pi)), else Gaussian
    const R y = (u0 * (R(1) + eta * R(2.5066282746310002)) < R(1)) ? rad : rad * p.cp;
    z = eta + y;
    return (y >= R(0)) || (z > R(0) && u3 * eta <= z);
  }
  if (eta >= R(-1)) {
    z = rad;
    return p.l1 <= eta * z;
  }
  z = (p.l0 + p.l1) / eta;
  return u2 <= exp(R(-0.5) * z * z);
}

template <typename R>
__device__ __forceinline__ bool z_iteration(R eta, R u0, R u1, R u2, R u3, R &z) {
  return z_accept<R>(eta, z_pre<R>(u0, u1, u2), u0, u2, u3, z);
}

// Z iterations it0, it0 + 1, ... with G of them in parallel: lane r tries
// it = base + r; the first accepted iteration (in order) wins.
template <int G, typename R>
__device__ __forceinline__ R zsample_grp(R eta, uint64_t seed, uint64_t rep, int64_t step, int64_t atom,
                                         int phase, int64_t k, int r, int it0, int &overflow) {
  overflow = 0;
  for (int base = it0; base < MD_ZS_MAXIT; base += G) {
    const int it = base + r;
    R z = R(0);
    bool ok = false;
    if (it < MD_ZS_MAXIT) {
      const uint64_t tag = (uint64_t)(uint32_t)phase | ((uint64_t)(it + 1) << 24);
      Uni4 u = draw4(seed, rep, step, atom, tag, k);
      ok = z_iteration<R>((R)eta, (R)u.u[0], (R)u.u[1], (R)u.u[2], (R)u.u[3], z);
    }
    const int first = group_min<G>(ok ? r : G);
    if (first < G) return __shfl(z, first, G);
  }
  overflow = 1;
  return R(0.5) * (eta + sqrt(eta * eta + R(4)));
}

__device__ __forceinline__ int ring_add(int s, int d, int M) {
  s += d;
  return s >= M ? s - M : s;
}

// One chain op over duration h for the atom of this group (wave-synchronous
// loop; groups that have finished stay masked until the wave is done).
//  J (BPS jumps of the LJ long part, Alg. 5 in the exponential-clock form of
//    Alg. 2): bound beta |v| l_s per candidate, constant over the op since a
//    reflection keeps |v|; proposal k at (E_0 + ... + E_k)/Lambda. In the
//    BOUNCE scheme (Sec. 3) the same chain covers the long part of the whole
//    pair potential: bounds l_LJ + l_Coulomb, F_ij the gradient of both.
//  C (Sec. 2.3 step (C), Alg. 1, Alg. 4; eps = eps0 |F| when adaptive):
//    constant acceleration a between jumps plus MRZ jumps of the Coulomb long
//    part; the bound is re-evaluated after each accepted jump (Sec. 2.4): from
//    (t_e, v_e), B_v = sqrt(|v_e|^2 + tau^2 |a|^2 + 2 tau (v_e.a)_+), tau = h - t_e.
//    With the BPS kernel on the Coulomb part (the eps -> infinity end of the
//    MRZ family, Sec. 2.2) the rate is beta (v.F)_+ against the bound
//    beta B_v l_s, and an accepted jump reflects v as in J.
// Block (rstep, i, rphase, k): u0 -> E_k, u1 -> bound part (adaptive C),
// u2 -> candidate, u3 -> acceptance; block (rstep, i, rphase | 1 << 24, k) ->
// first Z iteration.
// Ring position: proposals [w0, computed) sit in slots [ws, cs) of the ring.
// It outlives an op: an op that continues the stream an op of the same
// launch saved (same positions, same candidates) keeps its ring contents.
struct RingPos { int w0, ws, computed, cs; bool saved; };

// CB: the Coulomb jumps are BPS bounces (a separate instantiation, so that
// the MRZ chains carry none of the bounce code)
template <int G, int PREC, bool CB>
__device__ void chain_op(const MDView &V, const double4 *__restrict__ X, int i, int r, double4 xi,
                         double &vx, double &vy, double &vz, double me, double ax_d, double ay_d, double az_d,
                         const MDOp &op, AtomStats &st, const double *L, const double *iL,
                         typename ChainReal<PREC>::T *ring, uint2 *pwords, uint2 *zwords, int2 *jring,
                         SegL<typename SegCount<G>::T> &T, RingPos &rp) {
  using R = typename ChainReal<PREC>::T;
  constexpr int M = ring_slots(G);
  // The refill computes the velocity-independent part of the first Z
  // iteration of every proposal when G lanes share an atom (the window would
  // otherwise repeat it on every lane of the group); with fewer lanes only
  // the accepted proposals (about half) pay for it, in the window.
  constexpr bool kZPre = G >= 4;
  const bool isC = op.kind == OP_C;
  // jump component: C the Coulomb long part (both parts when the LJ one
  // jumps in C); J the LJ long part, or both in the BOUNCE scheme
  const int comp = isC ? (V.jlj == MD_JUMP_IN_C ? 2 : 1) : (V.jc == MD_JUMP_BOUNCE ? 2 : 0);
  const int a = V.type[i];
  const bool cont = op.stream == MD_STREAM_CONTINUE;
  if (!(cont && rp.saved)) {
    // the table of the saved op is the one this op needs (same kind, positions)
    const double absq = comp != 0 ? fabs(xi.w) : 0.0;
    const bool act_lj = comp != 1 && V.type_active[2 * a];
    const bool act_c = comp != 0 && V.type_active[2 * a + 1] && absq > 0.0;
    const bool active = act_lj || act_c;
    if (__any(active)) T.template build<G>(V, i, a, comp, absq, r);   // a whole wave or none builds
    else T.set_empty(a, comp, absq);
    rp.w0 = rp.computed = cont ? V.knext[i] : 0;
    rp.ws = rp.cs = 0;
  }
  rp.saved = false;
  const int *row = V.crow + (size_t)i * V.cap_c;
  const bool img = rep_images(L, V.rout);   // row entries carry explicit images
  const double inv_nr = 1.0 / (double)V.nr;
  const bool adaptive = isC && (V.jc == MD_JUMP_MRZ_ADAPTIVE);
  const bool bpsC = CB && isC;   // C with BPS bounces: no Z
  const bool mrz = isC && !bpsC;
  const R beta = (R)V.beta, eps0 = (R)V.eps0, mr = (R)me;
  const R f = sqrt(beta / (R(2) * R(MD_PI) * mr)) / eps0;   // 0 with bounces (eps0 = infinity)
  const R ax = (R)ax_d, ay = (R)ay_d, az = (R)az_d;
  const R aa = ax * ax + ay * ay + az * az;
  const uint64_t rep = (uint64_t)V.rep[i];
  const int li = V.loc[i];
  const int i0 = i - li;   // first atom of the replica
  const R h = (R)op.h;
  const R vn = sqrt((R)vx * (R)vx + (R)vy * (R)vy + (R)vz * (R)vz);   // J: |v| for the whole op
  // per-op constants of the MRZ rate and kernel (Sec. 2.4)
  const R sbm = sqrt(beta * mr);
  const R k_eta = eps0 * sbm;
  const R k_lam = adaptive ? sqrt(beta / mr) / eps0 : sqrt(beta) / (eps0 * sqrt(mr));
  const R k_coef = adaptive ? R(2) * eps0 / sbm : R(2) * eps0 / ((R(1) + eps0 * eps0) * sbm);
  const R W = (R)T.W, nfr = (R)T.nf;
  int n_counted = 0, n_viol = 0;   // lane-local, reduced over the group at the end
  int &w0 = rp.w0, &computed = rp.computed;   // proposal indices (below MD_MAX_PROPOSALS)
  int &ws = rp.ws, &cs = rp.cs;               // ring slots of w0 and of computed
  double vex = vx, vey = vy, vez = vz;   // velocity at the last event (FP64 state)
  R te = R(0), base = R(0);
  R tau = h, bBv = R(0), Wb = R(0), Lam = R(0), iLam = R(0);
  bool live = true, epoch = true;
  auto finish = [&]() {
    if (isC) { vx = vex + (double)tau * ax_d; vy = vey + (double)tau * ay_d; vz = vez + (double)tau * az_d; }
    live = false;
  };
  while (__any(live)) {
    if (live && epoch) {
      epoch = false;
      if (isC) {
        tau = h - te;
        const R vxr = (R)vex, vyr = (R)vey, vzr = (R)vez;
        const R vv = vxr * vxr + vyr * vyr + vzr * vzr;
        const R va = vxr * ax + vyr * ay + vzr * az;
        const R Bv = sqrt(vv + tau * tau * aa + R(2) * tau * (va > R(0) ? va : R(0)));
        bBv = beta * Bv;
        Wb = bBv * W;
        Lam = adaptive ? Wb + f * nfr : (bBv + f) * W;
        iLam = R(1) / Lam;
        base = R(0);
        if (!(Lam > R(0)) || !isfinite(Lam)) {
          if (!(Lam <= R(0)) && r == 0) atomicAdd(&V.ctl->nonfinite, 1ull);
          finish();
        }
      } else {
        Lam = beta * vn * W;
        iLam = R(1) / Lam;
        if (!(Lam > R(0))) finish();
        else if (!isfinite(Lam)) { if (r == 0) atomicAdd(&V.ctl->nonfinite, 1ull); finish(); }
      }
    }
    if (live && w0 >= MD_MAX_PROPOSALS) {
      if (r == 0) atomicAdd(&V.ctl->nonfinite, 1ull);
      finish();
    }
    // wave-synchronous refill: every atom tops up as many slots as are free
    // (at most G, one per lane); an atom below G takes G since M >= 2G. The
    // candidate gathers (row entries, then positions) are issued before the
    // work that needs no memory, so that it overlaps them.
    if (__any(live && computed - w0 < G)) {
      wave_lds_sync();   // reads of the slots being replaced are complete
      const int free_slots = M - (computed - w0);
      const int take = live ? (free_slots < G ? free_slots : G) : 0;
      if (r < take) {
        const int k = computed + r;
        const int sl = ring_add(cs, r, M);
        const u32x4 uw = draw4w(V.seed, rep, op.rstep, li, (uint64_t)op.rphase, k);
        // candidates of both branches first, so that their gathers overlap
        double ellb, ellf;
        int pb, pf, sb, sf;
        T.template pick2<seg_el_in_lds(G)>(V, u01(uw.w[2]), adaptive, pb, ellb, sb, pf, ellf, sf);
        const int eb = row[pb], ef = row[pf];
        ring[RF_E * M + sl] = -log(u01r(uw.w[0], R(0)));
        pwords[sl] = make_uint2(uw.w[1], uw.w[3]);
        ring[RF_BL * M + sl] = (R)ellb;
        if (adaptive) ring[RF_FL * M + sl] = (R)ellf;
        // the first Z iteration's uniforms, while the row entries are in flight
        if (mrz) {
          const u32x4 zw = draw4w(V.seed, rep, op.rstep, li, (uint64_t)(uint32_t)op.rphase | (1ull << 24), k);
          const R zu2 = u01r(zw.w[2], R(0));
          if (kZPre) {
            const ZPre<R> zp = z_pre<R>(u01r(zw.w[0], R(0)), u01r(zw.w[1], R(0)), zu2);
            ring[RF_ZL0 * M + sl] = zp.l0; ring[RF_ZL1 * M + sl] = zp.l1; ring[RF_ZCP * M + sl] = zp.cp;
          } else {
            ring[RF_ZL0 * M + sl] = u01r(zw.w[0], R(0)); ring[RF_ZL1 * M + sl] = u01r(zw.w[1], R(0));
          }
          ring[RF_ZU2 * M + sl] = zu2;
          zwords[sl] = make_uint2(zw.w[0], zw.w[3]);
        }
        const int jb = row_j(eb), jf = row_j(ef);
        const double4 xb = X[jb], xf = X[jf];
        double Fx, Fy, Fz;
        // segment sg = b * nr + ring: the partner's type without a load
        long_grad<PREC>(V, xi, xb, a, (int)(((double)sb + 0.5) * inv_nr), comp, L, iL, img, eb, Fx, Fy, Fz);
        ring[RF_BX * M + sl] = (R)Fx; ring[RF_BY * M + sl] = (R)Fy; ring[RF_BZ * M + sl] = (R)Fz;
        if (adaptive) {
          long_grad<PREC>(V, xi, xf, a, (int)(((double)sf + 0.5) * inv_nr), comp, L, iL, img, ef, Fx, Fy, Fz);
          ring[RF_FX * M + sl] = (R)Fx; ring[RF_FY * M + sl] = (R)Fy; ring[RF_FZ * M + sl] = (R)Fz;
        }
        jring[sl] = make_int2(jb - i0, jf - i0);   // replica-local indices (event hash)
      }
      computed += take;
      cs = ring_add(cs, take, M);
      wave_lds_sync();
    }
    if (!live) continue;
    // window [w0, w0 + G): lane r holds proposal w0 + r
    const int sl = ring_add(ws, r, M);
    R s = base, tot = base;
#pragma unroll
    for (int m = 0; m < G; ++m) {
      tot += ring[RF_E * M + ring_add(ws, m, M)];
      if (m == r) s = tot;
    }
    const uint2 pw = pwords[sl];
    const bool use_f = adaptive && !(u01r(pw.x, R(0)) * Lam < Wb);
    const int fo = use_f ? (RF_FX - RF_BX) * M : 0;
    const R Fx = ring[fo + RF_BX * M + sl], Fy = ring[fo + RF_BY * M + sl], Fz = ring[fo + RF_BZ * M + sl];
    const R ell = ring[fo + RF_BL * M + sl];
    const R F2 = norm2_nc(Fx, Fy, Fz);
    const R u3 = u01r(pw.y, R(0));
    // acceptance u3 <= lam / c and bound violation lam > c, tested without dividing
    bool out, acc = false, viol = false;
    R eta = R(0), tk = R(0);   // eta: MRZ argument of Theta, or v.F with BPS
    R zown = R(0);     // first Z iteration of this lane's proposal, taken if it is accepted
    bool zok = false;
    if (isC) {
      tk = te + s * iLam;
      out = tk > h;
      const R dtk = tk - te;
      const R vkx = (R)vex + dtk * ax, vky = (R)vey + dtk * ay, vkz = (R)vez + dtk * az;
      const R c = adaptive ? bBv * ell + f : ell * (bBv + f);
      R lam = R(0);
      const R vF = vkx * Fx + vky * Fy + vkz * Fz;
      bool decided = bpsC;
      if (bpsC) {
        eta = vF;
        lam = vF > R(0) ? beta * vF : R(0);
        acc = !out && lam > R(0) && u3 * c <= lam;
        viol = lam > c;
      } else if (!out && F2 > R(0)) {
        R scale;
        if (adaptive) {
          eta = k_eta * vF;
          scale = k_lam;
        } else {
          const R Fn = sqrt(F2);
          eta = k_eta * vF / Fn;
          scale = k_lam * Fn;
        }
        if (PREC == MD_FP64 && eta >= R(MD_THETA_SCREEN_LO)) {
          // Both decisions (acceptance u3 c <= lam, bound violation lam > c)
          // from the float screen when each lies outside its error bound;
          // they are then the FP64 decisions. FP64 Theta only otherwise.
          const R lam_s = scale * (R)theta_screen((float)eta);
          const R d = R(MD_THETA_SCREEN_TOL) * lam_s;
          const R thr = u3 * c;
          if ((lam_s - d >= thr || lam_s + d < thr) && (lam_s - d > c || lam_s + d <= c)) {
            acc = lam_s - d >= thr;
            viol = lam_s - d > c;
            decided = true;
          }
        }
        if (!decided) lam = scale * theta_r(eta);
      }
      if (!decided) {
        acc = !out && lam > R(0) && u3 * c <= lam;
        viol = lam > c;
      }
      // the first accepted proposal's Z is evaluated by its own lane, off the
      // sequential path after the group minimum
      if (acc && mrz) {
        const uint2 zz = zwords[sl];
        const ZPre<R> zp = kZPre ? ZPre<R>{ring[RF_ZL0 * M + sl], ring[RF_ZL1 * M + sl], ring[RF_ZCP * M + sl]}
                                 : z_pre<R>(ring[RF_ZL0 * M + sl], ring[RF_ZL1 * M + sl], ring[RF_ZU2 * M + sl]);
        zok = z_accept<R>(eta, zp, u01r(zz.x, R(0)), ring[RF_ZU2 * M + sl], u01r(zz.y, R(0)), zown);
      }
    } else {
      out = s * iLam > h;
      const R vF = (R)vx * Fx + (R)vy * Fy + (R)vz * Fz;
      const R c = vn * ell;
      acc = !out && vF > R(0) && u3 * c <= vF;
      viol = vF > c;
    }
    const int first = group_min<G>((out || acc) ? r : G);
    // proposals evaluated in this window: ranks before the event, plus an accepted one
    const bool counted = r < first || (r == first && acc);
    n_counted += counted ? 1 : 0;
    n_viol += (counted && viol) ? 1 : 0;
    if (first == G) { base = tot; w0 += G; ws = ring_add(ws, G, M); continue; }
    if (__shfl((int)out, first, G)) {
      // the proposal past the end is used up; the stream resumes after it
      w0 += first + 1;
      ws = ring_add(ws, first + 1, M);
      finish();
      continue;
    }
    // the accepted proposal's gradient, from the lane that holds it
    const int fs = ring_add(ws, first, M);
    const int fos = __shfl(fo, first, G);
    const R Fxs = __shfl(Fx, first, G), Fys = __shfl(Fy, first, G), Fzs = __shfl(Fz, first, G);
    const R F2s = __shfl(F2, first, G);
    const int2 jj = jring[fs];
    const int j = fos ? jj.y : jj.x;
    const int kstar = w0 + first;
    if (isC) {
      const R tks = __shfl(tk, first, G);
      R coef;
      if (bpsC) {
        coef = R(2) * __shfl(eta, first, G) / F2s;   // reflection at t_k
      } else {
        const R etas = __shfl(eta, first, G);
        R Z = __shfl(zown, first, G);
        if (!__shfl((int)zok, first, G)) {
          int ovf;
          Z = zsample_grp<G, R>(etas, V.seed, rep, op.rstep, li, op.rphase, kstar, r, 1, ovf);
          if (ovf && r == 0) atomicAdd(&V.ctl->n_zs_overflow, 1ull);
        }
        coef = adaptive ? k_coef * Z / (R(1) + eps0 * eps0 * F2s) : k_coef * Z / sqrt(F2s);
      }
      const R dts = tks - te;
      if (PREC == MD_FP32_MIXED) {
        // float kick, FP64 accumulation of the velocity
        vex += (double)(dts * ax - coef * Fxs);
        vey += (double)(dts * ay - coef * Fys);
        vez += (double)(dts * az - coef * Fzs);
      } else {
        vex = vex + dts * ax - coef * Fxs;
        vey = vey + dts * ay - coef * Fys;
        vez = vez + dts * az - coef * Fzs;
      }
      te = tks;
      epoch = true;   // new bound from (t_e, v_e)
    } else {
      const R vFs = (R)vx * Fxs + (R)vy * Fys + (R)vz * Fzs;
      const R c = R(2) * vFs / F2s;
      vx -= (double)(c * Fxs); vy -= (double)(c * Fys); vz -= (double)(c * Fzs);
      base = __shfl(s, first, G);
    }
    if (r == first) log_jump(V, st, op.step, op.phase, i, j, kstar);
    else log_jump_hash_only(st, op.step, op.phase, j);
    w0 = kstar + 1;
    ws = ring_add(ws, first + 1, M);
  }
  st.nprop += group_sum<G>(n_counted);
  st.nviol += group_sum<G>(n_viol);
  if (op.stream == MD_STREAM_SAVE) {
    if (r == 0) V.knext[i] = w0;
    rp.saved = true;
  }
}

// Chain kernel: the position-preserving prefix of a step program (B kicks,
// J and C chains) for every atom; G lanes per atom, 64/G atoms per wave and
// one or more independent waves per block (no block-wide barrier). Group g
// runs the chain of atom chain_perm[g] (-1: idle). Dynamic LDS per wave: the
// proposal rings of its 64/G atoms, then their segment tables.
#ifndef MD_CHAIN_WAVES_PER_SIMD
#define MD_CHAIN_WAVES_PER_SIMD 2   // register budget of the chain kernel: 512 / this per lane
#endif
template <int G, int PREC, bool CB>
__global__ __launch_bounds__(64 * MD_CHAIN_MAX_BLOCK_WAVES, MD_CHAIN_WAVES_PER_SIMD) void k_chain(
    MDView V, MDProg P, const double4 *__restrict__ X) {
  extern __shared__ double lds_chain[];
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int grp = gid / G, r = gid - (gid / G) * G;
  if (grp >= V.chain_groups) return;
  const int i = V.chain_perm[grp];
  if (i < 0) return;   // empty group of a partial wave
  const double4 xi = X[i];
  const double4 vv = V.v[i];
  double vx = vv.x, vy = vv.y, vz = vv.z;
  const double me = vv.w;
  const int rp = V.rep[i];
  const double L[3] = {V.box[3 * rp], V.box[3 * rp + 1], V.box[3 * rp + 2]};
  const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  AtomStats st;
  st.nprop = 0; st.nacc = 0; st.nviol = 0; st.hash = V.hash[i];
  const double4 fn = V.fnb[i], fb = V.fb[i];
  using R = typename ChainReal<PREC>::T;
  constexpr int M = ring_slots(G);
  constexpr int APB = 64 / G;
  constexpr int RB = ring_bytes(G, (int)sizeof(R));
  // each wave of the block owns one slice: the rings of its APB atoms, then their segment tables
  const int ab = ((int)threadIdx.x & 63) / G;
  constexpr bool kEl = seg_el_in_lds(G);
  char *wave_b = (char *)lds_chain + ((int)threadIdx.x >> 6) * (APB * RB + APB * 8 * seg_lds_doubles(V.S, G));
  char *base_b = wave_b + ab * RB;
  R *ring = (R *)base_b;
  uint2 *pwords = (uint2 *)(base_b + ring_rbytes(G, (int)sizeof(R)));
  uint2 *zwords = pwords + M;
  int2 *jring = (int2 *)(zwords + M);
  SegL<typename SegCount<G>::T> T;
  T.attach((double *)(wave_b + APB * RB) + ab * seg_lds_doubles(V.S, G), V.S, kEl);
  const int64_t sbase = P.dev_step ? (int64_t)V.ctl->step_base : 0;
  RingPos pos{0, 0, 0, 0, false};
  for (int o = 0; o < P.nops; ++o) {
    MDOp op = P.ops[o];
    op.step += sbase;
    op.rstep += sbase;
    if (op.kind == OP_B) {
      const double3 f = kick_force(V, op.flags, i, fn, fb);
      vx += op.h * f.x / me; vy += op.h * f.y / me; vz += op.h * f.z / me;
    } else {
      double ax = 0.0, ay = 0.0, az = 0.0;
      if (op.kind == OP_C) {
        // flags bit 0: short non-bonded forces only; bit 2: plus the reciprocal-space forces
        const bool wb = (op.flags & 1) == 0;
        const double4 fr = (op.flags & 4) ? V.frec[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        ax = (fn.x + (wb ? fb.x : 0.0) + fr.x) / me;
        ay = (fn.y + (wb ? fb.y : 0.0) + fr.y) / me;
        az = (fn.z + (wb ? fb.z : 0.0) + fr.z) / me;
      }
      chain_op<G, PREC, CB>(V, X, i, r, xi, vx, vy, vz, me, ax, ay, az, op, st, L, iL, ring, pwords, zwords, jring,
                            T, pos);
    }
  }
  if (r == 0) {
    if (!(isfinite(vx) && isfinite(vy) && isfinite(vz))) atomicAdd(&V.ctl->nonfinite, 1ull);
    V.v[i] = make_double4(vx, vy, vz, me);
    V.nprop[i] += st.nprop; V.nacc[i] += st.nacc; V.nviol[i] += st.nviol; V.hash[i] = st.hash;
  }
}

// ------------------------------------------------------------- launchers
// LDS bytes of one k_chain wave with G lanes per atom (rsize: bytes of the chain real type)
static size_t chain_lds_bytes(int G, int S, int rsize = 8) {
  return (size_t)(64 / G) *
         ((size_t)ring_bytes(G, rsize) + sizeof(double) * (size_t)seg_lds_doubles(S, G));
}
size_t chain_lds_bytes_host(int G, int S, int precision) {
  return chain_lds_bytes(G, S, precision == MD_FP32_MIXED ? 4 : 8);
}

// Occupancy of the MRZ instantiation. The bounce instantiation has the same
// LDS and at most the same registers (the launch bounds cap both), so this is
// also a lower bound for it.
template <int PREC>
static hipError_t chain_occupancy(int G, int threads, size_t lds, int *nb) {
  switch (G) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_chain<1, PREC, false>, threads, lds);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_chain<2, PREC, false>, threads, lds);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_chain<4, PREC, false>, threads, lds);
    case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_chain<8, PREC, false>, threads, lds);
    case 16: return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k_chain<16, PREC, false>, threads, lds);
  }
  return hipErrorInvalidValue;
}

// resident k_chain blocks of bw waves per CU (registers and LDS), 0 if unknown
int chain_blocks_per_cu(int G, int S, int precision, int bw) {
  int nb = 0;
  if (bw < 1 || bw > MD_CHAIN_MAX_BLOCK_WAVES) return 0;
  const size_t lds = (size_t)bw * chain_lds_bytes_host(G, S, precision);
  const hipError_t e = precision == MD_FP32_MIXED ? chain_occupancy<MD_FP32_MIXED>(G, 64 * bw, lds, &nb)
                                                  : chain_occupancy<MD_FP64>(G, 64 * bw, lds, &nb);
  return e == hipSuccess ? nb : 0;
}

template <int PREC, bool CB>
static void launch_chain_p(const MDView &V, const MDProg &P, const double4 *X, hipStream_t s) {
  const int G = V.chain_lanes, bw = V.chain_block_waves;
  const int nb = (int)(((long long)V.chain_groups * G + 64 * bw - 1) / (64 * bw));
  const size_t lds = (size_t)bw * chain_lds_bytes(G, V.S, PREC == MD_FP32_MIXED ? 4 : 8);
  const dim3 grid(nb), block(64 * bw);
  switch (G) {
    case 1: hipLaunchKernelGGL((k_chain<1, PREC, CB>), grid, block, lds, s, V, P, X); break;
    case 2: hipLaunchKernelGGL((k_chain<2, PREC, CB>), grid, block, lds, s, V, P, X); break;
    case 4: hipLaunchKernelGGL((k_chain<4, PREC, CB>), grid, block, lds, s, V, P, X); break;
    case 8: hipLaunchKernelGGL((k_chain<8, PREC, CB>), grid, block, lds, s, V, P, X); break;
    default: hipLaunchKernelGGL((k_chain<16, PREC, CB>), grid, block, lds, s, V, P, X); break;
  }
}

hipError_t launch_chain(const MDView &V, const MDProg &P, const double4 *X, hipStream_t s) {
  const bool cb = V.jc == MD_JUMP_BPS;
  if (V.precision == MD_FP32_MIXED) {
    if (cb) launch_chain_p<MD_FP32_MIXED, true>(V, P, X, s);
    else launch_chain_p<MD_FP32_MIXED, false>(V, P, X, s);
  } else {
    if (cb) launch_chain_p<MD_FP64, true>(V, P, X, s);
    else launch_chain_p<MD_FP64, false>(V, P, X, s);
  }
  return hipGetLastError();
}

// largest relative error of theta_screen against theta_fn over n points of
// [lo, hi]; nonnegative doubles order as their bit patterns
__global__ void k_theta_screen_err(double lo, double hi, int n, unsigned long long *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double eta = lo + (hi - lo) * ((double)t / (double)(n - 1));
  const double ref = theta_fn(eta);
  const double e = fabs((double)theta_screen((float)eta) - ref) / ref;
  atomicMax(out, (unsigned long long)__double_as_longlong(e));
}

hipError_t launch_theta_screen_err(double lo, double hi, int n, unsigned long long *out, hipStream_t s) {
  hipLaunchKernelGGL(k_theta_screen_err, dim3((n + 255) / 256), dim3(256), 0, s, lo, hi, n, out);
  return hipGetLastError();
}

