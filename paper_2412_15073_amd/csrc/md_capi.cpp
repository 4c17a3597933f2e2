// md_capi.cpp — C ABI of libjumpmd (declared in include/jumpmd.h): context
// setup, bound tables, neighbour-row scheduling, composition of the
// integrator steps into fused per-atom programs, observables.
//
// Paper: Gouraud et al., "Velocity Jumps for Molecular Dynamics", arXiv 2412.15073.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "md_internal.h"

namespace {

thread_local std::string g_create_error;

enum { ROW_SHORT = 1, ROW_FULL = 2, ROW_CAND = 4 };
enum { MODE_NONE = -1, MODE_JUMP = 0, MODE_BAOAB = 1, MODE_JUMP_RESPA = 2, MODE_BAOAB_RESPA = 3,
       MODE_JUMP_RESPA1 = 4, MODE_BAOAB_RESPA1 = 5 };

struct Timer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;  // kid, (start, end)
  size_t next = 0;
  double tot_ms[MD_K_COUNT] = {0};
  long long launches[MD_K_COUNT] = {0};
};

}  // namespace

struct md_ctx {
  hipStream_t stream = nullptr;
  int dev = 0;                 // device current at creation (the context's device)
  int n = 0, nt = 0, nrep = 0, nr = 1, S = 0;
  md_split split{};
  md_params par{};
  MDView V{};
  int cur = 0;                 // index of the position buffer holding the current positions
  int64_t step = 0;
  int fkind = -1;              // force kind held in fnb: 0 short, 1 full, -1 stale
  bool fb_valid = false;
  bool ewald = false;          // Ewald electrostatics (reciprocal sum in frec)
  bool spme = false;           // the reciprocal sum by smooth particle-mesh Ewald
  bool frec_valid = false;     // frec holds the reciprocal-space forces at the current positions
  bool flong_valid = false;    // flong holds the long real-space forces at the current positions
  double2 *d_spart = nullptr, *d_sfac = nullptr;   // Ewald partial and total structure factors
  double *d_pme_part = nullptr;                      // partial planes of the particle-mesh spreading
  double4 *d_fpart = nullptr;                       // Ewald partial forces per k-range
  double ew_ecoef = 0.0, ew_self = 0.0;            // Ewald energy prefactor (half space), self energy
  int rows_valid = 0;          // ROW_* bits valid for the current reference positions
  int64_t since_build = 0;
  int pc = 0, ps = 0;          // LDS key capacities of the row builder
  bool fuse_forces[2] = {false, false};   // per force kind: bonded blocks appended to the pair launch
  int nbonds = 0, nangles = 0;
  double kB = 1.0;
  std::vector<double> box;
  std::vector<int> rep_off;
  md_allocator alloc{};        // caller's allocator (alloc.alloc == nullptr: hipMalloc)
  struct Block { void *p; size_t bytes; };
  std::vector<Block> allocs;   // every device block of the context
  int *d_rep_off = nullptr;
  double *d_scratch = nullptr; size_t scratch_n = 0;
  unsigned long long *d_hist = nullptr; int hist_n = 0;
  double cap_factor = 1.5;     // initial row capacity / density estimate
  int nrep_max = 0;            // atoms of the largest replica
  int row_most = 1;            // longest possible row (entries)
  // Rollback point for regrowing the rows: the state at the first stepping
  // call after the last good synchronisation, and the stepping calls since.
  int64_t trace_n = 0;   // velocity-trace records taken since md_trace_velocities
  struct Snap {
    bool valid = false;
    double4 *x = nullptr, *v = nullptr, *xref = nullptr;
    int *knext = nullptr;
    long long *nprop = nullptr, *nacc = nullptr, *nviol = nullptr;
    unsigned long long *hash = nullptr, *maxd2 = nullptr;
    MDCtl *ctl = nullptr;
    int64_t step = 0, since_build = 0, trace_n = 0;
    int cur = 0, rows_valid = 0;
  } snap;
  struct Call { int kind; int64_t n; int which, phase; double h; };
  std::vector<Call> journal;
  bool replaying = false;
  int64_t n_regrows = 0;
  std::string err;
  bool prof = false;
  Timer tm;
  bool own_stream = false;
  // graph replay of K-step chunks (JUMP / BAOAB x current position buffer)
  bool capturing = false;
  int64_t step_rel0 = 0;
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  // host copies of device-side counters at the last sync
  MDCtl ctl_host{};
};

// ------------------------------------------------------------- utilities
static int fail(md_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return code;
}

#define HIPCHK(c, x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return fail((c), MD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Device memory of the context: from the caller's allocator when it gave
// one (e.g. PyTorch's caching allocator), otherwise hipMalloc.
static void *dalloc_bytes(md_ctx *c, size_t bytes) {
  bytes = bytes ? bytes : 1;
  void *p = nullptr;
  if (c->alloc.alloc) {
    p = c->alloc.alloc(c->alloc.ctx, bytes, (void *)c->stream);
    if (!p) { c->err = "allocator callback returned NULL for " + std::to_string(bytes) + " B"; return nullptr; }
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      c->err = std::string("hipMalloc(") + std::to_string(bytes) + " B): " + hipGetErrorString(e);
      return nullptr;
    }
  }
  c->allocs.push_back({p, bytes});
  return p;
}

template <class T>
static T *dalloc(md_ctx *c, size_t count) {
  return (T *)dalloc_bytes(c, sizeof(T) * count);
}

static void dfree(md_ctx *c, void *p) {
  for (size_t q = 0; q < c->allocs.size(); ++q) {
    if (c->allocs[q].p != p) continue;
    if (c->alloc.release) c->alloc.release(c->alloc.ctx, p, c->allocs[q].bytes, (void *)c->stream);
    else hipFree(p);
    c->allocs.erase(c->allocs.begin() + (long)q);
    return;
  }
}

static double4 *Xcur(md_ctx *c) { return c->cur == 0 ? c->V.x0 : c->V.x1; }
static double4 *Xoth(md_ctx *c) { return c->cur == 0 ? c->V.x1 : c->V.x0; }

static void prof_begin(md_ctx *c, int kid, hipEvent_t *e0) {
  if (!c->prof || c->capturing) return;
  Timer &t = c->tm;
  if (t.next + 2 > t.pool.size()) {
    for (int q = 0; q < 256; ++q) {
      hipEvent_t e;
      hipEventCreate(&e);
      t.pool.push_back(e);
    }
  }
  *e0 = t.pool[t.next++];
  hipEventRecord(*e0, c->stream);
  (void)kid;
}

static void prof_end(md_ctx *c, int kid, hipEvent_t e0) {
  if (!c->prof || c->capturing) return;
  Timer &t = c->tm;
  hipEvent_t e1 = t.pool[t.next++];
  hipEventRecord(e1, c->stream);
  t.pending.push_back({kid, {e0, e1}});
}

static void prof_collect(md_ctx *c) {
  Timer &t = c->tm;
  if (t.pending.empty()) return;
  hipStreamSynchronize(c->stream);
  for (auto &p : t.pending) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, p.second.first, p.second.second);
    t.tot_ms[p.first] += ms;
    t.launches[p.first] += 1;
  }
  t.pending.clear();
  t.next = 0;
}

// ---------------------------------------------------------- pair tables
// LJ 4 eps [(s/r)^12 - (s/r)^6] energy-shifted at r_c, as c12/r^12 - c6/r^6 - shift.
static void lj_value(double r, double eps, double sig, double rc, double *U, double *dU) {
  *U = 0.0; *dU = 0.0;
  if (eps == 0.0 || r >= rc) return;
  double s6 = std::pow(sig / r, 6.0), c6 = std::pow(sig / rc, 6.0);
  *U = 4.0 * eps * (s6 * s6 - s6) - 4.0 * eps * (c6 * c6 - c6);
  *dU = 4.0 * eps * (-12.0 * s6 * s6 + 6.0 * s6) / r;
}

// damped shifted-force Coulomb per unit charge product (including coulomb_k)
static void dsf_value(double r, double ke, double alpha, double rc, double *U, double *dU) {
  *U = 0.0; *dU = 0.0;
  if (r >= rc) return;
  double tas = 2.0 * alpha / std::sqrt(M_PI);
  double erc = std::erfc(alpha * rc);
  double fc = erc / (rc * rc) + tas * std::exp(-alpha * alpha * rc * rc) / rc;
  double er = std::erfc(alpha * r);
  *U = ke * (er / r - erc / rc + fc * (r - rc));
  *dU = ke * (-(er / (r * r) + tas * std::exp(-alpha * alpha * r * r) / r) + fc);
}

// ------------------------------------------------------------ programs
static MDOp op_base(int kind, double h) {
  MDOp o;
  memset(&o, 0, sizeof(o));
  o.kind = kind;
  o.h = h;
  return o;
}

struct ProgBuilder {
  MDProg P;
  bool has_a = false, has_chain_after_a = false;
  ProgBuilder() { memset(&P, 0, sizeof(P)); P.reset_slot = -1; P.disp_slot = 0; }
  // jump ops with their own proposal stream get the words (step, phase); an
  // O op keeps its velocity-trace record index in rstep
  void add(MDOp o) {
    if (o.kind == OP_A) has_a = true;
    if ((o.kind == OP_J || o.kind == OP_C) && has_a) has_chain_after_a = true;
    if ((o.kind == OP_J || o.kind == OP_C) && o.stream != MD_STREAM_CONTINUE) { o.rstep = o.step; o.rphase = o.phase; }
    P.ops[P.nops++] = o;
  }
};

static void add_B(ProgBuilder &b, double h, int flags) {
  MDOp o = op_base(OP_B, h);
  o.flags = flags;
  b.add(o);
}
static void add_A(ProgBuilder &b, double h) { b.add(op_base(OP_A, h)); }
static void add_O(md_ctx *c, ProgBuilder &b, double dt, int sub, int64_t step) {
  MDOp o = op_base(OP_O, dt);
  o.substep = sub;
  o.step = step;
  o.rstep = c->V.trace ? c->trace_n++ : -1;   // velocity-trace record
  o.c1 = std::exp(-c->par.gamma * dt);
  o.c2 = std::sqrt(-std::expm1(-2.0 * c->par.gamma * dt));
  b.add(o);
}
static void add_J(ProgBuilder &b, int phase, double h, int64_t step) {
  MDOp o = op_base(OP_J, h);
  o.phase = phase;
  o.step = step;
  b.add(o);
}
// (C') when Coulomb jumps are on, otherwise the plain kick it reduces to.
// stream: 0, MD_STREAM_SAVE, or MD_STREAM_CONTINUE (of the closing C' of the
// step before, whose words are (step - 1, OP_PHASE_C2))
// a_nb_only: the C acceleration (or the kick) takes the short non-bonded
// forces only (RESPA schemes); otherwise also the bonded forces and, with
// Ewald electrostatics, the reciprocal-space forces (plain JUMP)
static void add_C_or_B(md_ctx *c, ProgBuilder &b, int phase, double h, int64_t step, int a_nb_only,
                       int stream = 0) {
  if (c->par.jump_coul != MD_JUMP_NONE && c->par.jump_coul != MD_JUMP_BOUNCE) {
    MDOp o = op_base(OP_C, h);
    o.phase = phase;
    o.step = step;
    o.flags = a_nb_only ? 1 : (c->ewald ? 4 : 0);
    o.stream = stream;
    if (stream == MD_STREAM_CONTINUE) { o.rstep = step - 1; o.rphase = OP_PHASE_C2; }
    b.add(o);
  } else {
    add_B(b, h, a_nb_only ? 1 : (c->ewald ? 7 : 3));
  }
}
static void add_disp(ProgBuilder &b, int slot) {
  b.add(op_base(OP_DISP, 0.0));
  b.P.disp_slot = slot;
  b.P.reset_slot = slot ^ 1;
}

// A step program runs as at most two launches: the position-preserving
// prefix that holds the jump chains (k_chain), then the rest (k_local).
static int run_prog(md_ctx *c, ProgBuilder &b) {
  if (b.P.nops == 0) return MD_OK;
  if (b.has_chain_after_a) return fail(c, MD_ERR_ARG, "internal: jump chain after drift");
  if (c->capturing) {
    // step words become offsets from the device-side base set before each replay
    b.P.dev_step = 1;
    for (int o = 0; o < b.P.nops; ++o) { b.P.ops[o].step -= c->step_rel0; b.P.ops[o].rstep -= c->step_rel0; }
  }
  int cut = 0;
  bool chain = false;
  while (cut < b.P.nops && (b.P.ops[cut].kind == OP_B || b.P.ops[cut].kind == OP_J || b.P.ops[cut].kind == OP_C)) {
    chain |= (b.P.ops[cut].kind != OP_B);
    ++cut;
  }
  for (int o = cut; o < b.P.nops; ++o)
    if (b.P.ops[o].kind == OP_J || b.P.ops[o].kind == OP_C) return fail(c, MD_ERR_ARG, "internal: jump chain after drift");
  MDProg rest = b.P;
  if (chain) {
    MDProg pre = b.P;
    pre.nops = cut;
    pre.reset_slot = -1;
    hipEvent_t e0{};
    prof_begin(c, MD_K_CHAIN, &e0);
    HIPCHK(c, launch_chain(c->V, pre, Xcur(c), c->stream));
    prof_end(c, MD_K_CHAIN, e0);
    rest.nops = b.P.nops - cut;
    for (int o = 0; o < rest.nops; ++o) rest.ops[o] = b.P.ops[cut + o];
  }
  if (rest.nops > 0) {
    hipEvent_t e0{};
    prof_begin(c, MD_K_LOCAL, &e0);
    double4 *dst = b.has_a ? Xoth(c) : nullptr;
    HIPCHK(c, launch_local(c->V, rest, Xcur(c), dst, c->stream));
    prof_end(c, MD_K_LOCAL, e0);
  }
  if (b.has_a) {
    c->cur ^= 1;
    c->fkind = -1;
    c->fb_valid = false;
    c->frec_valid = false;
    c->flong_valid = false;
  }
  return MD_OK;
}

// -------------------------------------------------------- rows and forces
static int rows_for_mode(int mode) {
  if (mode == MODE_JUMP || mode == MODE_JUMP_RESPA || mode == MODE_JUMP_RESPA1) return ROW_SHORT | ROW_CAND;
  if (mode == MODE_BAOAB_RESPA1) return ROW_SHORT | ROW_FULL;
  return ROW_FULL;
}

// Build the requested rows at the reference positions without changing the
// rebuild schedule (initial build, after md_set_state, or a scheme switch).
static int build_rows_at_ref(md_ctx *c, int want, bool new_ref) {
  const double4 *X = new_ref ? Xcur(c) : c->V.xref;
  hipEvent_t e0{};
  prof_begin(c, MD_K_REBUILD, &e0);
  int w1 = want & (ROW_SHORT | ROW_CAND), w2 = want & ROW_FULL;
  if (w1) HIPCHK(c, launch_rebuild(c->V, X, w1, 0, 1, 0, 0.0, c->pc, c->ps, false, 0, c->stream));
  if (w2) HIPCHK(c, launch_rebuild(c->V, X, w2, 0, 1, 0, 0.0, c->pc, c->ps, false, 0, c->stream));
  prof_end(c, MD_K_REBUILD, e0);
  c->rows_valid = new_ref ? want : (c->rows_valid | want);
  if (new_ref) c->since_build = 0;
  return MD_OK;
}

static int ensure_rows(md_ctx *c, int want) {
  int missing = want & ~c->rows_valid;
  if (!missing) return MD_OK;
  bool fresh = (c->rows_valid == 0);
  return build_rows_at_ref(c, missing, fresh);
}

// Per-step schedule: rebuild when the maximum displacement since the last
// build exceeds skin/2 (decided on the device), or on the fixed period.
static int step_rebuild(md_ctx *c, int mode, int64_t step) {
  int want = rows_for_mode(mode);
  int slot = (int)(step & 1);
  double half = 0.5 * c->split.skin;
  double thr2 = half * half;
  hipEvent_t e0{};
  prof_begin(c, MD_K_REBUILD, &e0);
  c->since_build++;
  if (c->par.rebuild_every > 0) {
    bool forced = c->since_build >= c->par.rebuild_every;
    int w1 = want & (ROW_SHORT | ROW_CAND), w2 = want & ROW_FULL;
    if (forced) {
      if (w1) HIPCHK(c, launch_rebuild(c->V, Xcur(c), w1, slot, 1, 0, thr2, c->pc, c->ps, false, 1, c->stream));
      if (w2) HIPCHK(c, launch_rebuild(c->V, Xcur(c), w2, slot, 1, 0, thr2, c->pc, c->ps, false, 1, c->stream));
      c->rows_valid = want;
      c->since_build = 0;
    } else {
      HIPCHK(c, launch_rebuild(c->V, Xcur(c), want, slot, 0, 0, thr2, c->pc, c->ps, true, 1, c->stream));
    }
  } else {
    int w1 = want & (ROW_SHORT | ROW_CAND), w2 = want & ROW_FULL;
    if (w1) HIPCHK(c, launch_rebuild(c->V, Xcur(c), w1, slot, 0, 1, thr2, c->pc, c->ps, false, 1, c->stream));
    if (w2) HIPCHK(c, launch_rebuild(c->V, Xcur(c), w2, slot, 0, 1, thr2, c->pc, c->ps, false, 1, c->stream));
    // rows of the other kind are stale whenever a rebuild happened; the
    // device decides, so drop them conservatively
    c->rows_valid = want;
  }
  prof_end(c, MD_K_REBUILD, e0);
  return MD_OK;
}

static int eval_nb(md_ctx *c, int kind) {
  hipEvent_t e0{};
  prof_begin(c, MD_K_FORCE, &e0);
  HIPCHK(c, launch_force(c->V, Xcur(c), kind, false, c->stream));
  prof_end(c, MD_K_FORCE, e0);
  c->fkind = kind;
  return MD_OK;
}

static int eval_bonded(md_ctx *c) {
  if (c->nbonds + c->nangles > 0) {
    hipEvent_t e0{};
    prof_begin(c, MD_K_BONDED, &e0);
    HIPCHK(c, launch_bonded(c->V, Xcur(c), c->stream));
    prof_end(c, MD_K_BONDED, e0);
  }
  c->fb_valid = true;
  return MD_OK;
}

// pair forces of this kind and bonded forces, in one launch when both are due
static int eval_forces(md_ctx *c, int kind) {
  if (c->fkind != kind && !c->fb_valid && c->nbonds + c->nangles > 0 && c->fuse_forces[kind]) {
    hipEvent_t e0{};
    prof_begin(c, MD_K_FORCE, &e0);
    HIPCHK(c, launch_force(c->V, Xcur(c), kind, true, c->stream));
    prof_end(c, MD_K_FORCE, e0);
    c->fkind = kind;
    c->fb_valid = true;
    return MD_OK;
  }
  int rc;
  if (c->fkind != kind && (rc = eval_nb(c, kind))) return rc;
  if (!c->fb_valid && (rc = eval_bonded(c))) return rc;
  return MD_OK;
}

// Ewald reciprocal-space forces at the current positions (into V.frec)
static int eval_recip(md_ctx *c) {
  if (!c->ewald) return MD_OK;
  hipEvent_t e0{};
  prof_begin(c, MD_K_RECIP, &e0);
  if (c->spme) HIPCHK(c, launch_pme_forces(c->V, Xcur(c), c->d_pme_part, c->stream));
  else HIPCHK(c, launch_recip(c->V, Xcur(c), c->d_spart, c->d_sfac, c->d_fpart, c->stream));
  prof_end(c, MD_K_RECIP, e0);
  c->frec_valid = true;
  return MD_OK;
}

// long real-space part -grad (1 - chi) U at the current positions (into V.flong; full rows)
static int eval_long(md_ctx *c) {
  hipEvent_t e0{};
  prof_begin(c, MD_K_FORCE, &e0);
  HIPCHK(c, launch_force(c->V, Xcur(c), 2, false, c->stream));
  prof_end(c, MD_K_FORCE, e0);
  c->flong_valid = true;
  return MD_OK;
}

static int ensure_forces(md_ctx *c, int mode) {
  int rc = ensure_rows(c, rows_for_mode(mode));
  if (rc) return rc;
  const bool short_kind = mode == MODE_JUMP || mode == MODE_JUMP_RESPA || mode == MODE_JUMP_RESPA1 ||
                          mode == MODE_BAOAB_RESPA1;
  if ((rc = eval_forces(c, short_kind ? 0 : 1))) return rc;
  if (c->ewald && !c->frec_valid && (rc = eval_recip(c))) return rc;
  if (mode == MODE_BAOAB_RESPA1 && !c->flong_valid && (rc = eval_long(c))) return rc;
  return MD_OK;
}

// ------------------------------------------------------------ creation
static int validate(const md_system *s, const md_split *sp, const md_params *p) {
  if (!s || !sp || !p) return fail(nullptr, MD_ERR_ARG, "null argument");
  if (s->n_atoms <= 1 || s->n_types <= 0 || s->n_replicas <= 0)
    return fail(nullptr, MD_ERR_ARG, "need n_atoms > 1, n_types > 0, n_replicas > 0");
  if (!s->pos || !s->vel || !s->mass || !s->type || !s->lj_eps || !s->lj_sigma || !s->box)
    return fail(nullptr, MD_ERR_ARG, "missing system array");
  if (!(sp->switch_width > 0.0) || !(sp->r_s <= sp->r_c) || sp->skin < 0.0 || sp->r_s - sp->switch_width <= 0.0)
    return fail(nullptr, MD_ERR_ARG, "bad split (need 0 < r_s - w, w > 0, r_s <= r_c, skin >= 0)");
  if (sp->n_rings > 1 && !(sp->ring_width > 0.0)) return fail(nullptr, MD_ERR_ARG, "ring_width must be > 0");
  if (!(p->dt > 0.0) || p->gamma < 0.0 || !(p->kT > 0.0)) return fail(nullptr, MD_ERR_ARG, "bad dt/gamma/kT");
  if (p->jump_lj != MD_JUMP_NONE && p->jump_lj != MD_JUMP_BPS && p->jump_lj != MD_JUMP_IN_C)
    return fail(nullptr, MD_ERR_ARG, "jump_lj must be NONE, BPS or IN_C");
  if (p->jump_lj == MD_JUMP_IN_C && p->jump_coul != MD_JUMP_BPS && p->jump_coul != MD_JUMP_MRZ_CONST &&
      p->jump_coul != MD_JUMP_MRZ_ADAPTIVE)
    return fail(nullptr, MD_ERR_ARG, "jump_lj IN_C needs jump_coul BPS, MRZ_CONST or MRZ_ADAPTIVE");
  if (p->jump_coul != MD_JUMP_NONE && p->jump_coul != MD_JUMP_BPS && p->jump_coul != MD_JUMP_MRZ_CONST &&
      p->jump_coul != MD_JUMP_MRZ_ADAPTIVE && p->jump_coul != MD_JUMP_BOUNCE)
    return fail(nullptr, MD_ERR_ARG, "jump_coul must be NONE, BPS, MRZ_CONST, MRZ_ADAPTIVE or BOUNCE");
  if ((p->jump_coul == MD_JUMP_MRZ_CONST || p->jump_coul == MD_JUMP_MRZ_ADAPTIVE) && !(p->eps > 0.0))
    return fail(nullptr, MD_ERR_ARG, "eps must be > 0");
  if (p->precision != MD_FP64 && p->precision != MD_FP32_MIXED)
    return fail(nullptr, MD_ERR_ARG, "precision must be MD_FP64 or MD_FP32_MIXED");
  if (s->n_types * std::max(1, sp->n_rings) > 32)
    return fail(nullptr, MD_ERR_ARG, "n_types * n_rings must be <= 32");
  // every edge above r_c + skin: an atom never meets its own image, and only
  // the images next to the nearest one can come within r_c + skin
  for (int r = 0; r < s->n_replicas; ++r)
    for (int d = 0; d < 3; ++d)
      if (!(s->box[3 * r + d] > sp->r_c + sp->skin))
        return fail(nullptr, MD_ERR_ARG, "every box edge must exceed r_c + skin");
  double rlo = sp->r_s - sp->switch_width;
  for (int ab = 0; ab < s->n_types * s->n_types; ++ab)
    if (s->lj_eps[ab] != 0.0 && rlo < 1.25 * s->lj_sigma[ab])
      return fail(nullptr, MD_ERR_ARG, "r_s - switch_width must be >= 1.25 sigma for every LJ pair");
  const int n = s->n_atoms, nrep = s->n_replicas;
  for (int i = 0; i < n; ++i) {
    if (s->type[i] < 0 || s->type[i] >= s->n_types) return fail(nullptr, MD_ERR_ARG, "type out of range");
    if (!(s->mass[i] > 0.0) || !std::isfinite(s->mass[i])) return fail(nullptr, MD_ERR_ARG, "masses must be positive");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(s->pos[3 * i + d]) || !std::isfinite(s->vel[3 * i + d]))
        return fail(nullptr, MD_ERR_ARG, "positions and velocities must be finite");
    if (s->charge && !std::isfinite(s->charge[i])) return fail(nullptr, MD_ERR_ARG, "charges must be finite");
  }
  // replicas: offsets strictly increasing from 0 to N, at least two atoms each
  std::vector<int> rep_of(n, 0);
  if (s->replica_offset) {
    if (s->replica_offset[0] != 0 || s->replica_offset[nrep] != n)
      return fail(nullptr, MD_ERR_ARG, "replica_offset must run from 0 to n_atoms");
    for (int r = 0; r < nrep; ++r) {
      if (s->replica_offset[r + 1] - s->replica_offset[r] < 2)
        return fail(nullptr, MD_ERR_ARG, "replica_offset must increase by at least 2 atoms per replica");
      for (int i = s->replica_offset[r]; i < s->replica_offset[r + 1]; ++i) rep_of[i] = r;
    }
  } else if (nrep != 1) {
    return fail(nullptr, MD_ERR_ARG, "replica_offset required");
  }
  // replicas with an edge below 2 (r_c + skin) keep explicit images in their
  // rows: 13 bits of local atom index in the row builder's sort keys
  for (int r = 0; r < nrep; ++r) {
    const double rout = sp->r_c + sp->skin;
    const double *L = s->box + 3 * r;
    const int na = s->replica_offset ? s->replica_offset[r + 1] - s->replica_offset[r] : n;
    if ((L[0] < 2.0 * rout || L[1] < 2.0 * rout || L[2] < 2.0 * rout) && na > 8192)
      return fail(nullptr, MD_ERR_ARG, "a replica with an edge below 2 (r_c + skin) may hold at most 8192 atoms");
  }
  for (int r = 0; r < nrep; ++r)
    for (int d = 0; d < 3; ++d)
      if (!(s->box[3 * r + d] > 0.0) || !std::isfinite(s->box[3 * r + d]))
        return fail(nullptr, MD_ERR_ARG, "box edges must be positive");
  // bonded terms and exclusions: indices in [0, N) and inside the replica of their first atom
  auto in_rep = [&](int i, int first) { return i >= 0 && i < n && rep_of[i] == rep_of[first]; };
  if (s->n_bonds < 0 || s->n_angles < 0) return fail(nullptr, MD_ERR_ARG, "negative bond or angle count");
  if ((s->n_bonds > 0 && (!s->bond_ij || !s->bond_k || !s->bond_r0)) ||
      (s->n_angles > 0 && (!s->angle_ijk || !s->angle_k || !s->angle_t0)))
    return fail(nullptr, MD_ERR_ARG, "missing bond or angle array");
  for (int t = 0; t < s->n_bonds; ++t) {
    const int p = s->bond_ij[2 * t], q = s->bond_ij[2 * t + 1];
    if (p < 0 || p >= n || !in_rep(q, p) || p == q)
      return fail(nullptr, MD_ERR_ARG, "bond " + std::to_string(t) + ": atoms out of range or in different replicas");
  }
  for (int t = 0; t < s->n_angles; ++t) {
    const int p = s->angle_ijk[3 * t], m = s->angle_ijk[3 * t + 1], q = s->angle_ijk[3 * t + 2];
    if (p < 0 || p >= n || !in_rep(m, p) || !in_rep(q, p) || p == m || q == m || p == q)
      return fail(nullptr, MD_ERR_ARG, "angle " + std::to_string(t) + ": atoms out of range or in different replicas");
  }
  if (s->excl_ptr) {
    if (!s->excl_j && s->excl_ptr[n] > 0) return fail(nullptr, MD_ERR_ARG, "missing excl_j");
    if (s->excl_ptr[0] != 0) return fail(nullptr, MD_ERR_ARG, "excl_ptr[0] must be 0");
    for (int i = 0; i < n; ++i) {
      if (s->excl_ptr[i + 1] < s->excl_ptr[i]) return fail(nullptr, MD_ERR_ARG, "excl_ptr must be non-decreasing");
      for (int e = s->excl_ptr[i]; e < s->excl_ptr[i + 1]; ++e)
        if (!in_rep(s->excl_j[e], i))
          return fail(nullptr, MD_ERR_ARG, "exclusion of atom " + std::to_string(i) + " out of range or in another replica");
    }
  }
  if (p->bound_scale < 0.0 || !std::isfinite(p->bound_scale)) return fail(nullptr, MD_ERR_ARG, "bound_scale must be >= 0");
  if (p->row_capacity < 0.0 || !std::isfinite(p->row_capacity)) return fail(nullptr, MD_ERR_ARG, "row_capacity must be >= 0");
  if (p->event_capacity < 0 || p->event_capacity > (1ll << 31)) return fail(nullptr, MD_ERR_ARG, "event_capacity must be in [0, 2^31]");
  if (p->chain_order < 0 || p->chain_order > 2) return fail(nullptr, MD_ERR_ARG, "chain_order must be 0, 1 or 2");
  if (p->respa_outer < 0) return fail(nullptr, MD_ERR_ARG, "respa_outer must be >= 0 (0: 1)");
  if (sp->coulomb_kind != MD_COUL_DSF && sp->coulomb_kind != MD_COUL_EWALD && sp->coulomb_kind != MD_COUL_SPME)
    return fail(nullptr, MD_ERR_ARG, "coulomb_kind must be MD_COUL_DSF, MD_COUL_EWALD or MD_COUL_SPME");
  if (sp->coulomb_kind != MD_COUL_DSF && s->n_replicas != 1)
    return fail(nullptr, MD_ERR_ARG, "Ewald electrostatics: one replica per context");
  if (sp->coulomb_kind == MD_COUL_EWALD && (sp->ewald_kmax < 1 || sp->ewald_kmax > 64 || !(sp->coulomb_alpha > 0.0)))
    return fail(nullptr, MD_ERR_ARG, "Ewald electrostatics need 1 <= ewald_kmax <= 64 and coulomb_alpha > 0");
  if (sp->coulomb_kind == MD_COUL_SPME) {
    bool ok = sp->coulomb_alpha > 0.0 && (sp->pme_order == 4 || sp->pme_order == 6 || sp->pme_order == 8);
    for (int d = 0; d < 3; ++d) {
      const int K = sp->pme_grid[d];
      ok = ok && K >= 8 && K <= 256 && (K & (K - 1)) == 0 && K >= sp->pme_order;
    }
    if (!ok)
      return fail(nullptr, MD_ERR_ARG, "SPME needs coulomb_alpha > 0, pme_order 4, 6 or 8 and pme_grid edges "
                                       "that are powers of two in [8, 256]");
  }
  return MD_OK;
}

extern "C" int md_create(const md_system *s, const md_split *sp, const md_params *p, void *stream,
                         const md_allocator *alloc, md_ctx **out) {
  if (!out) return fail(nullptr, MD_ERR_ARG, "out is null");
  *out = nullptr;
  int rc = validate(s, sp, p);
  if (rc) return rc;
  if (p->graph_steps < 0 || (p->graph_steps & 1)) return fail(nullptr, MD_ERR_ARG, "graph_steps must be 0 or even");
  if (alloc && (!alloc->alloc || !alloc->release))
    return fail(nullptr, MD_ERR_ARG, "md_allocator needs both alloc and release");
  md_ctx *c = new md_ctx();
  if (alloc) c->alloc = *alloc;
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    return fail(nullptr, MD_ERR_HIP, "hipGetDevice failed");
  }
  // set-up of the allocation-free entry point on this device (once per device)
  if (rdf_scratch_setup(c->dev) != hipSuccess) {
    delete c;
    return fail(nullptr, MD_ERR_HIP, "hipGetSymbolAddress of the static scratch array failed");
  }
  c->stream = (hipStream_t)stream;
  if (!c->stream) {
    // graphs cannot be captured on the legacy default stream: use a private one
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(nullptr, MD_ERR_HIP, "hipStreamCreateWithFlags failed");
    }
    c->own_stream = true;
  }
  c->n = s->n_atoms;
  c->nt = s->n_types;
  c->nrep = s->n_replicas;
  c->split = *sp;
  c->par = *p;
  c->kB = s->kB > 0.0 ? s->kB : 1.0;
  if (c->par.respa_inner < 1) c->par.respa_inner = 1;
  if (c->par.bound_scale == 0.0) c->par.bound_scale = 1.0;
  c->cap_factor = c->par.row_capacity > 0.0 ? c->par.row_capacity : 1.5;
  c->nr = sp->n_rings > 0 ? sp->n_rings : 1;
  c->S = c->nt * c->nr;
  const int n = c->n, nt = c->nt, nr = c->nr, nrep = c->nrep;
  c->rep_off.resize(nrep + 1);
  if (nrep == 1 && !s->replica_offset) { c->rep_off[0] = 0; c->rep_off[1] = n; }
  else for (int r = 0; r <= nrep; ++r) c->rep_off[r] = s->replica_offset[r];
  if (c->rep_off[0] != 0 || c->rep_off[nrep] != n) { delete c; return fail(nullptr, MD_ERR_ARG, "bad replica_offset"); }
  c->box.assign(s->box, s->box + 3 * nrep);

  MDView &V = c->V;
  V.n = n; V.nt = nt; V.nrep = nrep; V.nr = nr; V.S = c->S;
  V.rs = sp->r_s; V.rc = sp->r_c; V.w = sp->switch_width; V.inv_w = 1.0 / sp->switch_width; V.rlo = sp->r_s - sp->switch_width;
  V.skin = sp->skin; V.rin = V.rlo - V.skin; V.rout = V.rc + V.skin;
  V.rw = nr == 1 ? V.rout - V.rin : sp->ring_width;
  V.alpha = sp->coulomb_alpha; V.ke = s->coulomb_k;
  V.two_a_sqpi = 2.0 * V.alpha / std::sqrt(M_PI);
  V.dsf_erfc_rc_over_rc = std::erfc(V.alpha * V.rc) / V.rc;
  V.dsf_fc = std::erfc(V.alpha * V.rc) / (V.rc * V.rc) + V.two_a_sqpi * std::exp(-V.alpha * V.alpha * V.rc * V.rc) / V.rc;
  V.beta = 1.0 / p->kT; V.kT = p->kT;
  // bounces are the eps -> infinity end of the MRZ family: the floor term of
  // the C-step bound, sqrt(beta / (2 pi m)) / eps, is then exactly zero
  V.eps0 = (p->jump_coul == MD_JUMP_BPS || p->jump_coul == MD_JUMP_BOUNCE) ? INFINITY : p->eps;
  V.jlj = p->jump_lj; V.jc = p->jump_coul; V.log_events = p->log_events; V.precision = p->precision;
  V.seed = p->seed;
  auto rep_of_atom = [&](int i) {
    return (int)(std::upper_bound(c->rep_off.begin(), c->rep_off.end(), i) - c->rep_off.begin()) - 1;
  };
  // Jump-chain layout. G (lanes per atom), automatic: the most lanes per atom
  // whose waves still fit the device in one round (resident blocks per CU
  // from the kernel's registers and LDS); when none does, 2 (on an ensemble
  // of 900k atoms, 2 lanes ran faster than 1 or 4).
  std::vector<int> chain_perm;
  {
    const int prec = p->precision, S = V.nt * V.nr;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int g = p->chain_lanes;
    if (g <= 0) {
      g = 2;
      for (int cand = 4; cand <= 16; cand *= 2) {
        if (chain_lds_bytes_host(cand, S, prec) > 65536) continue;
        int bpc = chain_blocks_per_cu(cand, S, prec, 1);
        if (bpc <= 0) bpc = 4;
        if ((long long)n * cand / 64 <= (long long)ncu * bpc) g = cand;
      }
      while (g < 16 && chain_lds_bytes_host(g, S, prec) > 65536) g *= 2;   // fewer atoms per wave
    }
    if (g != 1 && g != 2 && g != 4 && g != 8 && g != 16) { delete c; return fail(nullptr, MD_ERR_ARG, "chain_lanes must be 0, 1, 2, 4, 8 or 16"); }
    if (chain_lds_bytes_host(g, S, prec) > 65536) {
      delete c;
      return fail(nullptr, MD_ERR_ARG, "chain_lanes too small for this many segments (jump-chain LDS above 64 KiB per wave)");
    }
    V.chain_lanes = g;

    // Waves are type-pure (atoms of one type have similar jump counts, so a
    // wave is not held up by its busiest type), heaviest type first: jump
    // rates scale as 1/sqrt(mass) (MRZ rate sqrt(beta/m), BPS rate through
    // |v|), so light atoms run the longest chains.
    const int apw = 64 / g;
    std::vector<std::vector<int>> by_type(nt);
    std::vector<double> cost(nt, 0.0);
    for (int i = 0; i < n; ++i) {
      by_type[s->type[i]].push_back(i);
      cost[s->type[i]] += 1.0 / std::sqrt(s->mass[i]);
    }
    for (int t = 0; t < nt; ++t)
      if (!by_type[t].empty()) cost[t] /= (double)by_type[t].size();
    std::vector<int> torder(nt);
    for (int t = 0; t < nt; ++t) torder[t] = t;
    std::stable_sort(torder.begin(), torder.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    // Type-major order (the default): all waves of the heaviest type, then
    // the next type, partial waves last. Replica-major order: replica by
    // replica, each type-pure and heaviest type first, so that the resident
    // waves cover a run of consecutive replicas and gather from fewer
    // candidate rows. On the 256-replica water ensemble it ran 2 % slower
    // (5.26 against 5.14 ms per step): the load balance of heaviest-first
    // matters more there; the autotuner tries both.
    struct Chunk { const std::vector<int> *atoms; int beg, len; };
    std::vector<Chunk> waves;
    std::vector<std::vector<int>> by_rt;
    auto type_major = [&]() {
      std::vector<Chunk> part;
      waves.clear();
      for (int t : torder) {
        const int m = (int)by_type[t].size();
        for (int w = 0; w * apw < m; ++w) {
          Chunk ch{&by_type[t], w * apw, std::min(apw, m - w * apw)};
          (ch.len == apw ? waves : part).push_back(ch);
        }
      }
      waves.insert(waves.end(), part.begin(), part.end());
    };
    type_major();
    const int order = p->chain_order != 0 ? p->chain_order : 1;
    if (order == 2) {
      by_rt.assign((size_t)nrep * nt, {});
      for (int i = 0; i < n; ++i) by_rt[(size_t)rep_of_atom(i) * nt + s->type[i]].push_back(i);
      waves.clear();
      for (int r = 0; r < nrep; ++r)
        for (int t : torder) {
          const std::vector<int> &v = by_rt[(size_t)r * nt + t];
          for (int w = 0; w * apw < (int)v.size(); ++w) waves.push_back(Chunk{&v, w * apw, std::min(apw, (int)v.size() - w * apw)});
        }
    }
    V.chain_order = order;
    const long long nw = (long long)waves.size();

    // Block size. When every wave is resident at once, waves are packed into
    // blocks of bw (one block per CU) and the q-th wave of the order above
    // goes to block q mod nb, slot q / nb: a block's waves spread over the
    // CU's SIMDs, so the heaviest waves of the device land on distinct
    // SIMDs instead of sharing one. With more waves than resident slots,
    // one-wave blocks let the dispatcher balance the load.
    int bw = 1;
    const int bpc1 = chain_blocks_per_cu(g, S, prec, 1);
    if (bpc1 > 1 && nw <= (long long)ncu * bpc1)
      bw = (int)std::min<long long>({(long long)bpc1, (long long)MD_CHAIN_MAX_BLOCK_WAVES, (nw + ncu - 1) / ncu});
#ifdef MD_CHAIN_BLOCK_WAVES
    bw = std::max(1, std::min(MD_CHAIN_BLOCK_WAVES, MD_CHAIN_MAX_BLOCK_WAVES));
#endif
    while (bw > 1 && chain_blocks_per_cu(g, S, prec, bw) < 1) --bw;
    const long long nb = (nw + bw - 1) / bw;
    chain_perm.assign((size_t)(nb * bw * apw), -1);
    for (long long q = 0; q < nw; ++q) {
      const long long wv = (q % nb) * bw + q / nb;
      const Chunk &ch = waves[(size_t)q];
      for (int k = 0; k < ch.len; ++k) chain_perm[(size_t)(wv * apw + k)] = (*ch.atoms)[ch.beg + k];
    }
    V.chain_block_waves = bw;
    V.chain_groups = (int)chain_perm.size();
  }

  // --- host tables
  std::vector<double> c12(nt * nt), c6(nt * nt), shift(nt * nt), ell_lj(nt * nt * nr), ell_cu(nt * nt * nr), qmax(nt, 0.0);
  for (int ab = 0; ab < nt * nt; ++ab) {
    double e = s->lj_eps[ab], sg = s->lj_sigma[ab];
    c12[ab] = 4.0 * e * std::pow(sg, 12.0);
    c6[ab] = 4.0 * e * std::pow(sg, 6.0);
    shift[ab] = e == 0.0 ? 0.0 : c12[ab] / std::pow(V.rc, 12.0) - c6[ab] / std::pow(V.rc, 6.0);
  }
  // bounds on |grad (1-chi) U| for candidates of ring k (closest current
  // distance e_k - skin, not below r_s - w); see the ring technique, Sec. 3.1.1
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b)
      for (int k = 0; k < nr; ++k) {
        double ek = V.rin + k * V.rw;
        double ra = std::max(ek - V.skin, V.rlo);
        double lj = 0.0, cu = 0.0;
        if (ra < V.rc) {
          double Ul, dUl, Uc, dUc;
          lj_value(ra, s->lj_eps[a * nt + b], s->lj_sigma[a * nt + b], V.rc, &Ul, &dUl);
          dsf_value(ra, V.ke, V.alpha, V.rc, &Uc, &dUc);
          lj = std::fabs(dUl);
          cu = std::fabs(dUc);
          if (ra < V.rs) {
            lj += 15.0 / (8.0 * V.w) * std::fabs(Ul);
            cu += 15.0 / (8.0 * V.w) * std::fabs(Uc);
          }
        }
        ell_lj[(a * nt + b) * nr + k] = lj * c->par.bound_scale;
        ell_cu[(a * nt + b) * nr + k] = cu * c->par.bound_scale;
      }
  for (int i = 0; i < n; ++i) {
    double q = s->charge ? std::fabs(s->charge[i]) : 0.0;
    qmax[s->type[i]] = std::max(qmax[s->type[i]], q);
  }

  // --- cells per replica: edge >= (r_c + skin)/2, searched with a 5x5x5 stencil
  std::vector<int> cdim(3 * nrep), coff(nrep + 1, 0);
  double rho_max = 0.0;
  int nrep_max = 0;
  for (int r = 0; r < nrep; ++r) {
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) {
      double L = c->box[3 * r + d];
      cdim[3 * r + d] = std::max(1, (int)std::floor(L / (0.5 * V.rout)));
      vol *= L;
    }
    coff[r + 1] = coff[r] + cdim[3 * r] * cdim[3 * r + 1] * cdim[3 * r + 2];
    int nr_atoms = c->rep_off[r + 1] - c->rep_off[r];
    rho_max = std::max(rho_max, nr_atoms / vol);
    nrep_max = std::max(nrep_max, nr_atoms);
  }
  V.ncell_total = coff[nrep];
  auto sphere = [](double r) { return 4.0 / 3.0 * M_PI * r * r * r; };
  c->nrep_max = nrep_max;
  // longest possible row: every other atom of the largest replica, in up to
  // 27 images where some edge is below 2 (r_c + skin)
  bool any_img = false;
  int img_atoms = 0;   // atoms of the largest replica with explicit images
  for (int r = 0; r < nrep; ++r) {
    bool im = false;
    for (int d = 0; d < 3; ++d) im = im || c->box[3 * r + d] < 2.0 * V.rout;
    if (im) img_atoms = std::max(img_atoms, c->rep_off[r + 1] - c->rep_off[r]);
    any_img = any_img || im;
  }
  c->row_most = std::max(1, any_img ? 27 * nrep_max : nrep_max - 1);
  // the row builder's stencil queue of such a replica holds at most its atoms
  V.qimg = 0;
  if (any_img) { V.qimg = 64; while (V.qimg < img_atoms) V.qimg <<= 1; }
  auto capf = [&](double vol, int extra) {
    long long v = (long long)std::ceil(c->cap_factor * rho_max * vol) + extra;
    return (int)std::min<long long>(v, c->row_most);
  };
  V.cap_s = capf(sphere(V.rs + V.skin), 32);
  V.cap_f = capf(sphere(V.rout), 64);
  V.cap_c = capf(sphere(V.rout) - sphere(std::max(V.rin, 0.0)), 64);
  auto pow2 = [](int x) { int m = 1; while (m < x) m <<= 1; return m; };
  c->pc = pow2(std::max(V.cap_c, V.cap_f));
  c->ps = pow2(V.cap_s);
  if (n >= (1 << 23)) {
    delete c;
    return fail(nullptr, MD_ERR_ARG, "at most 2^23 - 1 atoms (23-bit atom field of the row entries)");
  }
  if (c->pc > 8192 || c->ps > 4096 || 4 * (c->pc + 64 + c->ps + V.qimg) > 65536) {
    delete c;
    return fail(nullptr, MD_ERR_ARG, "neighbour rows too long for the LDS row builder (density * (r_c + skin)^3 too large)");
  }

  // --- bonded incidence
  c->nbonds = s->n_bonds;
  c->nangles = s->n_angles;
  std::vector<int> bdeg(n + 1, 0);
  for (int t = 0; t < s->n_bonds; ++t) { bdeg[s->bond_ij[2 * t]]++; bdeg[s->bond_ij[2 * t + 1]]++; }
  for (int t = 0; t < s->n_angles; ++t)
    for (int q = 0; q < 3; ++q) bdeg[s->angle_ijk[3 * t + q]]++;
  std::vector<int> bptr(n + 1, 0);
  for (int i = 0; i < n; ++i) bptr[i + 1] = bptr[i] + bdeg[i];
  std::vector<int> bterm(std::max(1, bptr[n])), fillp(bptr.begin(), bptr.end() - 1);
  for (int t = 0; t < s->n_bonds; ++t)
    for (int q = 0; q < 2; ++q) bterm[fillp[s->bond_ij[2 * t + q]]++] = t << 1;
  for (int t = 0; t < s->n_angles; ++t)
    for (int q = 0; q < 3; ++q) bterm[fillp[s->angle_ijk[3 * t + q]]++] = (t << 1) | 1;

  // --- per-atom host arrays
  std::vector<double4> hx(n), hv(n);
  std::vector<int> rep(n), loc(n);
  for (int r = 0; r < nrep; ++r)
    for (int i = c->rep_off[r]; i < c->rep_off[r + 1]; ++i) { rep[i] = r; loc[i] = i - c->rep_off[r]; }
  for (int i = 0; i < n; ++i) {
    double q = s->charge ? s->charge[i] : 0.0;
    hx[i] = make_double4(s->pos[3 * i], s->pos[3 * i + 1], s->pos[3 * i + 2], q);
    hv[i] = make_double4(s->vel[3 * i], s->vel[3 * i + 1], s->vel[3 * i + 2], s->mass[i] / s->accel_factor);
  }

  // --- device allocation
  bool ok = true;
  auto A = [&](auto *&ptr, size_t cnt) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    ptr = dalloc<std::remove_const_t<T>>(c, cnt);
    if (!ptr) ok = false;
  };
  double4 *x0, *x1, *v, *fnb, *fb, *xref;
  A(x0, n); A(x1, n); A(v, n); A(fnb, n); A(fb, n); A(xref, n);
  int *d_type, *d_rep, *d_loc, *d_cdim, *d_coff;
  double *d_box, *d_c12, *d_c6, *d_shift, *d_elj, *d_ecu, *d_qmax, *d_qseg;
  A(d_type, n); A(d_rep, n); A(d_loc, n); A(d_cdim, 3 * nrep); A(d_coff, nrep + 1);
  A(d_box, 3 * nrep); A(d_c12, nt * nt); A(d_c6, nt * nt); A(d_shift, nt * nt);
  A(d_elj, nt * nt * nr); A(d_ecu, nt * nt * nr); A(d_qmax, nt); A(d_qseg, nt * nr);
  int *d_tact;
  A(d_tact, 2 * nt);
  int *d_xptr = nullptr, *d_xj = nullptr;
  if (s->excl_ptr) { A(d_xptr, n + 1); A(d_xj, std::max(1, s->excl_ptr[n])); }
  int *d_bptr, *d_bterm, *d_bij, *d_aijk;
  double *d_bk, *d_br0, *d_ak, *d_at0;
  A(d_bptr, n + 1); A(d_bterm, bterm.size());
  A(d_bij, std::max(1, 2 * s->n_bonds)); A(d_bk, std::max(1, s->n_bonds)); A(d_br0, std::max(1, s->n_bonds));
  A(d_aijk, std::max(1, 3 * s->n_angles)); A(d_ak, std::max(1, s->n_angles)); A(d_at0, std::max(1, s->n_angles));
  A(V.cell_count, V.ncell_total); A(V.cell_start, V.ncell_total + 1); A(V.cell_atoms, n);
  A(V.rep_maxd2, 2 * nrep); A(V.xcell, n); A(V.xcellf, n);
  int *d_chain_perm;
  A(d_chain_perm, chain_perm.size());
  int *d_cell_rep;
  A(d_cell_rep, V.ncell_total);
  A(V.atom_cell, n); A(V.atom_slot, n);
  A(V.srow, (size_t)n * V.cap_s); A(V.scnt, n);
  A(V.frow, (size_t)n * V.cap_f); A(V.fcnt, n);
  A(V.crow, (size_t)n * V.cap_c); A(V.ccnt, n); A(V.segst, (size_t)n * (c->S + 1));
  A(V.nprop, n); A(V.nacc, n); A(V.nviol, n); A(V.hash, n); A(V.knext, n);
  A(V.ctl, 1);
  V.ev_cap = p->log_events ? (p->event_capacity > 0 ? (long long)p->event_capacity : (1ll << 22)) : 0;
  if (V.ev_cap) A(V.ev, V.ev_cap);
  A(c->d_rep_off, nrep + 1);
  {   // rollback point of the row regrow (state at the first step after a good sync)
    md_ctx::Snap &q = c->snap;
    A(q.x, n); A(q.v, n); A(q.xref, n); A(q.knext, n);
    A(q.nprop, n); A(q.nacc, n); A(q.nviol, n); A(q.hash, n); A(q.maxd2, 2 * nrep); A(q.ctl, 1);
  }
  // Ewald reciprocal sum: k-vectors of the half space with 0 < |n|^2 <= kmax^2
  std::vector<double4> kv;
  std::vector<int4> kn;
  c->ewald = sp->coulomb_kind == MD_COUL_EWALD || sp->coulomb_kind == MD_COUL_SPME;
  c->spme = sp->coulomb_kind == MD_COUL_SPME;
  std::vector<double> pinf;
  std::vector<double2> ptw;
  if (c->spme) {
    // influence function G(m) = k_e / (2 pi V) exp(-pi^2 |m~|^2 / alpha^2) / |m~|^2 B(m),
    // B(m) = prod_d 1 / |sum_{k=0}^{p-2} M_p(k + 1) exp(2 pi i m_d k / K_d)|^2, G(0) = 0
    const int p = sp->pme_order;
    const int *K = sp->pme_grid;
    const double *L = c->box.data();
    const double vol = L[0] * L[1] * L[2];
    // M_p at the integers 1..p-1 by the recursion on the table of M_{n-1}
    std::vector<double> Mi(p + 1, 0.0), Mn(p + 1, 0.0);
    Mi[1] = 1.0;   // M_2 at 0, 1, 2
    for (int nn = 3; nn <= p; ++nn) {
      for (int u = 0; u <= nn; ++u)
        Mn[u] = ((double)u * (u <= nn - 1 ? Mi[u] : 0.0) + (double)(nn - u) * (u >= 1 ? Mi[u - 1] : 0.0)) / (nn - 1);
      Mi = Mn;
    }
    std::vector<double> bm[3];
    for (int d = 0; d < 3; ++d) {
      bm[d].assign(K[d], 0.0);
      for (int m = 0; m < K[d]; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= p - 2; ++k) {
          const double ph = 2.0 * M_PI * (double)((long long)m * k % K[d]) / K[d];
          re += Mi[k + 1] * std::cos(ph);
          im += Mi[k + 1] * std::sin(ph);
        }
        bm[d][m] = 1.0 / (re * re + im * im);
      }
    }
    pinf.assign((size_t)K[0] * K[1] * K[2], 0.0);
    for (int m0 = 0; m0 < K[0]; ++m0)
      for (int m1 = 0; m1 < K[1]; ++m1)
        for (int m2 = 0; m2 < K[2]; ++m2) {
          if (!m0 && !m1 && !m2) continue;
          const int mc[3] = {m0 <= K[0] / 2 ? m0 : m0 - K[0], m1 <= K[1] / 2 ? m1 : m1 - K[1],
                             m2 <= K[2] / 2 ? m2 : m2 - K[2]};
          double mm = 0.0;
          for (int d = 0; d < 3; ++d) mm += (mc[d] / L[d]) * (mc[d] / L[d]);
          pinf[((size_t)m0 * K[1] + m1) * K[2] + m2] = V.ke / (2.0 * M_PI * vol) *
              std::exp(-M_PI * M_PI * mm / (V.alpha * V.alpha)) / mm * bm[0][m0] * bm[1][m1] * bm[2][m2];
        }
    if (pme_fused(K)) {
      // the four-launch path reads G at (p, y', z'): frequencies (rev p, rev y', rev z')
      auto rev = [](int v, int Kd) {
        int r = 0;
        for (int b = 1; b < Kd; b <<= 1, v >>= 1) r = (r << 1) | (v & 1);
        return r;
      };
      std::vector<double> nat(pinf);
      for (int p0 = 0; p0 < K[0]; ++p0)
        for (int y = 0; y < K[1]; ++y)
          for (int z = 0; z < K[2]; ++z)
            pinf[((size_t)p0 * K[1] + y) * K[2] + z] =
                nat[((size_t)rev(p0, K[0]) * K[1] + rev(y, K[1])) * K[2] + rev(z, K[2])];
    }
    const int tn = std::max(K[0], std::max(K[1], K[2]));
    ptw.resize(tn / 2);
    for (int k = 0; k < tn / 2; ++k) ptw[k] = make_double2(std::cos(2.0 * M_PI * k / tn), std::sin(2.0 * M_PI * k / tn));
    V.spme = 1; V.porder = p; V.ptw_n = tn;
    for (int d = 0; d < 3; ++d) V.pk[d] = K[d];
    double2 *d_grid, *d_tw;
    double *d_inf;
    A(d_grid, pinf.size()); A(d_inf, pinf.size()); A(d_tw, ptw.size());
    if (pme_fused(K)) A(c->d_pme_part, (size_t)MD_PME_PARTS * pinf.size());
    V.pgrid = d_grid; V.pinf = d_inf; V.ptw = d_tw;
    A(V.frec, n); A(V.flong, n);
    double q2 = 0.0;
    for (int i = 0; i < n; ++i) q2 += s->charge ? s->charge[i] * s->charge[i] : 0.0;
    c->ew_self = -V.ke * V.alpha / std::sqrt(M_PI) * q2;
  } else if (c->ewald) {
    const int K = sp->ewald_kmax;
    const double *L = c->box.data();
    const double vol = L[0] * L[1] * L[2];
    for (int nx = 0; nx <= K; ++nx)
      for (int ny = -K; ny <= K; ++ny)
        for (int nz = -K; nz <= K; ++nz) {
          const int n2 = nx * nx + ny * ny + nz * nz;
          if (n2 == 0 || n2 > K * K) continue;
          if (nx == 0 && (ny < 0 || (ny == 0 && nz < 0))) continue;   // one of k, -k
          const double kx = 2.0 * M_PI * nx / L[0], ky = 2.0 * M_PI * ny / L[1], kz = 2.0 * M_PI * nz / L[2];
          const double k2 = kx * kx + ky * ky + kz * kz;
          kv.push_back(make_double4(kx, ky, kz, std::exp(-k2 / (4.0 * V.alpha * V.alpha)) / k2));
          const bool first = kn.empty() || kn.back().x != nx || kn.back().y != ny;
          kn.push_back(make_int4(nx, ny, nz, first ? 1 : 0));
        }
    V.nk = (int)kv.size();
    V.kmax = K;
    ewald_ranges(n, V.nk, K, V.ew_ranges, V.ew_apb, V.ew_ta, V.ew_krange);
    V.ew_fcoef = 2.0 * 4.0 * M_PI * V.ke / vol;
    c->ew_ecoef = 2.0 * 2.0 * M_PI * V.ke / vol;
    double q2 = 0.0;
    for (int i = 0; i < n; ++i) q2 += s->charge ? s->charge[i] * s->charge[i] : 0.0;
    c->ew_self = -V.ke * V.alpha / std::sqrt(M_PI) * q2;
    double4 *d_kv;
    A(d_kv, kv.size());
    V.kvec = d_kv;
    int4 *d_kn;
    A(d_kn, kn.size());
    V.kint = d_kn;
    A(V.frec, n); A(V.flong, n);
    A(c->d_spart, (size_t)V.ew_ranges * kv.size());
    A(c->d_fpart, (size_t)((V.nk + V.ew_krange - 1) / V.ew_krange) * n);
    A(c->d_sfac, kv.size());
  }
  c->scratch_n = std::max<size_t>(4 * (size_t)n + (size_t)s->n_bonds + (size_t)s->n_angles, 4096);
  c->scratch_n = std::max<size_t>(c->scratch_n, kv.size() + pinf.size() + (size_t)n);
  A(c->d_scratch, c->scratch_n);
  if (!ok) {
    std::string why = c->err;
    md_destroy(c);
    return fail(nullptr, MD_ERR_OOM, "device allocation failed: " + why);
  }

  hipStream_t st = c->stream;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (bytes && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess) ok = false;
  };
  up(x0, hx.data(), sizeof(double4) * n);
  up(v, hv.data(), sizeof(double4) * n);
  up(d_type, s->type, sizeof(int) * n);
  up(d_rep, rep.data(), sizeof(int) * n);
  up(d_loc, loc.data(), sizeof(int) * n);
  up(d_cdim, cdim.data(), sizeof(int) * 3 * nrep);
  up(d_coff, coff.data(), sizeof(int) * (nrep + 1));
  up(d_box, c->box.data(), sizeof(double) * 3 * nrep);
  up(d_c12, c12.data(), sizeof(double) * nt * nt);
  up(d_c6, c6.data(), sizeof(double) * nt * nt);
  up(d_shift, shift.data(), sizeof(double) * nt * nt);
  up(d_elj, ell_lj.data(), sizeof(double) * nt * nt * nr);
  up(d_ecu, ell_cu.data(), sizeof(double) * nt * nt * nr);
  up(d_qmax, qmax.data(), sizeof(double) * nt);
  {
    std::vector<double> qseg(nt * nr);   // max |q| of the type of each segment
    for (int sg = 0; sg < nt * nr; ++sg) qseg[sg] = qmax[sg / nr];
    up(d_qseg, qseg.data(), sizeof(double) * nt * nr);
    // per type: whether any LJ / Coulomb segment bound is nonzero (otherwise
    // the J / C chains of its atoms propose nothing)
    std::vector<int> tact(2 * nt, 0);
    for (int a = 0; a < nt; ++a)
      for (int sg = 0; sg < nt * nr; ++sg) {
        if (ell_lj[a * nt * nr + sg] > 0.0) tact[2 * a] = 1;
        if (qseg[sg] * ell_cu[a * nt * nr + sg] > 0.0) tact[2 * a + 1] = 1;
      }
    up(d_tact, tact.data(), sizeof(int) * 2 * nt);
  }
  if (s->excl_ptr) {
    up(d_xptr, s->excl_ptr, sizeof(int) * (n + 1));
    up(d_xj, s->excl_j, sizeof(int) * s->excl_ptr[n]);
  }
  up(d_bptr, bptr.data(), sizeof(int) * (n + 1));
  up(d_bterm, bterm.data(), sizeof(int) * bterm.size());
  up(d_bij, s->bond_ij, sizeof(int) * 2 * s->n_bonds);
  up(d_bk, s->bond_k, sizeof(double) * s->n_bonds);
  up(d_br0, s->bond_r0, sizeof(double) * s->n_bonds);
  up(d_aijk, s->angle_ijk, sizeof(int) * 3 * s->n_angles);
  up(d_ak, s->angle_k, sizeof(double) * s->n_angles);
  up(d_at0, s->angle_t0, sizeof(double) * s->n_angles);
  up(c->d_rep_off, c->rep_off.data(), sizeof(int) * (nrep + 1));
  up(d_chain_perm, chain_perm.data(), sizeof(int) * chain_perm.size());
  if (c->ewald && !c->spme) {
    up((void *)V.kvec, kv.data(), sizeof(double4) * kv.size());
    up((void *)V.kint, kn.data(), sizeof(int4) * kn.size());
  }
  if (c->spme) {
    up((void *)V.pinf, pinf.data(), sizeof(double) * pinf.size());
    up((void *)V.ptw, ptw.data(), sizeof(double2) * ptw.size());
  }
  c->fuse_forces[0] = force_fused_fits(V, 0);
  c->fuse_forces[1] = force_fused_fits(V, 1);
  {
    std::vector<int> cr(V.ncell_total);
    for (int r = 0; r < nrep; ++r)
      for (int q = coff[r]; q < coff[r + 1]; ++q) cr[q] = r;
    up(d_cell_rep, cr.data(), sizeof(int) * V.ncell_total);
  }
  if (hipMemsetAsync(V.rep_maxd2, 0, sizeof(unsigned long long) * 2 * nrep, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.cell_count, 0, sizeof(int) * V.ncell_total, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.ctl, 0, sizeof(MDCtl), st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.nprop, 0, sizeof(long long) * n, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.nacc, 0, sizeof(long long) * n, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.nviol, 0, sizeof(long long) * n, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(V.knext, 0, sizeof(int) * n, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(fnb, 0, sizeof(double4) * n, st) != hipSuccess) ok = false;
  if (hipMemsetAsync(fb, 0, sizeof(double4) * n, st) != hipSuccess) ok = false;
  {
    std::vector<unsigned long long> h0(n, 0xcbf29ce484222325ull);
    up(V.hash, h0.data(), sizeof(unsigned long long) * n);
    if (hipStreamSynchronize(st) != hipSuccess) ok = false;
  }
  if (!ok) { md_destroy(c); return fail(nullptr, MD_ERR_HIP, "upload failed"); }

  V.x0 = x0; V.x1 = x1; V.v = v; V.fnb = fnb; V.fb = fb; V.xref = xref;
  V.type = d_type; V.rep = d_rep; V.loc = d_loc; V.box = d_box;
  V.c12 = d_c12; V.c6 = d_c6; V.ljshift = d_shift; V.ell_lj = d_elj; V.ell_cu = d_ecu; V.qmax = d_qmax; V.qseg = d_qseg;
  V.type_active = d_tact;
  V.xptr = d_xptr; V.xj = d_xj; V.bptr = d_bptr; V.bterm = d_bterm;
  V.bond_ij = d_bij; V.bond_k = d_bk; V.bond_r0 = d_br0;
  V.angle_ijk = d_aijk; V.angle_k = d_ak; V.angle_t0 = d_at0;
  V.rep_cell_off = d_coff; V.rep_cdim = d_cdim;
  V.cell_rep = d_cell_rep; V.rep_off = c->d_rep_off; V.chain_perm = d_chain_perm;
  c->cur = 0;
  c->fkind = -1;
  c->fb_valid = false;
  c->frec_valid = false;
  c->flong_valid = false;
  c->rows_valid = 0;
  *out = c;
  return MD_OK;
}

extern "C" void md_destroy(md_ctx *c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  for (const md_ctx::Block &b : c->allocs) {
    if (c->alloc.release) c->alloc.release(c->alloc.ctx, b.p, b.bytes, (void *)c->stream);
    else hipFree(b.p);
  }
  c->allocs.clear();
  for (hipEvent_t e : c->tm.pool) hipEventDestroy(e);
  for (auto &g : c->gexec) if (g) hipGraphExecDestroy(g);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
}

extern "C" const char *md_last_error(const md_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

// -------------------------------------------------------------- stepping
static int baoab_plain(md_ctx *c, int64_t nsteps) {
  int rc = ensure_forces(c, MODE_BAOAB);
  if (rc) return rc;
  const double h = 0.5 * c->par.dt;
  const int fl = c->ewald ? 7 : 3;                   // non-bonded + bonded (+ reciprocal)
  for (int64_t it = 0; it <= nsteps; ++it) {
    ProgBuilder b;
    if (it > 0) add_B(b, h, fl);                     // tail of the previous step
    if (it < nsteps) {                               // head of this step
      add_B(b, h, fl);
      add_A(b, h);
      add_O(c, b, c->par.dt, 0, c->step);
      add_A(b, h);
      add_disp(b, (int)(c->step & 1));
    }
    if ((rc = run_prog(c, b))) return rc;
    if (it == nsteps) break;
    if ((rc = step_rebuild(c, MODE_BAOAB, c->step))) return rc;
    if ((rc = eval_forces(c, 1))) return rc;
    if ((rc = eval_recip(c))) return rc;
    c->step++;
  }
  return MD_OK;
}

static int jump_plain(md_ctx *c, int64_t nsteps) {
  int rc = ensure_forces(c, MODE_JUMP);
  if (rc) return rc;
  const double h = 0.5 * c->par.dt;
  // (J) steps: LJ bounces, or the BOUNCE scheme's bounces on the whole long part
  const bool lj = c->par.jump_lj == MD_JUMP_BPS || c->par.jump_coul == MD_JUMP_BOUNCE;
  for (int64_t it = 0; it <= nsteps; ++it) {
    ProgBuilder b;
    // The opening C' of a step continues the proposal stream of the closing
    // C' of the step before, after the proposal that ended it: both act at
    // the same positions, and those proposals were never used (fresh draws).
    if (it > 0) {                                    // J' C' closing the previous step
      if (lj) add_J(b, OP_PHASE_J2, h, c->step - 1);
      add_C_or_B(c, b, OP_PHASE_C2, h, c->step - 1, 0, MD_STREAM_SAVE);
    }
    if (it < nsteps) {                               // C' J' A O A
      add_C_or_B(c, b, OP_PHASE_C1, h, c->step, 0, MD_STREAM_CONTINUE);
      if (lj) add_J(b, OP_PHASE_J1, h, c->step);
      add_A(b, h);
      add_O(c, b, c->par.dt, 0, c->step);
      add_A(b, h);
      add_disp(b, (int)(c->step & 1));
    }
    if ((rc = run_prog(c, b))) return rc;
    if (it == nsteps) break;
    if ((rc = step_rebuild(c, MODE_JUMP, c->step))) return rc;
    if ((rc = eval_forces(c, 0))) return rc;
    if ((rc = eval_recip(c))) return rc;
    c->step++;
  }
  return MD_OK;
}

// Replay whole K-step chunks from a captured graph (captured lazily per
// scheme and position-buffer parity); the random-stream step base is set on
// the device before each replay. Steps left over run kernel by kernel.
static int graph_chunks(md_ctx *c, int mode, int64_t &n) {
  if (c->V.trace) return MD_OK;   // traced steps run as plain launches (one record index per O op)
  const int K = c->par.graph_steps;
  if (K <= 0 || c->par.rebuild_every > 0 || n < K) return MD_OK;
  int (*plain)(md_ctx *, int64_t) = mode == MODE_JUMP ? jump_plain : baoab_plain;
  int rc;
  if (c->step & 1) {            // chunks start on even steps (displacement-slot parity)
    if ((rc = plain(c, 1))) return rc;
    n -= 1;
    if (n < K) return MD_OK;
  }
  if ((rc = ensure_forces(c, mode))) return rc;
  const int key = (mode == MODE_JUMP ? 0 : 2) + c->cur;
  if (!c->gexec[key]) {
    const int64_t step0 = c->step;
    const int cur0 = c->cur, fk0 = c->fkind, rows0 = c->rows_valid;
    const bool fb0 = c->fb_valid, fr0 = c->frec_valid;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    c->step_rel0 = step0;
    rc = plain(c, K);
    c->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->step = step0; c->cur = cur0; c->fkind = fk0; c->rows_valid = rows0; c->fb_valid = fb0; c->frec_valid = fr0;
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(c, MD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { c->gexec[key] = nullptr; return fail(c, MD_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e)); }
  }
  while (n >= K) {
    HIPCHK(c, launch_set_step(c->V.ctl, (long long)c->step, c->stream));
    HIPCHK(c, hipGraphLaunch(c->gexec[key], c->stream));
    c->step += K;
    n -= K;
  }
  // a chunk ends with the forces and rows of this scheme current
  c->fkind = mode == MODE_JUMP ? 0 : 1;
  c->fb_valid = true;
  c->frec_valid = c->ewald;
  c->rows_valid = rows_for_mode(mode);
  return MD_OK;
}

static int respa(md_ctx *c, int64_t n_outer, bool jump) {
  const int mode = jump ? MODE_JUMP_RESPA : MODE_BAOAB_RESPA;
  int rc = ensure_forces(c, mode);
  if (rc) return rc;
  const int m = c->par.respa_inner;
  const double h = 0.5 * c->par.dt, H = 0.5 * c->par.dt * m;
  const bool lj = jump && (c->par.jump_lj == MD_JUMP_BPS || c->par.jump_coul == MD_JUMP_BOUNCE);
  for (int64_t it = 0; it <= n_outer; ++it) {
    // end of the previous outer step: closing inner kick, then J' C' (or the
    // outer non-bonded kick of BAOAB-RESPA)
    ProgBuilder b;
    if (it > 0) {
      add_B(b, h, 2);
      if (jump) {
        if (lj) add_J(b, OP_PHASE_J2, H, c->step - 1);
        add_C_or_B(c, b, OP_PHASE_C2, H, c->step - 1, 1, MD_STREAM_SAVE);
      } else {
        add_B(b, H, 1);
      }
    }
    if (it == n_outer) { if ((rc = run_prog(c, b))) return rc; break; }
    // start of this outer step, fused with the first inner B_b A O A
    if (jump) {
      add_C_or_B(c, b, OP_PHASE_C1, H, c->step, 1, MD_STREAM_CONTINUE);   // as in jump_plain
      if (lj) add_J(b, OP_PHASE_J1, H, c->step);
    } else {
      add_B(b, H, 1);
    }
    for (int sub = 0; sub < m; ++sub) {
      if (sub > 0) add_B(b, h, 2);                   // closing kick of inner step sub-1
      add_B(b, h, 2);
      add_A(b, h);
      add_O(c, b, c->par.dt, sub, c->step);
      add_A(b, h);
      if (sub == m - 1) add_disp(b, (int)(c->step & 1));
      if ((rc = run_prog(c, b))) return rc;
      if ((rc = eval_bonded(c))) return rc;
      b = ProgBuilder();
    }
    if ((rc = step_rebuild(c, mode, c->step))) return rc;
    if ((rc = eval_nb(c, jump ? 0 : 1))) return rc;
    c->step++;
  }
  return MD_OK;
}

// Three-level schemes (Ewald; Sec. 2.3.2, Sec. 3.3, Table 2). Inner steps
// B_b A O A B_b at dt; middle steps at M = respa_inner*dt: JUMP-RESPA1 runs
// the JUMP-RESPA step (C' J' [inner] J' C', short forces and all jumps),
// BAOAB-RESPA1 kicks with the short forces chi U; outer steps at
// respa_outer*M: a kick of half an outer step with the reciprocal-space
// forces (BAOAB-RESPA1: plus the long real-space part (1 - chi) U) on either
// side of the middle steps. Programs fuse the closing ops of one middle step
// with the opening ops of the next (and the two outer kicks between outer
// steps) into one position-preserving prefix, as in respa().
static int respa1(md_ctx *c, int64_t n_outer, bool jump) {
  const int mode = jump ? MODE_JUMP_RESPA1 : MODE_BAOAB_RESPA1;
  int rc = ensure_forces(c, mode);
  if (rc) return rc;
  const int m = c->par.respa_inner, p = std::max(1, c->par.respa_outer);
  const double h = 0.5 * c->par.dt, H = 0.5 * c->par.dt * m, HH = H * p;
  const bool lj = jump && (c->par.jump_lj == MD_JUMP_BPS || c->par.jump_coul == MD_JUMP_BOUNCE);
  const int outer_flags = jump ? 4 : (4 | 8);   // reciprocal (+ long real part)
  const int64_t n_mid = n_outer * p;
  for (int64_t it = 0; it <= n_mid; ++it) {
    ProgBuilder b;
    if (it > 0) {                                    // closing ops of middle step it-1
      add_B(b, h, 2);
      if (jump) {
        if (lj) add_J(b, OP_PHASE_J2, H, c->step - 1);
        add_C_or_B(c, b, OP_PHASE_C2, H, c->step - 1, 1, MD_STREAM_SAVE);
      } else {
        add_B(b, H, 1);
      }
      if (it % p == 0) add_B(b, HH, outer_flags);    // end of an outer step
    }
    if (it == n_mid) { if ((rc = run_prog(c, b))) return rc; break; }
    if (it % p == 0) add_B(b, HH, outer_flags);      // start of an outer step
    if (jump) {
      add_C_or_B(c, b, OP_PHASE_C1, H, c->step, 1, MD_STREAM_CONTINUE);
      if (lj) add_J(b, OP_PHASE_J1, H, c->step);
    } else {
      add_B(b, H, 1);
    }
    for (int sub = 0; sub < m; ++sub) {
      if (sub > 0) add_B(b, h, 2);
      add_B(b, h, 2);
      add_A(b, h);
      add_O(c, b, c->par.dt, sub, c->step);
      add_A(b, h);
      if (sub == m - 1) add_disp(b, (int)(c->step & 1));
      if ((rc = run_prog(c, b))) return rc;
      if ((rc = eval_bonded(c))) return rc;
      b = ProgBuilder();
    }
    if ((rc = step_rebuild(c, mode, c->step))) return rc;
    if ((rc = eval_nb(c, 0))) return rc;
    if ((it + 1) % p == 0) {                         // forces of the outer level at the outer boundary
      if ((rc = eval_recip(c))) return rc;
      if (!jump && (rc = eval_long(c))) return rc;
    }
    c->step++;
  }
  return MD_OK;
}

static int run_phase(md_ctx *c, int which, int phase, double h);
static int take_snapshot(md_ctx *c);

// Stepping calls are journaled since the rollback point (md_ctx::Snap), so
// that a row regrow can replay them.
enum { CALL_BAOAB = 0, CALL_JUMP, CALL_JUMP_RESPA, CALL_BAOAB_RESPA, CALL_PHASE, CALL_JUMP_RESPA1,
       CALL_BAOAB_RESPA1 };

static int run_call(md_ctx *c, const md_ctx::Call &k) {
  int64_t n = k.n;
  int rc;
  switch (k.kind) {
    case CALL_BAOAB:
      rc = graph_chunks(c, MODE_BAOAB, n);
      return rc ? rc : (n > 0 ? baoab_plain(c, n) : MD_OK);
    case CALL_JUMP:
      rc = graph_chunks(c, MODE_JUMP, n);
      return rc ? rc : (n > 0 ? jump_plain(c, n) : MD_OK);
    case CALL_JUMP_RESPA: return respa(c, n, true);
    case CALL_BAOAB_RESPA: return respa(c, n, false);
    case CALL_PHASE: return run_phase(c, k.which, k.phase, k.h);
    case CALL_JUMP_RESPA1: return respa1(c, n, true);
    case CALL_BAOAB_RESPA1: return respa1(c, n, false);
  }
  return fail(c, MD_ERR_ARG, "internal: unknown call");
}

static int step_call(md_ctx *c, const md_ctx::Call &k) {
  if (!c->snap.valid) {
    int rc = take_snapshot(c);
    if (rc) return rc;
  }
  c->journal.push_back(k);
  return run_call(c, k);
}

extern "C" int md_step_baoab(md_ctx *c, int64_t nsteps) {
  if (!c || nsteps < 0) return fail(c, MD_ERR_ARG, "bad argument");
  return step_call(c, {CALL_BAOAB, nsteps, 0, 0, 0.0});
}

extern "C" int md_step_jump(md_ctx *c, int64_t nsteps) {
  if (!c || nsteps < 0) return fail(c, MD_ERR_ARG, "bad argument");
  return step_call(c, {CALL_JUMP, nsteps, 0, 0, 0.0});
}

extern "C" int md_step_jump_respa(md_ctx *c, int64_t n_outer) {
  if (!c || n_outer < 0) return fail(c, MD_ERR_ARG, "bad argument");
  if (c->ewald) return fail(c, MD_ERR_ARG, "Ewald electrostatics: use md_step_jump_respa1");
  return step_call(c, {CALL_JUMP_RESPA, n_outer, 0, 0, 0.0});
}

extern "C" int md_step_baoab_respa(md_ctx *c, int64_t n_outer) {
  if (!c || n_outer < 0) return fail(c, MD_ERR_ARG, "bad argument");
  if (c->ewald) return fail(c, MD_ERR_ARG, "Ewald electrostatics: use md_step_baoab_respa1");
  return step_call(c, {CALL_BAOAB_RESPA, n_outer, 0, 0, 0.0});
}

extern "C" int md_step_jump_respa1(md_ctx *c, int64_t n_outer) {
  if (!c || n_outer < 0) return fail(c, MD_ERR_ARG, "bad argument");
  if (!c->ewald) return fail(c, MD_ERR_ARG, "the three-level schemes need Ewald electrostatics (MD_COUL_EWALD)");
  return step_call(c, {CALL_JUMP_RESPA1, n_outer, 0, 0, 0.0});
}

extern "C" int md_step_baoab_respa1(md_ctx *c, int64_t n_outer) {
  if (!c || n_outer < 0) return fail(c, MD_ERR_ARG, "bad argument");
  if (!c->ewald) return fail(c, MD_ERR_ARG, "the three-level schemes need Ewald electrostatics (MD_COUL_EWALD)");
  return step_call(c, {CALL_BAOAB_RESPA1, n_outer, 0, 0, 0.0});
}

// -------------------------------------------------------------- sync
// Row regrow: the rows of the context outgrew their capacities (the row
// builder records the longest requested row of each kind). New capacities
// take the requested lengths plus a quarter; the row buffers are reallocated
// and the captured graphs (which hold the old addresses) dropped.
static int regrow(md_ctx *c, const MDCtl &h) {
  MDView &V = c->V;
  const int most = c->row_most;
  auto grown = [&](int need, int have, int extra) {
    return std::min(most, std::max(have, need + need / 4 + extra));
  };
  int cap_s = h.ovf_short ? grown(h.ovf_short, V.cap_s, 32) : V.cap_s;
  const int need_long = h.ovf_long ? grown(h.ovf_long, std::max(V.cap_c, V.cap_f), 64) : 0;
  int cap_c = std::max(V.cap_c, need_long), cap_f = std::max(V.cap_f, need_long);
  auto pow2 = [](int x) { int m = 1; while (m < x) m <<= 1; return m; };
  int pc = std::max(c->pc, pow2(std::max(cap_c, cap_f)));
  if (h.ovf_queue) pc = std::max(pc, pow2(h.ovf_queue + h.ovf_queue / 4 - 64));
  const int ps = std::max(c->ps, pow2(cap_s));
  if (pc > 8192 || ps > 4096 || 4 * (pc + 64 + ps + V.qimg) > 65536)
    return fail(c, MD_ERR_CAPACITY, "neighbour rows of " + std::to_string(std::max(h.ovf_long, h.ovf_queue)) +
                                        " candidates / " + std::to_string(h.ovf_short) +
                                        " short entries exceed the row builder's limits (8192 / 4096)");
  auto realloc_rows = [&](int *&rows, int &cap, int want) -> bool {
    if (want == cap) return true;
    dfree(c, rows);
    rows = dalloc<int>(c, (size_t)c->n * want);
    cap = want;
    return rows != nullptr;
  };
  if (!realloc_rows(V.srow, V.cap_s, cap_s) || !realloc_rows(V.frow, V.cap_f, cap_f) ||
      !realloc_rows(V.crow, V.cap_c, cap_c))
    return fail(c, MD_ERR_OOM, "row regrow: " + c->err);
  c->pc = pc;
  c->ps = ps;
  for (auto &g : c->gexec)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  c->n_regrows++;
  return MD_OK;
}

static int take_snapshot(md_ctx *c) {
  md_ctx::Snap &q = c->snap;
  const MDView &V = c->V;
  const size_t n = (size_t)c->n;
  hipStream_t st = c->stream;
  HIPCHK(c, hipMemcpyAsync(q.x, Xcur(c), sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.v, V.v, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.xref, V.xref, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.knext, V.knext, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.nprop, V.nprop, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.nacc, V.nacc, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.nviol, V.nviol, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.hash, V.hash, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.maxd2, V.rep_maxd2, 8 * 2 * (size_t)c->nrep, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(q.ctl, V.ctl, sizeof(MDCtl), hipMemcpyDeviceToDevice, st));
  q.step = c->step;
  q.trace_n = c->trace_n;
  q.since_build = c->since_build;
  q.cur = c->cur;
  q.rows_valid = c->rows_valid;
  q.valid = true;
  c->journal.clear();
  return MD_OK;
}

// Back to the snapshot: state, statistics, event count and rebuild
// schedule; the rows valid then are rebuilt at the reference positions
// of then, and forces are re-evaluated at the next step (all deterministic).
static int restore_snapshot(md_ctx *c) {
  md_ctx::Snap &q = c->snap;
  const MDView &V = c->V;
  const size_t n = (size_t)c->n;
  hipStream_t st = c->stream;
  c->cur = q.cur;
  HIPCHK(c, hipMemcpyAsync(Xcur(c), q.x, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.v, q.v, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.xref, q.xref, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.knext, q.knext, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.nprop, q.nprop, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.nacc, q.nacc, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.nviol, q.nviol, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.hash, q.hash, 8 * n, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.rep_maxd2, q.maxd2, 8 * 2 * (size_t)c->nrep, hipMemcpyDeviceToDevice, st));
  HIPCHK(c, hipMemcpyAsync(V.ctl, q.ctl, sizeof(MDCtl), hipMemcpyDeviceToDevice, st));
  c->step = q.step;
  c->trace_n = q.trace_n;
  c->since_build = q.since_build;
  c->fkind = -1;
  c->fb_valid = false;
  c->frec_valid = false;
  c->flong_valid = false;
  c->rows_valid = 0;
  if (q.rows_valid) return build_rows_at_ref(c, q.rows_valid, false);
  return MD_OK;
}

static int run_call(md_ctx *c, const md_ctx::Call &k);
static int report_flags(md_ctx *c);

// Synchronise and report. Rows that outgrew their capacity are recovered
// here: back to the snapshot, regrow, replay the stepping calls since (the
// counter-based random streams make the replay identical to a run that
// never overflowed); without a snapshot (no step since the last good sync)
// only the rows are rebuilt. Then the device-side error flags are reported.
static int settle(md_ctx *c) {
  for (int attempt = 0;; ++attempt) {
    HIPCHK(c, hipMemcpyAsync(&c->ctl_host, c->V.ctl, sizeof(MDCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const MDCtl h = c->ctl_host;
    if (!(h.ovf_short || h.ovf_long || h.ovf_queue)) break;
    int rc = attempt < 8 ? regrow(c, h) : fail(c, MD_ERR_CAPACITY, "rows kept overflowing after regrowing");
    if (rc == MD_OK && c->snap.valid) {
      rc = restore_snapshot(c);
      c->replaying = true;
      for (size_t q = 0; rc == MD_OK && q < c->journal.size(); ++q) rc = run_call(c, c->journal[q]);
      c->replaying = false;
    } else if (rc == MD_OK) {
      const int zero[3] = {0, 0, 0};
      HIPCHK(c, hipMemcpyAsync(&c->V.ctl->ovf_short, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
      const int rv = c->rows_valid;
      c->rows_valid = 0;
      c->fkind = -1;
      c->fb_valid = false;
      c->frec_valid = false;
      c->flong_valid = false;
      if (rv) rc = build_rows_at_ref(c, rv, false);
    }
    if (rc != MD_OK) {
      // unrecoverable: the state of the last good synchronisation
      const std::string why = c->err;
      if (c->snap.valid) (void)restore_snapshot(c);
      const int zero[3] = {0, 0, 0};
      (void)hipMemcpyAsync(&c->V.ctl->ovf_short, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream);
      (void)hipStreamSynchronize(c->stream);
      c->snap.valid = false;
      c->journal.clear();
      return fail(c, rc, why);
    }
  }
  c->snap.valid = false;
  c->journal.clear();
  return report_flags(c);
}

// Device-side error flags of the last synchronisation (ctl_host), after any
// row overflow has been dealt with.
static int report_flags(md_ctx *c) {
  const MDCtl &h = c->ctl_host;
  if (h.nonfinite) return fail(c, MD_ERR_UNSTABLE, "non-finite velocities");
  if (c->par.rebuild_every > 0 && h.n_list_err)
    return fail(c, MD_ERR_LIST, "displacement beyond skin/2 between scheduled rebuilds");
  if (c->par.strict_bounds) {
    std::vector<long long> nv(c->n);
    HIPCHK(c, hipMemcpy(nv.data(), c->V.nviol, sizeof(long long) * c->n, hipMemcpyDeviceToHost));
    for (long long x : nv)
      if (x) return fail(c, MD_ERR_BOUND, "an acceptance probability exceeded 1 (rate bound violated)");
  }
  return MD_OK;
}

extern "C" int md_sync(md_ctx *c) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  return settle(c);
}

extern "C" int md_observables(md_ctx *c, uint32_t flags, md_obs *o) {
  if (!c || !o) return fail(c, MD_ERR_ARG, "null argument");
  memset(o, 0, sizeof(*o));
  int rc = settle(c);
  int nb = 0;
  HIPCHK(c, launch_ke(c->V, c->d_scratch, &nb, c->stream));
  std::vector<double> part(nb);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->d_scratch, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ke = 0.0;
  for (double x : part) ke += x;
  o->step = c->step;
  o->time = c->step * c->par.dt;
  o->ke = ke;
  o->temperature = 2.0 * ke / (3.0 * c->n * c->kB);
  std::vector<long long> a(c->n), b(c->n), v(c->n);
  std::vector<unsigned long long> hsh(c->n);
  HIPCHK(c, hipMemcpy(a.data(), c->V.nprop, 8 * c->n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(b.data(), c->V.nacc, 8 * c->n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(v.data(), c->V.nviol, 8 * c->n, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(hsh.data(), c->V.hash, 8 * c->n, hipMemcpyDeviceToHost));
  uint64_t H = 0xcbf29ce484222325ull;
  for (int i = 0; i < c->n; ++i) {
    o->n_prop += a[i]; o->n_acc += b[i]; o->n_bound_viol += v[i];
    for (int q = 0; q < 8; ++q) { H ^= (hsh[i] >> (8 * q)) & 0xffull; H *= 0x100000001b3ull; }
  }
  o->event_hash = H;
  o->n_rebuilds = (int64_t)c->ctl_host.n_rebuilds;
  o->n_zsampler_overflow = (int64_t)c->ctl_host.n_zs_overflow;
  o->n_list_errors = (int64_t)c->ctl_host.n_list_err;
  o->n_regrows = c->n_regrows;
  if (flags & MD_OBS_PE) {
    int rows = c->rows_valid;
    const bool split_rows = (rows & (ROW_SHORT | ROW_CAND)) == (ROW_SHORT | ROW_CAND);
    if (!split_rows && !(rows & ROW_FULL)) {
      int r2 = ensure_rows(c, ROW_FULL);
      if (r2 || (r2 = settle(c))) return r2;   // a regrow rebuilds the rows before they are used
      rows = c->rows_valid;
    }
    double4 *X = Xcur(c);
    double *es = c->d_scratch, *el = c->d_scratch + c->n, *dummy = c->d_scratch + 2 * c->n;
    double *eb = c->d_scratch + 3 * c->n;
    std::vector<double> hs(c->n), hl(c->n), hb(std::max(1, c->nbonds + c->nangles));
    double ps = 0.0, pl = 0.0, pb = 0.0;
    if ((rows & (ROW_SHORT | ROW_CAND)) == (ROW_SHORT | ROW_CAND) && !(rows & ROW_FULL)) {
      HIPCHK(c, launch_pair_energy(c->V, X, 0, es, dummy, c->stream));
      HIPCHK(c, hipMemcpyAsync(hs.data(), es, 8 * c->n, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, launch_pair_energy(c->V, X, 1, dummy, el, c->stream));
      HIPCHK(c, hipMemcpyAsync(hl.data(), el, 8 * c->n, hipMemcpyDeviceToHost, c->stream));
    } else {
      HIPCHK(c, launch_pair_energy(c->V, X, 2, es, el, c->stream));
      HIPCHK(c, hipMemcpyAsync(hs.data(), es, 8 * c->n, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(hl.data(), el, 8 * c->n, hipMemcpyDeviceToHost, c->stream));
    }
    if (c->nbonds + c->nangles) {
      HIPCHK(c, launch_bonded_energy(c->V, X, c->nbonds, c->nangles, eb, c->stream));
      HIPCHK(c, hipMemcpyAsync(hb.data(), eb, 8 * (c->nbonds + c->nangles), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->n; ++i) { ps += hs[i]; pl += hl[i]; }
    for (int t = 0; t < c->nbonds + c->nangles; ++t) pb += hb[t];
    o->pe_short = ps; o->pe_long = pl; o->pe_bonded = pb;
    if (c->spme) {
      const size_t ng = (size_t)c->V.pk[0] * c->V.pk[1] * c->V.pk[2];
      std::vector<double> he(ng + (size_t)c->n);
      HIPCHK(c, launch_pme_energy(c->V, X, c->d_pme_part, c->d_scratch, c->stream));
      HIPCHK(c, hipMemcpyAsync(he.data(), c->d_scratch, sizeof(double) * he.size(), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      double ek = 0.0, ex = 0.0;
      for (size_t m = 0; m < ng; ++m) ek += he[m];
      for (int i = 0; i < c->n; ++i) ex += he[ng + i];
      o->pe_recip = ek + c->ew_self + ex;
    } else if (c->ewald) {
      const size_t ne = (size_t)c->V.nk + (size_t)c->n;
      std::vector<double> he(ne);
      HIPCHK(c, launch_ewald_energy(c->V, X, c->d_spart, c->d_sfac, c->d_scratch, c->stream));
      HIPCHK(c, hipMemcpyAsync(he.data(), c->d_scratch, sizeof(double) * ne, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      double ek = 0.0, ex = 0.0;
      for (int k = 0; k < c->V.nk; ++k) ek += he[k];
      for (int i = 0; i < c->n; ++i) ex += he[c->V.nk + i];
      o->pe_recip = c->ew_ecoef * ek + c->ew_self + ex;
    }
  }
  return rc;
}

// ------------------------------------------------------------- state I/O
extern "C" int md_get_state(md_ctx *c, double *pos, double *vel) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  const int rc = settle(c);
  std::vector<double4> h(c->n);
  if (pos) {
    HIPCHK(c, hipMemcpyAsync(h.data(), Xcur(c), sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->n; ++i) { pos[3 * i] = h[i].x; pos[3 * i + 1] = h[i].y; pos[3 * i + 2] = h[i].z; }
  }
  if (vel) {
    HIPCHK(c, hipMemcpyAsync(h.data(), c->V.v, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->n; ++i) { vel[3 * i] = h[i].x; vel[3 * i + 1] = h[i].y; vel[3 * i + 2] = h[i].z; }
  }
  return rc;
}

extern "C" int md_set_state(md_ctx *c, const double *pos, const double *vel, int64_t step) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  (void)settle(c);   // pending steps finish (a new state also clears their errors)
  std::vector<double4> h(c->n);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (pos) {
    HIPCHK(c, hipMemcpy(h.data(), Xcur(c), sizeof(double4) * c->n, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n; ++i) { h[i].x = pos[3 * i]; h[i].y = pos[3 * i + 1]; h[i].z = pos[3 * i + 2]; }
    HIPCHK(c, hipMemcpy(Xcur(c), h.data(), sizeof(double4) * c->n, hipMemcpyHostToDevice));
    c->rows_valid = 0;
    c->fkind = -1;
    c->fb_valid = false;
    c->frec_valid = false;
    c->flong_valid = false;
  }
  if (vel) {
    HIPCHK(c, hipMemcpy(h.data(), c->V.v, sizeof(double4) * c->n, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n; ++i) { h[i].x = vel[3 * i]; h[i].y = vel[3 * i + 1]; h[i].z = vel[3 * i + 2]; }
    HIPCHK(c, hipMemcpy(c->V.v, h.data(), sizeof(double4) * c->n, hipMemcpyHostToDevice));
  }
  if (step >= 0) c->step = step;
  return MD_OK;
}

extern "C" int md_get_accel(md_ctx *c, int32_t kind, double *acc) {
  if (!c || !acc || kind < 0 || kind > 4) return fail(c, MD_ERR_ARG, "bad argument");
  if (kind == 4 && !c->ewald) return fail(c, MD_ERR_ARG, "no reciprocal-space forces without Ewald electrostatics");
  int rc = settle(c);
  if (rc) return rc;
  const double4 *src = c->V.fnb;
  if (kind == 2) {
    if ((rc = eval_bonded(c))) return rc;
    src = c->V.fb;
  } else if (kind == 4) {
    if ((rc = eval_recip(c))) return rc;
    src = c->V.frec;
  } else {
    if ((rc = ensure_rows(c, kind == 0 ? (ROW_SHORT | ROW_CAND) : ROW_FULL))) return rc;
    if ((rc = settle(c))) return rc;   // rows regrown before use if they overflowed
    if (kind == 3) {
      if (!c->V.flong) return fail(c, MD_ERR_ARG, "long real-space forces need Ewald electrostatics");
      if ((rc = eval_long(c))) return rc;
      src = c->V.flong;
    } else if ((rc = eval_nb(c, kind))) {
      return rc;
    }
  }
  std::vector<double4> f(c->n), v(c->n);
  HIPCHK(c, hipMemcpyAsync(f.data(), src, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(v.data(), c->V.v, sizeof(double4) * c->n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < c->n; ++i) {
    acc[3 * i] = f[i].x / v[i].w; acc[3 * i + 1] = f[i].y / v[i].w; acc[3 * i + 2] = f[i].z / v[i].w;
  }
  return MD_OK;
}

extern "C" int md_get_atom_stats(md_ctx *c, int64_t *np, int64_t *na, int64_t *nv, uint64_t *hash) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  const int rc = settle(c);
  if (np) HIPCHK(c, hipMemcpy(np, c->V.nprop, 8 * c->n, hipMemcpyDeviceToHost));
  if (na) HIPCHK(c, hipMemcpy(na, c->V.nacc, 8 * c->n, hipMemcpyDeviceToHost));
  if (nv) HIPCHK(c, hipMemcpy(nv, c->V.nviol, 8 * c->n, hipMemcpyDeviceToHost));
  if (hash) HIPCHK(c, hipMemcpy(hash, c->V.hash, 8 * c->n, hipMemcpyDeviceToHost));
  return rc;
}

extern "C" int md_get_events(md_ctx *c, md_event *buf, int64_t cap, int64_t *n) {
  if (!c || !n || cap < 0) return fail(c, MD_ERR_ARG, "bad argument");
  int rc = settle(c);
  const long long logged = (long long)c->ctl_host.n_events;
  const long long ne = std::min<long long>(logged, c->V.ev_cap);
  *n = ne;
  if (rc == MD_OK && logged > ne)
    rc = fail(c, MD_ERR_EVENTS, std::to_string(logged) + " jumps logged, the log holds " + std::to_string(ne));
  if (!buf || ne == 0) return rc;
  std::vector<MDEventDev> h(ne);
  HIPCHK(c, hipMemcpy(h.data(), c->V.ev, sizeof(MDEventDev) * ne, hipMemcpyDeviceToHost));
  std::sort(h.begin(), h.end(), [](const MDEventDev &a, const MDEventDev &b) {
    if (a.step != b.step) return a.step < b.step;
    if (a.phase != b.phase) return a.phase < b.phase;
    if (a.atom != b.atom) return a.atom < b.atom;
    return a.proposal < b.proposal;
  });
  for (long long e = 0; e < std::min<long long>(ne, cap); ++e) {
    buf[e].step = h[e].step; buf[e].phase = h[e].phase; buf[e].atom = h[e].atom;
    buf[e].partner = h[e].partner; buf[e].proposal = h[e].proposal;
  }
  return rc;
}

extern "C" int md_rdf(md_ctx *c, int32_t ta, int32_t tb, double r_max, int32_t n_bins, double *hist) {
  if (!c || !hist || n_bins <= 0 || !(r_max > 0.0) || ta < 0 || tb < 0 || ta >= c->nt || tb >= c->nt)
    return fail(c, MD_ERR_ARG, "bad argument");
  const int rc = settle(c);
  if (c->hist_n < n_bins) {   // through the context's allocator, kept for later calls
    if (c->d_hist) dfree(c, c->d_hist);
    c->d_hist = dalloc<unsigned long long>(c, (size_t)n_bins);
    c->hist_n = c->d_hist ? n_bins : 0;
    if (!c->d_hist) return fail(c, MD_ERR_OOM, c->err);
  }
  HIPCHK(c, launch_fill_u64(c->d_hist, n_bins, 0ull, c->stream));
  HIPCHK(c, launch_rdf(c->V, Xcur(c), c->d_rep_off, ta, tb, r_max, n_bins, c->d_hist, c->stream));
  std::vector<unsigned long long> h(n_bins);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->d_hist, sizeof(unsigned long long) * n_bins, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int b = 0; b < n_bins; ++b) hist[b] = (double)h[b];
  return rc;
}

// Velocity trace: the ring lives in the context's device memory; O ops take
// consecutive record indices while it is active (add_O), and graph replay is
// off meanwhile (a captured graph would repeat its record indices).
extern "C" int md_trace_velocities(md_ctx *c, int32_t n_atoms, int64_t capacity) {
  if (!c || n_atoms < 0 || n_atoms > c->n || (n_atoms > 0 && capacity < 1))
    return fail(c, MD_ERR_ARG, "trace: need 0 <= n_atoms <= N and capacity >= 1");
  const int rc = settle(c);   // pending steps (and replays) record into the old ring
  if (c->V.trace) dfree(c, c->V.trace);
  c->V.trace = nullptr;
  c->V.ntrace = 0;
  c->V.trace_cap = 0;
  c->trace_n = 0;
  if (n_atoms == 0) return rc;
  if ((double)n_atoms * (double)capacity > 4.0e9)
    return fail(c, MD_ERR_ARG, "trace: n_atoms x capacity above 4e9 records");
  c->V.trace = dalloc<double4>(c, (size_t)n_atoms * (size_t)capacity);
  if (!c->V.trace) return fail(c, MD_ERR_OOM, "trace: " + c->err);
  c->V.ntrace = n_atoms;
  c->V.trace_cap = capacity;
  return rc;
}

extern "C" int md_get_trace(md_ctx *c, double *out, int64_t max_records, int64_t *n_out, int64_t *n_recorded) {
  if (!c || !c->V.trace || max_records < 0 || (max_records > 0 && !out))
    return fail(c, MD_ERR_ARG, "trace: no active trace, or bad output");
  const int rc = settle(c);
  const int64_t cap = c->V.trace_cap, tn = c->trace_n, na = c->V.ntrace;
  const int64_t k = std::min(max_records, std::min(tn, cap));
  std::vector<double4> buf((size_t)(k * na));
  for (int64_t r = 0; r < k; ++r) {   // record tn - k + r sits in slot (tn - k + r) % cap
    const int64_t slot = (tn - k + r) % cap;
    HIPCHK(c, hipMemcpyAsync(buf.data() + r * na, c->V.trace + slot * na, sizeof(double4) * na,
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t q = 0; q < k * na; ++q) {
    out[3 * q] = buf[q].x; out[3 * q + 1] = buf[q].y; out[3 * q + 2] = buf[q].z;
  }
  if (n_out) *n_out = k;
  if (n_recorded) *n_recorded = tn;
  return rc;
}

// Allocation-free variant of md_rdf: the counts live in the library's static
// device scratch array (per device, at the address looked up at creation),
// cleared by a fill kernel, converted to doubles on the device and copied
// straight into the caller's array. No device or host allocation; rows that
// outgrew their capacity are not regrown here (that allocates).
extern "C" int md_rdf_noalloc(md_ctx *c, int32_t ta, int32_t tb, double r_max, int32_t n_bins, double *hist) {
  if (!c || !hist || n_bins <= 0 || !(r_max > 0.0) || ta < 0 || tb < 0 || ta >= c->nt || tb >= c->nt)
    return fail(c, MD_ERR_ARG, "bad argument");
  if (n_bins > MD_RDF_NOALLOC_MAX_BINS)
    return fail(c, MD_ERR_ARG, "n_bins above the static scratch of md_rdf_noalloc (" +
                                   std::to_string(MD_RDF_NOALLOC_MAX_BINS) + " bins)");
  unsigned long long *sp = rdf_scratch_ptr(c->dev);
  if (!sp) return fail(c, MD_ERR_HIP, "static scratch not set up on this device");
  HIPCHK(c, hipMemcpyAsync(&c->ctl_host, c->V.ctl, sizeof(MDCtl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->ctl_host.ovf_short || c->ctl_host.ovf_long || c->ctl_host.ovf_queue)
    return fail(c, MD_ERR_CAPACITY, "neighbour rows outgrew their capacity since the last synchronisation; "
                                    "md_sync regrows them (it allocates) and must run first");
  HIPCHK(c, launch_rdf_noalloc(c->V, Xcur(c), c->d_rep_off, ta, tb, r_max, n_bins, sp, c->stream));
  HIPCHK(c, hipMemcpyAsync(hist, (const double *)(sp + MD_RDF_NOALLOC_MAX_BINS), sizeof(double) * n_bins,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->snap.valid = false;   // a synchronisation with no overflow pending: the state is good
  c->journal.clear();
  return report_flags(c);
}

extern "C" int md_get_cand_row(md_ctx *c, int32_t i, int32_t *j, int32_t *img, int32_t cap, int32_t *n,
                               int32_t *seg) {
  if (!c || !n || i < 0 || i >= c->n || cap < 0) return fail(c, MD_ERR_ARG, "bad argument");
  int rc = settle(c);
  if (rc || (rc = ensure_rows(c, ROW_SHORT | ROW_CAND)) || (rc = settle(c))) return rc;
  int cnt = 0;
  HIPCHK(c, hipMemcpy(&cnt, c->V.ccnt + i, sizeof(int), hipMemcpyDeviceToHost));
  *n = cnt;
  const int m = std::min(cnt, cap);
  if ((j || img) && m > 0) {
    std::vector<int> e(m);
    HIPCHK(c, hipMemcpy(e.data(), c->V.crow + (size_t)i * c->V.cap_c, sizeof(int) * m, hipMemcpyDeviceToHost));
    const int r = (int)(std::upper_bound(c->rep_off.begin(), c->rep_off.end(), i) - c->rep_off.begin()) - 1;
    const double *L = c->box.data() + 3 * (size_t)r;
    const double rout = c->V.rout;
    const bool has_img = L[0] < 2.0 * rout || L[1] < 2.0 * rout || L[2] < 2.0 * rout;
    for (int q = 0; q < m; ++q) {
      if (j) j[q] = e[q] & 0x7fffff;
      if (img) img[q] = has_img ? (int32_t)((uint32_t)e[q] >> 23) : -1;
    }
  }
  if (seg) HIPCHK(c, hipMemcpy(seg, c->V.segst + (size_t)i * (c->S + 1), sizeof(int) * (c->S + 1),
                               hipMemcpyDeviceToHost));
  return MD_OK;
}

extern "C" int md_get_row_counts(md_ctx *c, int32_t which, int32_t *counts) {
  if (!c || !counts || which < 0 || which > 2) return fail(c, MD_ERR_ARG, "bad argument");
  int want = which == 0 ? ROW_SHORT : (which == 1 ? ROW_FULL : ROW_CAND);
  int rc = settle(c);
  if (rc || (rc = ensure_rows(c, want == ROW_FULL ? ROW_FULL : (ROW_SHORT | ROW_CAND))) || (rc = settle(c)))
    return rc;
  const int *src = which == 0 ? c->V.scnt : (which == 1 ? c->V.fcnt : c->V.ccnt);
  HIPCHK(c, hipMemcpy(counts, src, sizeof(int) * c->n, hipMemcpyDeviceToHost));
  return MD_OK;
}

extern "C" int md_run_phase(md_ctx *c, int32_t which, int32_t phase, double h) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  if (which != 'C' && which != 'J' && which != 'O') return fail(c, MD_ERR_ARG, "which must be 'C', 'J' or 'O'");
  return step_call(c, {CALL_PHASE, 0, which, phase, h});
}

static int run_phase(md_ctx *c, int which, int phase, double h) {
  int rc = ensure_forces(c, MODE_JUMP);
  if (rc) return rc;
  ProgBuilder b;
  if (which == 'C') {
    if (c->par.jump_coul == MD_JUMP_NONE || c->par.jump_coul == MD_JUMP_BOUNCE)
      return fail(c, MD_ERR_ARG, "no C-step jumps configured");
    MDOp o = op_base(OP_C, h); o.phase = phase; o.step = c->step; o.flags = 0; b.add(o);
  } else if (which == 'J') {
    add_J(b, phase, h, c->step);
  } else if (which == 'O') {
    add_O(c, b, h, 0, c->step);
  } else {
    return fail(c, MD_ERR_ARG, "which must be 'C', 'J' or 'O'");
  }
  return run_prog(c, b);
}

extern "C" int md_profile(md_ctx *c, int32_t enable) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  prof_collect(c);
  c->prof = enable != 0;
  for (int k = 0; k < MD_K_COUNT; ++k) { c->tm.tot_ms[k] = 0.0; c->tm.launches[k] = 0; }
  return MD_OK;
}

extern "C" int md_profile_read(md_ctx *c, int32_t kid, double *total_ms, int64_t *launches) {
  if (!c || kid < 0 || kid >= MD_K_COUNT) return fail(c, MD_ERR_ARG, "bad argument");
  prof_collect(c);
  if (total_ms) *total_ms = c->tm.tot_ms[kid];
  if (launches) *launches = c->tm.launches[kid];
  return MD_OK;
}

extern "C" int md_counters(md_ctx *c, int64_t *pairs_last, int64_t *proposals_total) {
  if (!c) return fail(c, MD_ERR_ARG, "null context");
  const int rc = settle(c);
  if (pairs_last) {
    *pairs_last = -1;
    if (c->fkind == 0 || c->fkind == 1) {
      int which = c->fkind;
      int need = which == 0 ? ROW_SHORT : ROW_FULL;
      if ((c->rows_valid & need) == need) {
        unsigned long long *cnt = (unsigned long long *)c->d_scratch;
        HIPCHK(c, launch_fill_u64(cnt, 1, 0ull, c->stream));
        HIPCHK(c, launch_count_pairs(c->V, Xcur(c), which, which == 0 ? c->split.r_s : c->split.r_c, cnt,
                                     c->stream));
        unsigned long long h = 0;
        HIPCHK(c, hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *pairs_last = (int64_t)h;
      }
    }
  }
  if (proposals_total) {
    std::vector<long long> a(c->n);
    HIPCHK(c, hipMemcpy(a.data(), c->V.nprop, 8 * c->n, hipMemcpyDeviceToHost));
    long long s = 0;
    for (long long x : a) s += x;
    *proposals_total = s;
  }
  return rc;
}

// ---------------------------------------------------------- diagnostics
extern "C" int md_theta_screen_error(double eta_lo, double eta_hi, int32_t n, double *max_rel_err) {
  if (n < 2 || !(eta_lo < eta_hi) || !max_rel_err) return fail(nullptr, MD_ERR_ARG, "need n >= 2, eta_lo < eta_hi");
  unsigned long long *d = nullptr;
  if (hipMalloc(&d, sizeof(unsigned long long)) != hipSuccess) return fail(nullptr, MD_ERR_OOM, "device allocation failed");
  unsigned long long h = 0;
  hipError_t e = hipMemset(d, 0, sizeof(h));
  if (e == hipSuccess) e = launch_theta_screen_err(eta_lo, eta_hi, n, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(&h, d, sizeof(h), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) return fail(nullptr, MD_ERR_HIP, std::string("theta screen check: ") + hipGetErrorString(e));
  double v;
  std::memcpy(&v, &h, sizeof(v));
  *max_rel_err = v;
  return MD_OK;
}

// ------------------------------------------------------------- autotuner
// Launch and list settings are searched by timing: each trial creates a
// context with one setting from the caller's state, runs `warm` untimed steps
// (rows built, graphs captured) and times `steps` steps with HIP events on
// the context's stream. Coordinate descent over chain lanes (jump schemes),
// list skin, ring count (jump schemes) and graph replay (single-step schemes),
// then lanes once more at the chosen skin and rings. Results are cached per
// process by a fingerprint of the system's shape and the run settings.
namespace {
struct TuneEntry { md_split sp; md_params p; double ms; std::vector<md_tune_trial> trials; };
std::vector<std::pair<uint64_t, TuneEntry>> g_tune_cache;

uint64_t fnv_mix(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t q = 0; q < n; ++q) { h ^= b[q]; h *= 0x100000001b3ull; }
  return h;
}

uint64_t tune_key(const md_system *s, const md_split *sp, const md_params *p, int scheme, int steps) {
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv_mix(h, &s->n_atoms, sizeof(int32_t));
  h = fnv_mix(h, &s->n_replicas, sizeof(int32_t));
  h = fnv_mix(h, &s->n_types, sizeof(int32_t));
  h = fnv_mix(h, s->box, sizeof(double) * 3 * (size_t)s->n_replicas);
  if (s->replica_offset) h = fnv_mix(h, s->replica_offset, sizeof(int32_t) * (size_t)(s->n_replicas + 1));
  h = fnv_mix(h, sp, sizeof(md_split));
  const double pk[4] = {p->dt, p->gamma, p->kT, p->eps};
  const int32_t pi[7] = {p->jump_lj, p->jump_coul, p->precision, p->respa_inner, p->rebuild_every, scheme,
                          p->chain_order};
  h = fnv_mix(h, pk, sizeof(pk));
  h = fnv_mix(h, pi, sizeof(pi));
  return fnv_mix(h, &steps, sizeof(steps));
}
}  // namespace

static int run_scheme(md_ctx *c, int scheme, int64_t n) {
  switch (scheme) {
    case MD_SCHEME_BAOAB: return md_step_baoab(c, n);
    case MD_SCHEME_JUMP: return md_step_jump(c, n);
    case MD_SCHEME_JUMP_RESPA: return md_step_jump_respa(c, n);
    case MD_SCHEME_BAOAB_RESPA: return md_step_baoab_respa(c, n);
  }
  return fail(c, MD_ERR_ARG, "unknown scheme");
}

// one trial: ms per step of `scheme` with this split and these parameters
static int tune_trial(const md_system *s, const md_split &sp, const md_params &p, void *stream,
                      const md_allocator *alloc, int scheme, int warm, int steps, double *ms) {
  md_ctx *c = nullptr;
  int rc = md_create(s, &sp, &p, stream, alloc, &c);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(c, MD_ERR_HIP, "hipEventCreate");
  if (!rc) rc = run_scheme(c, scheme, warm);
  if (!rc) rc = md_sync(c);
  if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(c, MD_ERR_HIP, "hipEventRecord");
  if (!rc) rc = run_scheme(c, scheme, steps);
  if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(c, MD_ERR_HIP, "hipEventRecord");
  if (!rc) rc = md_sync(c);
  float f = 0.0f;
  if (!rc && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = fail(c, MD_ERR_HIP, "hipEventElapsedTime");
  if (!rc) *ms = (double)f / steps;
  if (rc) g_create_error = c->err;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  md_destroy(c);
  return rc;
}

extern "C" int md_tune(const md_system *s, const md_split *sp, const md_params *p, void *stream,
                       const md_allocator *alloc, int32_t scheme, int32_t steps, md_split *sp_out,
                       md_params *p_out, double *ms_out, md_tune_trial *trials, int32_t cap, int32_t *n_trials) {
  if (!s || !sp || !p || !sp_out || !p_out || steps < 1 || cap < 0 ||
      scheme < MD_SCHEME_BAOAB || scheme > MD_SCHEME_BAOAB_RESPA)
    return fail(nullptr, MD_ERR_ARG, "md_tune: bad argument");
  int rc = validate(s, sp, p);
  if (rc) return rc;
  const uint64_t key = tune_key(s, sp, p, scheme, steps);
  const TuneEntry *hit = nullptr;
  for (const auto &e : g_tune_cache)
    if (e.first == key) hit = &e.second;
  TuneEntry res;
  if (hit) {
    res = *hit;
  } else {
    const bool jumps = scheme == MD_SCHEME_JUMP || scheme == MD_SCHEME_JUMP_RESPA;
    const bool graphs = (scheme == MD_SCHEME_JUMP || scheme == MD_SCHEME_BAOAB) && p->rebuild_every == 0;
    const int warm = std::max(10, steps / 4);
    double Lmin = s->box[0];
    for (int q = 0; q < 3 * s->n_replicas; ++q) Lmin = std::min(Lmin, s->box[q]);
    // ring_width spans the candidate distances [r_s - w - skin, r_c + skin)
    auto with = [&](double skin, int rings) {
      md_split t = *sp;
      t.skin = skin;
      t.n_rings = rings;
      t.ring_width = rings > 1 ? ((t.r_c + skin) - (t.r_s - t.switch_width - skin)) / rings : 0.0;
      return t;
    };
    md_split best_sp = *sp;
    md_params best_p = *p;
    best_p.graph_steps = graphs ? p->graph_steps : 0;
    double best = INFINITY;
    auto trial = [&](const md_split &t, const md_params &q) -> bool {
      if (validate(s, &t, &q) != MD_OK || (q.graph_steps & 1)) return false;
      double ms = 0.0;
      if (tune_trial(s, t, q, stream, alloc, scheme, warm, steps, &ms) != MD_OK) return false;
      res.trials.push_back(md_tune_trial{q.chain_lanes, t.skin, t.n_rings, q.graph_steps, q.chain_order, ms});
      if (ms < best) { best = ms; best_sp = t; best_p = q; return true; }
      return false;
    };
    auto tune_lanes = [&]() {
      if (!jumps) return;
      const md_split t = best_sp;
      const md_params base = best_p;
      for (int g : {0, 1, 2, 4, 8, 16}) {
        if (g == base.chain_lanes) continue;
        md_params q = base;
        q.chain_lanes = g;
        trial(t, q);
      }
    };
    trial(best_sp, best_p);   // the caller's setting
    if (!std::isfinite(best)) return fail(nullptr, MD_ERR_ARG, "md_tune: the caller's setting does not run: " +
                                                                  g_create_error);
    tune_lanes();
    if (jumps && s->n_replicas > 1) {
      const md_split t0 = best_sp;
      const md_params base = best_p;
      for (int o : {1, 2}) {
        if (o == base.chain_order) continue;
        md_params q = base;
        q.chain_order = o;
        trial(t0, q);
      }
    }
    {
      const md_split t0 = best_sp;
      const md_params q = best_p;
      for (double f : {0.6, 0.8, 1.2, 1.5, 2.0}) {
        const double skin = sp->skin * f;
        if (!(skin > 0.0) || !(Lmin > sp->r_c + skin)) continue;
        trial(with(skin, t0.n_rings), q);
      }
    }
    if (jumps) {
      const md_split t0 = best_sp;
      const md_params q = best_p;
      const int nr0 = std::max(1, sp->n_rings);
      for (int rings : {nr0 / 2, (3 * nr0) / 2, 2 * nr0}) {
        if (rings < 1 || rings == t0.n_rings || s->n_types * rings > 32) continue;
        trial(with(t0.skin, rings), q);
      }
    }
    if (graphs) {
      const md_split t0 = best_sp;
      const md_params base = best_p;
      for (int gs : {0, 10, 20, 50}) {
        if (gs == base.graph_steps) continue;
        md_params q = base;
        q.graph_steps = gs;
        trial(t0, q);
      }
    }
    if (best_sp.skin != sp->skin || best_sp.n_rings != sp->n_rings) tune_lanes();
    res.sp = best_sp;
    res.p = best_p;
    res.ms = best;
    g_tune_cache.emplace_back(key, res);
  }
  *sp_out = res.sp;
  *p_out = res.p;
  if (ms_out) *ms_out = res.ms;
  if (n_trials) *n_trials = (int32_t)res.trials.size();
  if (trials)
    for (int32_t q = 0; q < std::min<int32_t>(cap, (int32_t)res.trials.size()); ++q) trials[q] = res.trials[q];
  return MD_OK;
}
