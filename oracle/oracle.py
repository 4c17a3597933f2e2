"""ctypes binding of the CPU FP64 oracle (libjumpmd_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of bench.py. The GPU library never imports this module and this
module never imports the GPU package. System/split/params objects are taken
by duck typing (any object with the documented attributes).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjumpmd_oracle.so")
# JUMPMD_ORACLE_LIBRARY may name another build of the oracle (the mutation
# tests load builds with a planted mistake this way)
_LIB_ENV = "JUMPMD_ORACLE_LIBRARY"

JUMP_NONE, JUMP_BPS, JUMP_MRZ_CONST, JUMP_MRZ_ADAPTIVE, JUMP_BOUNCE, JUMP_IN_C = 0, 1, 2, 3, 4, 5
PH_O, PH_J1, PH_J2, PH_C1, PH_C2 = 1, 2, 3, 4, 5
F_SHORT, F_FULL, F_BONDED, F_LONG, F_RECIP = 0, 1, 2, 3, 4
COUL_DSF, COUL_EWALD, COUL_SPME = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


class OrcSystem(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_types", C.c_int32),
                ("pos", _dp), ("vel", _dp), ("mass", _dp), ("charge", _dp),
                ("type", _ip), ("lj_eps", _dp), ("lj_sigma", _dp),
                ("box", C.c_double * 3),
                ("n_bonds", C.c_int32), ("bond_ij", _ip), ("bond_k", _dp), ("bond_r0", _dp),
                ("n_angles", C.c_int32), ("angle_ijk", _ip), ("angle_k", _dp), ("angle_t0", _dp),
                ("excl_ptr", _ip), ("excl_j", _ip),
                ("coulomb_k", C.c_double), ("accel_factor", C.c_double), ("kB", C.c_double)]


class OrcSplit(C.Structure):
    _fields_ = [("r_s", C.c_double), ("r_c", C.c_double), ("switch_width", C.c_double),
                ("skin", C.c_double), ("coulomb_alpha", C.c_double),
                ("n_rings", C.c_int32), ("ring_width", C.c_double),
                ("coulomb_kind", C.c_int32), ("ewald_kmax", C.c_int32),
                ("pme_grid", C.c_int32 * 3), ("pme_order", C.c_int32)]


class OrcParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
                ("seed", C.c_uint64), ("replica", C.c_uint64),
                ("jump_lj", C.c_int32), ("jump_coul", C.c_int32), ("eps", C.c_double),
                ("respa_inner", C.c_int32), ("rebuild_every", C.c_int32),
                ("log_events", C.c_int32), ("respa_outer", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get(_LIB_ENV, LIB_PATH)
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            from oracle import build_oracle
            build_oracle.build()
        L = C.CDLL(path)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcSystem), C.POINTER(OrcSplit), C.POINTER(OrcParams),
                                 C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        for fn in ("orc_step_baoab", "orc_step_jump", "orc_step_jump_respa", "orc_step_baoab_respa",
                   "orc_step_jump_respa1", "orc_step_baoab_respa1"):
            getattr(L, fn).argtypes = [C.c_void_p, C.c_int64]
            getattr(L, fn).restype = C.c_int
        L.orc_get_state.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_int64]
        for fn in ("orc_step_index", "orc_n_rebuilds", "orc_n_zsampler_overflow",
                   "orc_n_list_errors", "orc_n_events"):
            getattr(L, fn).argtypes = [C.c_void_p]
            getattr(L, fn).restype = C.c_int64
        L.orc_atom_stats.argtypes = [C.c_void_p, _lp, _lp, _lp, _up]
        L.orc_zsampler_regimes.argtypes = [C.c_void_p, _lp]
        L.orc_event_hash.argtypes = [C.c_void_p]
        L.orc_event_hash.restype = C.c_uint64
        L.orc_get_events.argtypes = [C.c_void_p, _lp]
        L.orc_energies.argtypes = [C.c_void_p, _dp]
        L.orc_accel.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_rdf.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int, _dp]
        L.orc_build_lists.argtypes = [C.c_void_p]
        L.orc_n_segments.argtypes = [C.c_void_p]
        L.orc_n_segments.restype = C.c_int32
        L.orc_cand_count.argtypes = [C.c_void_p, C.c_int32]
        L.orc_cand_count.restype = C.c_int64
        L.orc_cand_row.argtypes = [C.c_void_p, C.c_int32, _ip, _ip]
        L.orc_seg_start.argtypes = [C.c_void_p, C.c_int32, _ip]
        L.orc_pairs_within.argtypes = [C.c_void_p, C.c_double, _ip, C.c_int64]
        L.orc_pairs_within.restype = C.c_int64
        L.orc_bounds.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_set_bound_scale.argtypes = [C.c_void_p, C.c_double]
        L.orc_phase_c.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_int]
        L.orc_phase_j.argtypes = [C.c_void_p, C.c_int32, C.c_double]
        L.orc_phase_o.argtypes = [C.c_void_p, C.c_double, C.c_int32]
        L.orc_philox4x32.argtypes = [_u32p, _u32p, _u32p]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_event_mix.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int32]
        L.orc_event_mix.restype = C.c_uint64
        L.orc_theta.argtypes = [C.c_double]
        L.orc_theta.restype = C.c_double
        L.orc_zsample.argtypes = [C.c_double, C.c_uint64, C.c_uint64, C.c_int64, C.c_int64,
                                  C.c_int32, C.c_int64, _ip]
        L.orc_zsample.restype = C.c_double
        L.orc_pair_terms.argtypes = [C.c_double] * 9 + [_dp]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


# ------------------------------------------------------------------ primitives
def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def u01(w):
    return lib().orc_u01(C.c_uint32(int(w)))


def event_mix(h, step, phase, j):
    return lib().orc_event_mix(C.c_uint64(int(h)), int(step), int(phase), int(j))


def theta(eta):
    return lib().orc_theta(float(eta))


def zsample(eta, seed=1, replica=0, step=0, atom=0, phase=PH_C1, k=0):
    it = C.c_int32(0)
    z = lib().orc_zsample(float(eta), seed, replica, step, atom, phase, k, C.byref(it))
    return z, it.value


def pair_terms(r, eps, sigma, qq, coulomb_k, alpha, r_s, w, r_c):
    out = np.zeros(6)
    lib().orc_pair_terms(r, eps, sigma, qq, coulomb_k, alpha, r_s, w, r_c, _ptr(out, _dp))
    return out


# ------------------------------------------------------------------ simulation
class OracleSim:
    """One replica of a system advanced by the oracle."""

    def __init__(self, system, split, params, replica=0):
        self._keep = []
        s = system

        def arr(x, dt):
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a

        pos, vel = arr(s.pos, np.float64), arr(s.vel, np.float64)
        self.n = s.n_atoms
        sy = OrcSystem()
        sy.n_atoms, sy.n_types = s.n_atoms, s.n_types
        sy.pos, sy.vel = _ptr(pos, _dp), _ptr(vel, _dp)
        sy.mass = _ptr(arr(s.mass, np.float64), _dp)
        sy.charge = _ptr(arr(s.charge, np.float64), _dp)
        sy.type = _ptr(arr(s.type, np.int32), _ip)
        sy.lj_eps = _ptr(arr(s.lj_eps, np.float64), _dp)
        sy.lj_sigma = _ptr(arr(s.lj_sigma, np.float64), _dp)
        for c in range(3):
            sy.box[c] = float(s.box[c])
        sy.n_bonds = len(s.bond_k)
        sy.bond_ij = _ptr(arr(s.bond_ij, np.int32), _ip)
        sy.bond_k = _ptr(arr(s.bond_k, np.float64), _dp)
        sy.bond_r0 = _ptr(arr(s.bond_r0, np.float64), _dp)
        sy.n_angles = len(s.angle_k)
        sy.angle_ijk = _ptr(arr(s.angle_ijk, np.int32), _ip)
        sy.angle_k = _ptr(arr(s.angle_k, np.float64), _dp)
        sy.angle_t0 = _ptr(arr(s.angle_t0, np.float64), _dp)
        if s.excl_ptr is not None:
            sy.excl_ptr = _ptr(arr(s.excl_ptr, np.int32), _ip)
            sy.excl_j = _ptr(arr(s.excl_j, np.int32), _ip)
        sy.coulomb_k, sy.accel_factor, sy.kB = s.coulomb_k, s.accel_factor, s.kB
        sp = OrcSplit(split.r_s, split.r_c, split.switch_width, split.skin,
                      split.coulomb_alpha, split.n_rings, split.ring_width,
                      getattr(split, "coulomb_kind", 0), getattr(split, "ewald_kmax", 0),
                      (C.c_int32 * 3)(*getattr(split, "pme_grid", (0, 0, 0))), getattr(split, "pme_order", 0))
        pa = OrcParams(params.dt, params.gamma, params.kT, params.seed, replica,
                       params.jump_lj, params.jump_coul, params.eps, params.respa_inner,
                       params.rebuild_every, params.log_events, getattr(params, "respa_outer", 1))
        err = C.create_string_buffer(256)
        self._h = lib().orc_create(C.byref(sy), C.byref(sp), C.byref(pa), err, 256)
        if not self._h:
            raise ValueError("oracle create failed: " + err.value.decode())

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    # stepping
    def step_baoab(self, n):
        lib().orc_step_baoab(self._h, n)

    def step_jump(self, n):
        lib().orc_step_jump(self._h, n)

    def step_jump_respa(self, n):
        lib().orc_step_jump_respa(self._h, n)

    def step_baoab_respa(self, n):
        lib().orc_step_baoab_respa(self._h, n)

    def step_jump_respa1(self, n):
        if lib().orc_step_jump_respa1(self._h, n) != 0:
            raise RuntimeError("JUMP-RESPA1 needs Ewald electrostatics")

    def step_baoab_respa1(self, n):
        if lib().orc_step_baoab_respa1(self._h, n) != 0:
            raise RuntimeError("BAOAB-RESPA1 needs Ewald electrostatics")

    # state
    def state(self):
        x = np.zeros(3 * self.n)
        v = np.zeros(3 * self.n)
        lib().orc_get_state(self._h, _ptr(x, _dp), _ptr(v, _dp))
        return x.reshape(-1, 3), v.reshape(-1, 3)

    def set_state(self, pos=None, vel=None, step=-1):
        p = None if pos is None else np.ascontiguousarray(pos, dtype=np.float64).ravel()
        v = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).ravel()
        lib().orc_set_state(self._h, _ptr(p, _dp), _ptr(v, _dp), step)

    @property
    def step_index(self):
        return lib().orc_step_index(self._h)

    @property
    def n_rebuilds(self):
        return lib().orc_n_rebuilds(self._h)

    @property
    def n_zsampler_overflow(self):
        return lib().orc_n_zsampler_overflow(self._h)

    @property
    def n_list_errors(self):
        return lib().orc_n_list_errors(self._h)

    def zsampler_regimes(self):
        """Accepted MRZ jumps by Z-sampler regime: eta < -1, -1 <= eta <= 0, eta > 0."""
        out = np.zeros(3, np.int64)
        lib().orc_zsampler_regimes(self._h, _ptr(out, _lp))
        return out

    def atom_stats(self):
        n = self.n
        a, b, c = (np.zeros(n, np.int64) for _ in range(3))
        h = np.zeros(n, np.uint64)
        lib().orc_atom_stats(self._h, _ptr(a, _lp), _ptr(b, _lp), _ptr(c, _lp), _ptr(h, _up))
        return {"n_prop": a, "n_acc": b, "n_viol": c, "hash": h}

    def event_hash(self):
        return lib().orc_event_hash(self._h)

    def events(self):
        """Accepted jumps (step, phase, i, j, k), sorted by (step, phase, i, k)."""
        n = lib().orc_n_events(self._h)
        buf = np.zeros(5 * n, np.int64)
        if n:
            lib().orc_get_events(self._h, _ptr(buf, _lp))
        ev = buf.reshape(-1, 5)
        return ev[np.lexsort((ev[:, 4], ev[:, 2], ev[:, 1], ev[:, 0]))]

    def energies(self):
        out = np.zeros(7)
        lib().orc_energies(self._h, _ptr(out, _dp))
        return dict(zip(("ke", "T", "pe_short", "pe_long", "pe_bonded", "pe_full", "pe_recip"), out))

    def accel(self, kind):
        a = np.zeros(3 * self.n)
        lib().orc_accel(self._h, kind, _ptr(a, _dp))
        return a.reshape(-1, 3)

    def rdf_counts(self, ta, tb, r_max, n_bins):
        h = np.zeros(n_bins)
        lib().orc_rdf(self._h, ta, tb, r_max, n_bins, _ptr(h, _dp))
        return h

    # lists
    def build_lists(self):
        lib().orc_build_lists(self._h)

    @property
    def n_segments(self):
        return lib().orc_n_segments(self._h)

    def cand_row(self, i):
        return self.cand_row_images(i)[0]

    def cand_row_images(self, i):
        """Candidate row of atom i: partners j and the lattice vector n of
        each candidate image (displacement x_i - x_j - n L), shape [len, 3]."""
        n = lib().orc_cand_count(self._h, i)
        j = np.zeros(n, np.int32)
        img = np.zeros((n, 3), np.int32)
        if n:
            lib().orc_cand_row(self._h, i, _ptr(j, _ip), _ptr(img, _ip))
        return j, img

    def seg_start(self, i):
        s = np.zeros(self.n_segments + 1, np.int32)
        lib().orc_seg_start(self._h, i, _ptr(s, _ip))
        return s

    def pairs_within(self, rcut):
        cnt = lib().orc_pairs_within(self._h, rcut, None, 0)
        ij = np.zeros(2 * max(cnt, 1), np.int32)
        lib().orc_pairs_within(self._h, rcut, _ptr(ij, _ip), cnt)
        return ij[: 2 * cnt].reshape(-1, 2)

    def bounds(self, n_types, n_rings):
        m = n_types * n_types * n_rings
        a, b, q = np.zeros(m), np.zeros(m), np.zeros(n_types)
        lib().orc_bounds(self._h, _ptr(a, _dp), _ptr(b, _dp), _ptr(q, _dp))
        return a.reshape(n_types, n_types, n_rings), b.reshape(n_types, n_types, n_rings), q

    def set_bound_scale(self, scale):
        lib().orc_set_bound_scale(self._h, scale)

    # phases
    def phase_c(self, phase, h, a_kind=0):
        lib().orc_phase_c(self._h, phase, h, a_kind)

    def phase_j(self, phase, h):
        lib().orc_phase_j(self._h, phase, h)

    def phase_o(self, h, substep=0):
        lib().orc_phase_o(self._h, h, substep)
