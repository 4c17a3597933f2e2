"""ctypes binding of libjumpmd.so (C ABI in include/jumpmd.h).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of the library. PyTorch supplies the HIP stream and the device
memory (its caching allocator, through the md_allocator callbacks), so torch
owns every block the library uses. Importing this module raises if the
library has not been built, and there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjumpmd.so")

MD_OK, MD_ERR_ARG, MD_ERR_HIP, MD_ERR_BOUND, MD_ERR_LIST, MD_ERR_UNSTABLE, MD_ERR_OOM, MD_ERR_CAPACITY = \
    0, -1, -2, -3, -4, -5, -6, -7
MD_ERR_EVENTS = -8
MD_OBS_PE = 1
MD_K_LOCAL, MD_K_FORCE, MD_K_BONDED, MD_K_REBUILD, MD_K_CHAIN, MD_K_RECIP = 0, 1, 2, 3, 4, 5
PHASE = {"J1": 2, "J2": 3, "C1": 4, "C2": 5}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint64)


class MDSystem(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_types", C.c_int32), ("n_replicas", C.c_int32),
                ("pos", _dp), ("vel", _dp), ("mass", _dp), ("charge", _dp), ("type", _ip),
                ("lj_eps", _dp), ("lj_sigma", _dp), ("box", _dp), ("replica_offset", _ip),
                ("n_bonds", C.c_int32), ("bond_ij", _ip), ("bond_k", _dp), ("bond_r0", _dp),
                ("n_angles", C.c_int32), ("angle_ijk", _ip), ("angle_k", _dp), ("angle_t0", _dp),
                ("excl_ptr", _ip), ("excl_j", _ip),
                ("coulomb_k", C.c_double), ("accel_factor", C.c_double), ("kB", C.c_double)]


class MDSplit(C.Structure):
    _fields_ = [("r_s", C.c_double), ("r_c", C.c_double), ("switch_width", C.c_double),
                ("skin", C.c_double), ("coulomb_alpha", C.c_double),
                ("n_rings", C.c_int32), ("ring_width", C.c_double),
                ("coulomb_kind", C.c_int32), ("ewald_kmax", C.c_int32),
                ("pme_grid", C.c_int32 * 3), ("pme_order", C.c_int32)]


class MDParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("gamma", C.c_double), ("kT", C.c_double), ("seed", C.c_uint64),
                ("jump_lj", C.c_int32), ("jump_coul", C.c_int32), ("eps", C.c_double),
                ("precision", C.c_int32), ("rebuild_every", C.c_int32), ("respa_inner", C.c_int32),
                ("log_events", C.c_int32), ("strict_bounds", C.c_int32), ("chain_lanes", C.c_int32),
                ("graph_steps", C.c_int32), ("bound_scale", C.c_double), ("row_capacity", C.c_double),
                ("event_capacity", C.c_int64), ("chain_order", C.c_int32), ("respa_outer", C.c_int32)]


class MDObs(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("ke", C.c_double), ("temperature", C.c_double),
                ("pe_short", C.c_double), ("pe_long", C.c_double), ("pe_bonded", C.c_double),
                ("n_prop", C.c_int64), ("n_acc", C.c_int64), ("n_bound_viol", C.c_int64),
                ("n_rebuilds", C.c_int64), ("n_zsampler_overflow", C.c_int64),
                ("n_list_errors", C.c_int64), ("event_hash", C.c_uint64), ("n_regrows", C.c_int64),
                ("pe_recip", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class MDAllocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("release", _RELEASE_FN)]


class TorchAllocator:
    """md_allocator backed by PyTorch's caching allocator: every device block
    of a context is a torch allocation on the context's stream (torch owns
    it). Counts the bytes handed out (live and in total)."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else device
        self.bytes_live = 0
        self.bytes_total = 0
        self.n_blocks = 0

        def alloc(_ctx, nbytes, stream):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=int(stream or 0))
            except Exception:
                return None
            self.bytes_live += int(nbytes)
            self.bytes_total += int(nbytes)
            self.n_blocks += 1
            return p

        def release(_ctx, ptr, nbytes, _stream):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass
            self.bytes_live -= int(nbytes)

        self._fns = (_ALLOC_FN(alloc), _RELEASE_FN(release))   # kept alive with the contexts using them
        self.struct = MDAllocator(None, self._fns[0], self._fns[1])


class MDTuneTrial(C.Structure):
    _fields_ = [("chain_lanes", C.c_int32), ("skin", C.c_double), ("n_rings", C.c_int32),
                ("graph_steps", C.c_int32), ("chain_order", C.c_int32), ("ms_per_step", C.c_double)]


class MDEvent(C.Structure):
    _fields_ = [("step", C.c_int64), ("phase", C.c_int32), ("atom", C.c_int32),
                ("partner", C.c_int32), ("proposal", C.c_int32)]


EXPORTS = ["md_create", "md_destroy", "md_last_error", "md_step_baoab", "md_step_jump",
           "md_step_jump_respa", "md_step_baoab_respa", "md_step_jump_respa1", "md_step_baoab_respa1", "md_observables", "md_sync", "md_get_state",
           "md_set_state", "md_get_accel", "md_get_atom_stats", "md_get_events", "md_rdf", "md_rdf_noalloc",
           "md_get_cand_row", "md_get_row_counts", "md_run_phase", "md_profile", "md_profile_read",
           "md_counters", "md_theta_screen_error", "md_tune", "md_trace_velocities", "md_get_trace"]

_lib = None


class MDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libjumpmd error {code}: {msg}")
        self.code = code


def load():
    """Load libjumpmd.so (raises if it is missing: no fallback path exists).

    JUMPMD_LIBRARY may name another build of the same library."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("JUMPMD_LIBRARY", LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run paper_2412_15073_amd/build.py (hipcc, gfx950)")
    # PyTorch ships its own HIP runtime. Loading torch first makes the
    # library's libamdhip64.so.7 / libhsa-runtime64.so.1 dependencies resolve
    # (by SONAME) to the copies torch already mapped: one runtime per process,
    # and torch streams are valid handles for the library.
    import torch  # noqa: F401
    L = C.CDLL(path)
    L.md_create.argtypes = [C.POINTER(MDSystem), C.POINTER(MDSplit), C.POINTER(MDParams), C.c_void_p,
                            C.POINTER(MDAllocator), C.POINTER(C.c_void_p)]
    L.md_destroy.argtypes = [C.c_void_p]
    L.md_destroy.restype = None
    L.md_last_error.argtypes = [C.c_void_p]
    L.md_last_error.restype = C.c_char_p
    for fn in ("md_step_baoab", "md_step_jump", "md_step_jump_respa", "md_step_baoab_respa",
               "md_step_jump_respa1", "md_step_baoab_respa1"):
        getattr(L, fn).argtypes = [C.c_void_p, C.c_int64]
    L.md_observables.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(MDObs)]
    L.md_sync.argtypes = [C.c_void_p]
    L.md_get_state.argtypes = [C.c_void_p, _dp, _dp]
    L.md_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_int64]
    L.md_get_accel.argtypes = [C.c_void_p, C.c_int32, _dp]
    L.md_get_atom_stats.argtypes = [C.c_void_p, _lp, _lp, _lp, _up]
    L.md_get_events.argtypes = [C.c_void_p, C.POINTER(MDEvent), C.c_int64, _lp]
    L.md_tune.argtypes = [C.POINTER(MDSystem), C.POINTER(MDSplit), C.POINTER(MDParams), C.c_void_p,
                          C.POINTER(MDAllocator), C.c_int32, C.c_int32, C.POINTER(MDSplit), C.POINTER(MDParams),
                          C.POINTER(C.c_double), C.POINTER(MDTuneTrial), C.c_int32, C.POINTER(C.c_int32)]
    L.md_rdf.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_int32, _dp]
    L.md_rdf_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_int32, _dp]
    L.md_trace_velocities.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
    L.md_get_trace.argtypes = [C.c_void_p, _dp, C.c_int64, _lp, _lp]
    L.md_get_cand_row.argtypes = [C.c_void_p, C.c_int32, _ip, _ip, C.c_int32, _ip, _ip]
    L.md_get_row_counts.argtypes = [C.c_void_p, C.c_int32, _ip]
    L.md_run_phase.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double]
    L.md_profile.argtypes = [C.c_void_p, C.c_int32]
    L.md_profile_read.argtypes = [C.c_void_p, C.c_int32, _dp, _lp]
    L.md_counters.argtypes = [C.c_void_p, _lp, _lp]
    L.md_theta_screen_error.argtypes = [C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double)]
    for fn in EXPORTS:
        if fn not in ("md_destroy", "md_last_error"):
            getattr(L, fn).restype = C.c_int
    _lib = L
    return L


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def theta_screen_error(eta_lo, eta_hi, n):
    """Largest relative error of the device's float screen of Theta against
    FP64 Theta over n points of [eta_lo, eta_hi] (md_theta_screen_error)."""
    L = load()
    out = C.c_double(0.0)
    rc = L.md_theta_screen_error(float(eta_lo), float(eta_hi), int(n), C.byref(out))
    if rc != 0:
        raise MDError(rc, L.md_last_error(None).decode())
    return out.value


def _concat(systems):
    """Concatenate replicas into one global atom index space."""
    off = np.concatenate([[0], np.cumsum([s.n_atoms for s in systems])]).astype(np.int32)
    cat = lambda f, dt: np.ascontiguousarray(np.concatenate([np.asarray(getattr(s, f)) for s in systems]), dtype=dt)
    out = dict(pos=cat("pos", np.float64).reshape(-1), vel=cat("vel", np.float64).reshape(-1),
               mass=cat("mass", np.float64), charge=cat("charge", np.float64), type=cat("type", np.int32))
    out["bond_ij"] = np.ascontiguousarray(np.concatenate(
        [np.asarray(s.bond_ij, np.int64).reshape(-1, 2) + o for s, o in zip(systems, off)]), dtype=np.int32)
    out["angle_ijk"] = np.ascontiguousarray(np.concatenate(
        [np.asarray(s.angle_ijk, np.int64).reshape(-1, 3) + o for s, o in zip(systems, off)]), dtype=np.int32)
    out["bond_k"], out["bond_r0"] = cat("bond_k", np.float64), cat("bond_r0", np.float64)
    out["angle_k"], out["angle_t0"] = cat("angle_k", np.float64), cat("angle_t0", np.float64)
    if systems[0].excl_ptr is not None:
        ptrs, js, base = [np.zeros(1, np.int64)], [], 0
        for s, o in zip(systems, off):
            p = np.asarray(s.excl_ptr, np.int64)
            ptrs.append(p[1:] + base)
            js.append(np.asarray(s.excl_j, np.int64) + o)
            base += p[-1]
        out["excl_ptr"] = np.ascontiguousarray(np.concatenate(ptrs), dtype=np.int32)
        out["excl_j"] = np.ascontiguousarray(np.concatenate(js), dtype=np.int32)
    else:
        out["excl_ptr"] = out["excl_j"] = None
    out["box"] = np.ascontiguousarray(np.concatenate([np.asarray(s.box, np.float64) for s in systems]))
    out["offsets"] = off
    return out


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _marshal_system(system):
    """MDSystem of a systems.System or systems.Batch, with the arrays it points
    into (kept alive by the caller)."""
    systems = list(system.systems) if hasattr(system, "systems") else [system]
    s0 = systems[0]
    a = _concat(systems)
    a["eps"] = np.ascontiguousarray(s0.lj_eps, dtype=np.float64)
    a["sig"] = np.ascontiguousarray(s0.lj_sigma, dtype=np.float64)
    sy = MDSystem()
    sy.n_atoms, sy.n_types, sy.n_replicas = int(a["offsets"][-1]), s0.n_types, len(systems)
    sy.pos, sy.vel = _ptr(a["pos"], _dp), _ptr(a["vel"], _dp)
    sy.mass, sy.charge, sy.type = _ptr(a["mass"], _dp), _ptr(a["charge"], _dp), _ptr(a["type"], _ip)
    sy.lj_eps, sy.lj_sigma = _ptr(a["eps"], _dp), _ptr(a["sig"], _dp)
    sy.box, sy.replica_offset = _ptr(a["box"], _dp), _ptr(a["offsets"], _ip)
    sy.n_bonds, sy.bond_ij = len(a["bond_k"]), _ptr(a["bond_ij"], _ip)
    sy.bond_k, sy.bond_r0 = _ptr(a["bond_k"], _dp), _ptr(a["bond_r0"], _dp)
    sy.n_angles, sy.angle_ijk = len(a["angle_k"]), _ptr(a["angle_ijk"], _ip)
    sy.angle_k, sy.angle_t0 = _ptr(a["angle_k"], _dp), _ptr(a["angle_t0"], _dp)
    sy.excl_ptr, sy.excl_j = _ptr(a["excl_ptr"], _ip), _ptr(a["excl_j"], _ip)
    sy.coulomb_k, sy.accel_factor, sy.kB = s0.coulomb_k, s0.accel_factor, s0.kB
    return sy, a


def _marshal_split(split):
    return MDSplit(split.r_s, split.r_c, split.switch_width, split.skin, split.coulomb_alpha,
                   split.n_rings, split.ring_width, getattr(split, "coulomb_kind", 0),
                   getattr(split, "ewald_kmax", 0), (C.c_int32 * 3)(*getattr(split, "pme_grid", (0, 0, 0))),
                   getattr(split, "pme_order", 0))


def _marshal_params(params):
    return MDParams(params.dt, params.gamma, params.kT, params.seed, params.jump_lj, params.jump_coul,
                    params.eps, params.precision, params.rebuild_every, params.respa_inner,
                    params.log_events, params.strict_bounds, getattr(params, "chain_lanes", 0),
                    getattr(params, "graph_steps", 0), getattr(params, "bound_scale", 0.0),
                    getattr(params, "row_capacity", 0.0), getattr(params, "event_capacity", 0),
                    getattr(params, "chain_order", 0), getattr(params, "respa_outer", 1))


def _allocator(allocator):
    if allocator == "torch":
        return TorchAllocator() if _gpu_visible() else None
    return allocator


SCHEMES = {"baoab": 0, "jump": 1, "jump_respa": 2, "baoab_respa": 3}


def tune(system, split, params, scheme="jump", steps=50, stream=None, allocator="torch"):
    """md_tune: the fastest lanes / skin / rings / graph setting for this
    system and scheme. Returns (split, params, ms_per_step, trials): copies of
    the inputs with the chosen setting, and every setting timed."""
    import copy
    L = load()
    sy, keep = _marshal_system(system)
    sp, pa = _marshal_split(split), _marshal_params(params)
    alloc = _allocator(allocator)
    sp_o, pa_o, ms = MDSplit(), MDParams(), C.c_double(0.0)
    cap = 256
    tr = (MDTuneTrial * cap)()
    nt = C.c_int32(0)
    st = stream if stream is not None else _current_stream()
    rc = L.md_tune(C.byref(sy), C.byref(sp), C.byref(pa), st, C.byref(alloc.struct) if alloc is not None else None,
                   SCHEMES[scheme], steps, C.byref(sp_o), C.byref(pa_o), C.byref(ms), tr, cap, C.byref(nt))
    del keep
    if rc != MD_OK:
        raise MDError(rc, L.md_last_error(None).decode())
    split2, params2 = copy.copy(split), copy.copy(params)
    split2.skin, split2.n_rings, split2.ring_width = sp_o.skin, sp_o.n_rings, sp_o.ring_width
    params2.chain_lanes, params2.graph_steps = pa_o.chain_lanes, pa_o.graph_steps
    params2.chain_order = pa_o.chain_order
    trials = [{"chain_lanes": t.chain_lanes, "skin": t.skin, "n_rings": t.n_rings, "graph_steps": t.graph_steps,
               "chain_order": t.chain_order, "ms_per_step": t.ms_per_step} for t in tr[: min(cap, nt.value)]]
    return split2, params2, ms.value, trials


class Sim:
    """One libjumpmd context. `system` is a systems.System or systems.Batch."""

    def __init__(self, system, split, params, stream=None, allocator="torch"):
        """allocator: "torch" (PyTorch's caching allocator, when a GPU is
        visible), None (the library's own hipMalloc) or a TorchAllocator."""
        L = load()
        sy, a = _marshal_system(system)
        self._keep = a
        self.n = int(a["offsets"][-1])
        self.offsets = a["offsets"]
        sp, pa = _marshal_split(split), _marshal_params(params)
        self.stream = stream if stream is not None else _current_stream()
        allocator = _allocator(allocator)
        self.allocator = allocator
        h = C.c_void_p()
        rc = L.md_create(C.byref(sy), C.byref(sp), C.byref(pa), self.stream,
                         C.byref(allocator.struct) if allocator is not None else None, C.byref(h))
        if rc != MD_OK:
            raise MDError(rc, L.md_last_error(None).decode())
        self._h = h
        self._lib = L   # kept for close() during interpreter shutdown

    def close(self):
        if getattr(self, "_h", None):
            self._lib.md_destroy(self._h)
            self._h = None

    __del__ = close

    def _chk(self, rc):
        if rc != MD_OK:
            raise MDError(rc, load().md_last_error(self._h).decode())

    # stepping (asynchronous on the stream)
    def step_baoab(self, n):
        self._chk(load().md_step_baoab(self._h, n))

    def step_jump(self, n):
        self._chk(load().md_step_jump(self._h, n))

    def step_jump_respa(self, n):
        self._chk(load().md_step_jump_respa(self._h, n))

    def step_jump_respa1(self, n):
        self._chk(load().md_step_jump_respa1(self._h, n))

    def step_baoab_respa1(self, n):
        self._chk(load().md_step_baoab_respa1(self._h, n))

    def step_baoab_respa(self, n):
        self._chk(load().md_step_baoab_respa(self._h, n))

    def sync(self):
        self._chk(load().md_sync(self._h))

    def observables(self, pe=False):
        o = MDObs()
        self._chk(load().md_observables(self._h, MD_OBS_PE if pe else 0, C.byref(o)))
        return {f: getattr(o, f) for f, _ in MDObs._fields_}

    def state(self):
        x, v = np.zeros(3 * self.n), np.zeros(3 * self.n)
        self._chk(load().md_get_state(self._h, _ptr(x, _dp), _ptr(v, _dp)))
        return x.reshape(-1, 3), v.reshape(-1, 3)

    def set_state(self, pos=None, vel=None, step=-1):
        p = None if pos is None else np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
        v = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64).reshape(-1)
        self._chk(load().md_set_state(self._h, _ptr(p, _dp), _ptr(v, _dp), step))

    def accel(self, kind):
        a = np.zeros(3 * self.n)
        self._chk(load().md_get_accel(self._h, kind, _ptr(a, _dp)))
        return a.reshape(-1, 3)

    def atom_stats(self):
        a, b, c = (np.zeros(self.n, np.int64) for _ in range(3))
        h = np.zeros(self.n, np.uint64)
        self._chk(load().md_get_atom_stats(self._h, _ptr(a, _lp), _ptr(b, _lp), _ptr(c, _lp), _ptr(h, _up)))
        return {"n_prop": a, "n_acc": b, "n_viol": c, "hash": h}

    def events(self):
        n = C.c_int64(0)
        self._chk(load().md_get_events(self._h, None, 0, C.byref(n)))
        buf = (MDEvent * max(1, n.value))()
        self._chk(load().md_get_events(self._h, buf, n.value, C.byref(n)))
        return np.array([[e.step, e.phase, e.atom, e.partner, e.proposal] for e in buf[: n.value]],
                        dtype=np.int64).reshape(-1, 5)

    def rdf_counts(self, ta, tb, r_max, n_bins):
        h = np.zeros(n_bins)
        self._chk(load().md_rdf(self._h, ta, tb, r_max, n_bins, _ptr(h, _dp)))
        return h

    def trace_velocities(self, n_atoms, capacity):
        """Record the velocities of atoms [0, n_atoms) at every O update (once
        per smallest time step) into a device ring of `capacity` records;
        n_atoms = 0 stops."""
        self._chk(load().md_trace_velocities(self._h, n_atoms, capacity))
        self._trace = (n_atoms, capacity)

    def trace(self):
        """(velocities [records, n_atoms, 3] of the last min(recorded,
        capacity) records in time order, records taken so far)."""
        na, cap = self._trace
        out = np.zeros((cap, na, 3))
        k, tn = C.c_int64(0), C.c_int64(0)
        self._chk(load().md_get_trace(self._h, _ptr(out, _dp), cap, C.byref(k), C.byref(tn)))
        return out[:k.value], tn.value

    def cand_row(self, i, n_segments, images=False):
        n = C.c_int32(0)
        seg = np.zeros(n_segments + 1, np.int32)
        self._chk(load().md_get_cand_row(self._h, i, None, None, 0, C.byref(n), _ptr(seg, _ip)))
        j = np.zeros(max(1, n.value), np.int32)
        img = np.zeros(max(1, n.value), np.int32)
        self._chk(load().md_get_cand_row(self._h, i, _ptr(j, _ip), _ptr(img, _ip), n.value, C.byref(n),
                                         _ptr(seg, _ip)))
        if images:
            return j[: n.value], img[: n.value], seg
        return j[: n.value], seg

    def row_counts(self, which):
        c = np.zeros(self.n, np.int32)
        self._chk(load().md_get_row_counts(self._h, which, _ptr(c, _ip)))
        return c

    def run_phase(self, which, phase, h):
        self._chk(load().md_run_phase(self._h, ord(which), PHASE.get(phase, phase) if isinstance(phase, str) else phase, h))

    def profile(self, enable=True):
        self._chk(load().md_profile(self._h, 1 if enable else 0))

    def profile_read(self, kid):
        ms, n = C.c_double(0), C.c_int64(0)
        self._chk(load().md_profile_read(self._h, kid, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def proposals_total(self):
        p, q = C.c_int64(0), C.c_int64(0)
        self._chk(load().md_counters(self._h, C.byref(p), C.byref(q)))
        return q.value
