"""Seeded synthetic inputs: systems, cutoff splits and run parameters.

This module only builds input data (geometry, force-field parameters, initial
Maxwell-Boltzmann velocities, run settings). It holds none of the integrator's
arithmetic and imports neither the GPU binding nor the oracle, so both sides can
be fed the same inputs.

Workloads (the paper runs SPC/Fw water boxes in Tinker-HP, Sec. 4; none of its
input files are available, so these generated systems stand in for them):
  * LJ fluid: fcc lattice, reduced units;
  * flexible 3-site water: O on a cubic lattice (random vacancies when the
    molecule count is not a cube), random orientations, SPC-like charges,
    SPC/Fw force constants, LJ on O only, box edge from a number density.
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# jump kinds (same numbering on both sides of the boundary)
JUMP_NONE, JUMP_BPS, JUMP_MRZ_CONST, JUMP_MRZ_ADAPTIVE, JUMP_BOUNCE, JUMP_IN_C = 0, 1, 2, 3, 4, 5
COUL_DSF, COUL_EWALD, COUL_SPME = 0, 1, 2
FP64, FP32_MIXED = 0, 1

# water units: Angstrom, ps, amu, kJ/mol, e
COULOMB_K = 1389.35458        # kJ mol^-1 A e^-2
ACCEL_KJ = 100.0              # 1 kJ mol^-1 A^-1 amu^-1 = 100 A ps^-2
KB_KJ = 0.00831446261815324   # kJ mol^-1 K^-1
KCAL = 4.184                  # kJ per kcal


@dataclass
class System:
    n_atoms: int
    n_types: int
    pos: np.ndarray          # [N,3] float64, unwrapped
    vel: np.ndarray          # [N,3]
    mass: np.ndarray         # [N]
    charge: np.ndarray       # [N]
    type: np.ndarray         # [N] int32
    lj_eps: np.ndarray       # [T*T]
    lj_sigma: np.ndarray     # [T*T]
    box: np.ndarray          # [3]
    bond_ij: np.ndarray      # [B,2]
    bond_k: np.ndarray
    bond_r0: np.ndarray
    angle_ijk: np.ndarray    # [A,3] (vertex in the middle)
    angle_k: np.ndarray
    angle_t0: np.ndarray
    excl_ptr: Optional[np.ndarray]
    excl_j: Optional[np.ndarray]
    coulomb_k: float = 0.0
    accel_factor: float = 1.0
    kB: float = 1.0
    name: str = ""


@dataclass
class Split:
    r_s: float
    r_c: float
    switch_width: float
    skin: float
    coulomb_alpha: float = 0.0
    n_rings: int = 1
    ring_width: float = 0.0
    coulomb_kind: int = 0     # 0: damped shifted-force Coulomb; 1: the same plus the Ewald reciprocal sum;
                              # 2: the same with the reciprocal sum by smooth particle-mesh Ewald
    ewald_kmax: int = 0       # Ewald: lattice vectors n with 0 < |n|^2 <= kmax^2
    pme_grid: tuple = (0, 0, 0)   # SPME: grid points per box edge (powers of two on the GPU)
    pme_order: int = 0        # SPME: B-spline order (4, 6 or 8)


@dataclass
class Params:
    dt: float
    gamma: float
    kT: float
    seed: int = 1
    jump_lj: int = JUMP_NONE
    jump_coul: int = JUMP_NONE
    eps: float = 1.0
    respa_inner: int = 1
    respa_outer: int = 1      # middle steps per outer step of the three-level RESPA schemes
    rebuild_every: int = 0
    log_events: int = 0
    precision: int = FP64
    strict_bounds: int = 0
    chain_lanes: int = 0      # lanes per atom in the GPU jump chains (0 = automatic)
    graph_steps: int = 0      # steps per replayed HIP graph chunk (0 = no graphs)
    bound_scale: float = 0.0  # jump-rate bounds multiplied by this (0 = 1: as derived)
    row_capacity: float = 0.0 # initial row capacity / density estimate (0 = 1.5)
    event_capacity: int = 0   # accepted jumps the GPU event log holds (0 = 2^22)
    chain_order: int = 0      # wave order of the GPU jump chains (0 auto, 1 by type, 2 by replica)


@dataclass
class Batch:
    """Independent replicas advanced together (each keeps its own box)."""
    systems: List[System]
    offsets: np.ndarray = field(default=None)

    def __post_init__(self):
        if self.offsets is None:
            self.offsets = np.concatenate([[0], np.cumsum([s.n_atoms for s in self.systems])]).astype(np.int32)


def _mb_velocities(rng, mass, kT, accel):
    # Maxwell-Boltzmann at kT: each component normal with variance kT/m
    sd = np.sqrt(kT * accel / mass)
    return rng.standard_normal((len(mass), 3)) * sd[:, None]


# ----------------------------------------------------------------- LJ fluid
def lj_fcc(n_cells: int = 6, rho: float = 0.8442, kT: float = 0.722, seed: int = 1,
           jitter: float = 0.0) -> System:
    """fcc lattice of 4*n_cells^3 LJ atoms at reduced density rho (sigma = eps = m = 1);
    jitter > 0 displaces every atom by a seeded uniform offset in [-jitter, jitter]^3."""
    n = 4 * n_cells ** 3
    L = (n / rho) ** (1.0 / 3.0)
    a = L / n_cells
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(*[np.arange(n_cells)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = ((g[:, None, :] + basis[None, :, :]).reshape(-1, 3) + 0.25) * a
    rng = np.random.default_rng(seed)
    mass = np.ones(n)
    vel = _mb_velocities(rng, mass, kT, 1.0)
    if jitter > 0.0:
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    z2 = np.zeros((0, 2), np.int32)
    z3 = np.zeros((0, 3), np.int32)
    return System(n_atoms=n, n_types=1, pos=pos, vel=vel, mass=mass, charge=np.zeros(n),
                  type=np.zeros(n, np.int32), lj_eps=np.array([1.0]), lj_sigma=np.array([1.0]),
                  box=np.array([L, L, L]), bond_ij=z2, bond_k=np.zeros(0), bond_r0=np.zeros(0),
                  angle_ijk=z3, angle_k=np.zeros(0), angle_t0=np.zeros(0),
                  excl_ptr=None, excl_j=None, coulomb_k=0.0, accel_factor=1.0, kB=1.0,
                  name=f"lj_fcc_{n}")


# ------------------------------------------------------------------- water
WATER = dict(q_o=-0.82, q_h=0.41, sigma_o=3.166, eps_o=0.650, m_o=15.9994, m_h=1.008,
             b0=1.0, theta0_deg=109.47,
             k_b=1059.162 * KCAL,      # SPC/Fw, kJ mol^-1 A^-2, U = (k/2)(b-b0)^2
             k_theta=75.90 * KCAL)     # SPC/Fw, kJ mol^-1 rad^-2, U = (k/2)(th-th0)^2


def _random_rotations(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def water_box(n_mol: int, density: float = 0.0334, T: float = 300.0, seed: int = 1,
              jitter: float = 0.0) -> System:
    """n_mol flexible 3-site waters (O,H,H per molecule) in a cubic box of
    n_mol/density A^3; O on the sites of an n_side^3 cubic lattice (random
    vacancies if n_mol < n_side^3), random orientations. jitter > 0 displaces
    every atom by a seeded uniform offset in [-jitter, jitter]^3 A (bonds and
    angles off their minimum)."""
    p = WATER
    L = (n_mol / density) ** (1.0 / 3.0)
    n_side = int(np.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    a = L / n_side
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(n_side)] * 3, indexing="ij"), -1).reshape(-1, 3)
    if len(g) > n_mol:
        g = g[np.sort(rng.choice(len(g), n_mol, replace=False))]
    o = (g + 0.5) * a
    th = np.deg2rad(p["theta0_deg"])
    local = np.array([[0.0, 0.0, 0.0],
                      [p["b0"] * np.sin(th / 2), 0.0, p["b0"] * np.cos(th / 2)],
                      [-p["b0"] * np.sin(th / 2), 0.0, p["b0"] * np.cos(th / 2)]])
    R = _random_rotations(rng, n_mol)
    pos = (o[:, None, :] + np.einsum("mij,aj->mai", R, local)).reshape(-1, 3)
    n = 3 * n_mol
    typ = np.tile(np.array([0, 1, 1], np.int32), n_mol)
    mass = np.where(typ == 0, p["m_o"], p["m_h"]).astype(np.float64)
    charge = np.where(typ == 0, p["q_o"], p["q_h"]).astype(np.float64)
    base = 3 * np.arange(n_mol, dtype=np.int32)
    bond_ij = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1)])
    angle_ijk = np.stack([base + 1, base, base + 2], 1)
    excl_ptr = (2 * np.arange(n + 1)).astype(np.int32)
    ex = np.stack([np.stack([base + 1, base + 2], 1),
                   np.stack([base, base + 2], 1),
                   np.stack([base, base + 1], 1)], 1).reshape(-1).astype(np.int32)
    kT = KB_KJ * T
    vel = _mb_velocities(rng, mass, kT, ACCEL_KJ)
    if jitter > 0.0:
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    return System(n_atoms=n, n_types=2, pos=pos, vel=vel, mass=mass, charge=charge, type=typ,
                  lj_eps=np.array([p["eps_o"], 0.0, 0.0, 0.0]),
                  lj_sigma=np.array([p["sigma_o"], 1.0, 1.0, 1.0]),
                  box=np.array([L, L, L]), bond_ij=bond_ij,
                  bond_k=np.full(len(bond_ij), p["k_b"]), bond_r0=np.full(len(bond_ij), p["b0"]),
                  angle_ijk=angle_ijk, angle_k=np.full(n_mol, p["k_theta"]),
                  angle_t0=np.full(n_mol, th), excl_ptr=excl_ptr, excl_j=ex,
                  coulomb_k=COULOMB_K, accel_factor=ACCEL_KJ, kB=KB_KJ, name=f"water_{n_mol}")


def water_replica_recipe(n_rep: int = 256, n_min: int = 216, n_max: int = 2048, seed: int = 1):
    """(molecules, seed) of each replica of the ensemble: sizes uniform in
    [n_min, n_max] molecules."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_rep)
    return [(int(m), seed * 100003 + r) for r, m in enumerate(sizes)]


def water_replicas(n_rep: int = 256, n_min: int = 216, n_max: int = 2048, seed: int = 1,
                   density: float = 0.0334) -> Batch:
    """Replica sizes uniform in [n_min, n_max] molecules, each box at the density."""
    return Batch([water_box(m, density=density, seed=sr)
                  for m, sr in water_replica_recipe(n_rep, n_min, n_max, seed)])


# ------------------------------------------------------------------ configs
def lj_split(skin: float = 0.3, n_rings: int = 1, ring_width: float = 0.0) -> Split:
    """switch at r_s = 3.0 sigma (width 0.5), long part out to r_c = 5.0 sigma"""
    return Split(r_s=3.0, r_c=5.0, switch_width=0.5, skin=skin, n_rings=n_rings, ring_width=ring_width)


def lj_params(seed: int = 1, jumps: bool = True) -> Params:
    return Params(dt=0.005, gamma=1.0, kT=0.722, seed=seed,
                  jump_lj=JUMP_BPS if jumps else JUMP_NONE)


def water_split(r_s: float = 5.0, r_c: float = 10.0, w: float = 1.0, skin: float = 1.0,
                alpha: float = 0.2, n_rings: int = 4, ring_width: Optional[float] = None) -> Split:
    if ring_width is None:
        ring_width = ((r_c + skin) - (r_s - w - skin)) / n_rings
    return Split(r_s=r_s, r_c=r_c, switch_width=w, skin=skin, coulomb_alpha=alpha,
                 n_rings=n_rings, ring_width=ring_width)


def water_params(seed: int = 1, dt: float = 0.001, gamma: float = 1.0, T: float = 300.0,
                 eps0_per_kcal: float = 0.1, jumps: bool = True, precision: int = FP64) -> Params:
    """eps0 given in (kcal/mol/A)^-1 and converted to (kJ/mol/A)^-1"""
    return Params(dt=dt, gamma=gamma, kT=KB_KJ * T, seed=seed,
                  jump_lj=JUMP_BPS if jumps else JUMP_NONE,
                  jump_coul=JUMP_MRZ_ADAPTIVE if jumps else JUMP_NONE,
                  eps=eps0_per_kcal / KCAL, precision=precision)


def with_(obj, **kw):
    return replace(obj, **kw)


def two_charges(L: float = 10.0776, r0: float = 3.5, q: float = 1.0, coulomb_k: float = 13.0,
                lj_eps: float = 1.0, kT: float = 0.722, seed: int = 1) -> System:
    """Two like charges with LJ cores in a cubic box (reduced units), r0 apart
    along x; the smallest system on which both jump kinds act."""
    rng = np.random.default_rng(seed)
    pos = np.array([[0.25 * L, 0.5 * L, 0.5 * L], [0.25 * L + r0, 0.5 * L, 0.5 * L]])
    mass = np.ones(2)
    vel = _mb_velocities(rng, mass, kT, 1.0)
    z2 = np.zeros((0, 2), np.int32)
    z3 = np.zeros((0, 3), np.int32)
    return System(n_atoms=2, n_types=1, pos=pos, vel=vel, mass=mass, charge=np.array([q, q]),
                  type=np.zeros(2, np.int32), lj_eps=np.array([lj_eps]), lj_sigma=np.array([1.0]),
                  box=np.array([L, L, L]), bond_ij=z2, bond_k=np.zeros(0), bond_r0=np.zeros(0),
                  angle_ijk=z3, angle_k=np.zeros(0), angle_t0=np.zeros(0), excl_ptr=None, excl_j=None,
                  coulomb_k=coulomb_k, accel_factor=1.0, kB=1.0, name="two_charges")


def ion_lattice(n_side: int = 4, spacing: float = 3.3, q: float = 1.0, coulomb_k: float = 13.0,
                lj_eps: float = 0.0, lj_sigma: float = 1.0, jitter: float = 0.1, kT: float = 1.0,
                seed: int = 1, neutral_every: int = 0) -> System:
    """n_side^3 particles on a simple cubic lattice (reduced units) with
    alternating charges +q/-q (two types), optional LJ between all pairs and a
    seeded jitter; with spacing - 2*jitter above r_s no pair is inside the
    short range, so all forces come from the long part. neutral_every = m > 0
    makes every m-th site a neutral third type."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(n_side)] * 3, indexing="ij"), -1).reshape(-1, 3)
    n = len(g)
    pos = (g + 0.5) * spacing + rng.uniform(-jitter, jitter, size=(n, 3))
    typ = (g.sum(1) % 2).astype(np.int32)
    charge = np.where(typ == 0, q, -q).astype(np.float64)
    nt = 2
    if neutral_every > 0:
        typ[::neutral_every] = 2
        charge[::neutral_every] = 0.0
        nt = 3
    mass = np.ones(n)
    vel = _mb_velocities(rng, mass, kT, 1.0)
    L = n_side * spacing
    z2 = np.zeros((0, 2), np.int32)
    z3 = np.zeros((0, 3), np.int32)
    return System(n_atoms=n, n_types=nt, pos=pos, vel=vel, mass=mass, charge=charge, type=typ,
                  lj_eps=np.full(nt * nt, lj_eps), lj_sigma=np.full(nt * nt, lj_sigma), box=np.array([L, L, L]),
                  bond_ij=z2, bond_k=np.zeros(0), bond_r0=np.zeros(0), angle_ijk=z3, angle_k=np.zeros(0),
                  angle_t0=np.zeros(0), excl_ptr=None, excl_j=None, coulomb_k=coulomb_k, accel_factor=1.0,
                  kB=1.0, name=f"ion_lattice_{n}")
