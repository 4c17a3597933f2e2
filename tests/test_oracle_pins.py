"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test checks the oracle against what the paper or mathematics fixes:
library known answers, closed forms, quadrature, invariants, brute force and
statistical laws. A plausible slip anywhere in the oracle (dropped term,
wrong sign or index, transposed operand) should fail one of them.
"""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sps
import scipy.stats as st

from oracle import oracle as O
from paper_2412_15073_amd import systems as S
from tests.helpers import lj_small, water_small, fnv1a64, event_mix, rel_err


# ------------------------------------------------------------ random numbers
GOLDEN = __import__("pathlib").Path(__file__).parent / "golden"


def test_philox4x32_known_answers():
    """Philox4x32-10 against the published known-answer vectors (Random123)."""
    n = 0
    for line in (GOLDEN / "philox4x32_10_kat.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        np.testing.assert_array_equal(O.philox4x32(w[0:4], w[4:6]), np.array(w[6:10], np.uint32))
        n += 1
    assert n == 3


def test_philox4x32_is_a_bijection_of_the_counter():
    """Distinct counters give distinct blocks (no collisions over a sample),
    and words are uniform: mean and variance of u01 over 4 x 20000 draws."""
    key = [0x12345678, 0x9ABCDEF0]
    outs = np.array([O.philox4x32([c, 7, 3, 0], key) for c in range(20000)], dtype=np.uint64)
    packed = set(map(tuple, outs.tolist()))
    assert len(packed) == len(outs)
    u = (outs.astype(np.float64) + 0.5) / 2.0 ** 32
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / u.size)


def test_uniform_open_interval():
    assert O.u01(0) == 2.0 ** -33
    assert O.u01(2 ** 32 - 1) == 1.0 - 2.0 ** -33
    assert O.u01(1 << 31) == 0.5 + 2.0 ** -33


# ----------------------------------------------------------- pair potentials
RS, W, RC = 3.0, 0.5, 5.0


def _terms(r, eps=1.0, sig=1.0, qq=0.0, ke=1.0, alpha=0.2):
    return O.pair_terms(r, eps, sig, qq, ke, alpha, RS, W, RC)


def test_lj_closed_form_points():
    rmin = 2.0 ** (1.0 / 6.0)
    assert abs(_terms(rmin)[1]) < 1e-12                       # minimum of 4(r^-12 - r^-6)
    shift = 4.0 * (RC ** -12 - RC ** -6)
    assert abs(_terms(1.0)[0] + shift) < 1e-14                # U(sigma) = -shift
    assert abs(_terms(rmin)[0] - (-1.0 - shift)) < 1e-12      # depth -eps
    assert _terms(RC)[0] == 0.0 and _terms(RC + 1e-9)[1] == 0.0
    assert abs(_terms(RC - 1e-9)[0]) < 1e-9                   # continuous at r_c


@pytest.mark.parametrize("r", [0.95, 1.3, 2.2, 2.8, 3.4, 4.6])
def test_pair_derivatives_finite_difference(r):
    h = 1e-6
    for kw in (dict(eps=1.0), dict(eps=0.0, qq=-1.7, alpha=0.2), dict(eps=0.0, qq=2.0, alpha=0.0)):
        up, dn, mid = _terms(r + h, **kw), _terms(r - h, **kw), _terms(r, **kw)
        for iU, idU in ((0, 1), (2, 3)):
            fd = (up[iU] - dn[iU]) / (2 * h)
            assert abs(fd - mid[idU]) <= 1e-6 * max(1.0, abs(mid[idU])), (kw, r, fd, mid[idU])


def test_dsf_alpha_zero_is_shifted_force_coulomb():
    for r in (0.7, 1.9, 3.3, 4.99):
        U = _terms(r, eps=0.0, qq=1.0, alpha=0.0)[2]
        exact = 1.0 / r - 1.0 / RC + (r - RC) / RC ** 2
        assert abs(U - exact) < 1e-14


def test_dsf_energy_is_integral_of_shifted_force():
    """U(r) = int_r^rc F(s) ds with the damped force shifted to vanish at r_c
    (Fennell-Gezelter definition), evaluated by quadrature with scipy's erfc."""
    a = 0.35

    def force(s):
        f = lambda t: sps.erfc(a * t) / t ** 2 + 2 * a / np.sqrt(np.pi) * np.exp(-a * a * t * t) / t
        return f(s) - f(RC)

    for r in (0.8, 2.0, 3.7, 4.8):
        ref, _ = si.quad(force, r, RC, epsabs=1e-14, epsrel=1e-13)
        assert abs(_terms(r, eps=0.0, qq=1.0, alpha=a)[2] - ref) < 1e-11


def test_switch_shape():
    rlo = RS - W
    assert _terms(rlo)[4] == 1.0 and _terms(RS)[4] == 0.0
    assert abs(_terms(rlo + W / 2)[4] - 0.5) < 1e-15          # symmetric smoothstep
    assert abs(abs(_terms(rlo + W / 2)[5]) - 15.0 / (8.0 * W)) < 1e-12   # max |chi'|
    grid = np.linspace(rlo, RS, 2001)
    d = np.array([_terms(r)[5] for r in grid])
    assert np.abs(d).max() <= 15.0 / (8.0 * W) + 1e-12
    h = 1e-5
    for r in (rlo + 0.1, rlo + 0.3):
        fd = (_terms(r + h)[4] - _terms(r - h)[4]) / (2 * h)
        assert abs(fd - _terms(r)[5]) < 1e-7
    # C2 at both ends: chi'' -> 0 linearly in the distance to the end
    for delta in (1e-3, 1e-4, 1e-5):
        for r in (rlo + delta, RS - delta):
            hh = delta / 10
            dd = (_terms(r + hh)[5] - _terms(r - hh)[5]) / (2 * hh)
            assert abs(dd) < 600 * delta


# -------------------------------------------------------------- MRZ pieces
@pytest.mark.parametrize("eta", [-6.0, -2.5, -1.0, -0.2, 0.0, 0.7, 3.0, 8.0])
def test_theta_is_expected_positive_part(eta):
    ref, _ = si.quad(lambda g: (eta + g) * np.exp(-g * g / 2) / np.sqrt(2 * np.pi), -eta, np.inf,
                     epsabs=1e-15, epsrel=1e-12)
    assert abs(O.theta(eta) - ref) <= 1e-12 * max(ref, 1e-300) + 1e-300
    h = 1e-6
    assert abs((O.theta(eta + h) - O.theta(eta - h)) / (2 * h) - st.norm.cdf(eta)) < 1e-7


def test_theta_at_zero():
    assert abs(O.theta(0.0) - 1.0 / np.sqrt(2 * np.pi)) < 1e-16


def _z_cdf(eta):
    z = np.linspace(0, eta + 12 if eta > 0 else 14.0 / max(1.0, abs(eta)) + 6, 20001)
    dens = z * np.exp(-0.5 * (z - eta) ** 2)
    cdf = np.concatenate([[0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(z))])
    cdf /= cdf[-1]
    return lambda x: np.interp(x, z, cdf)


@pytest.mark.parametrize("eta", [-5.0, -2.0, -1.0, -0.4, 0.0, 0.5, 3.0])
def test_zsampler_law(eta):
    """Z = eta + G~ has density z exp(-(z-eta)^2/2) on z > 0: closed-form
    mean and a KS test against the numerically integrated CDF."""
    n = 20000
    z = np.array([O.zsample(eta, seed=7, step=3, atom=11, k=k)[0] for k in range(n)])
    Phi, phi = st.norm.cdf(eta), st.norm.pdf(eta)
    mean = ((eta * eta + 1) * Phi + eta * phi) / (eta * Phi + phi)
    assert abs(z.mean() - mean) < 5 * z.std() / np.sqrt(n)
    assert st.kstest(z, _z_cdf(eta)).pvalue > 1e-3
    assert (z > 0).all()


@pytest.mark.parametrize("e", [0.3, 1.0, 3.0])
def test_mrz_kernel_reproduces_force_in_generator(e):
    """The MRZ rate/kernel pair (Sec. 2.2) stands in for the drift -F/m: for
    every f, E_mu[lambda (Qf - f)] = -beta E_mu[(F.v) f], i.e. the kernel maps
    lambda*mu onto (lambda - beta F.v)*mu. In s = sqrt(beta m) v.F/|F| (standard
    normal under mu, lambda ~ Theta(e s), Theta(x) - x = Theta(-x)) this reads:
    s ~ Theta(e s) phi(s)  =>  s' = s - 2e/(1+e^2) (e s + G~) ~ Theta(-e s) phi(s).
    A wrong sign, factor or sampler regime breaks the mirror image."""
    lim = 10 + 10 * e
    grid = np.linspace(-lim, lim, 40001)
    dens = np.array([O.theta(e * s) for s in grid]) * st.norm.pdf(grid)
    cdf = np.concatenate([[0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    rng = np.random.default_rng(5)
    s = np.interp(rng.random(15000), cdf, grid)
    z = np.array([O.zsample(e * si_, seed=9, k=k)[0] for k, si_ in enumerate(s)])
    s2 = s - 2 * e / (1 + e * e) * z
    # the mirrored variable -s' must follow the original law
    assert st.kstest(-s2, lambda x: np.interp(x, grid, cdf)).pvalue > 1e-3
    # and s' itself must not (the jump does change the law)
    assert st.kstest(s2, lambda x: np.interp(x, grid, cdf)).pvalue < 1e-6


# ------------------------------------------------------------------ forces
def _oracle(system, split, params):
    return O.OracleSim(system, split, params)


def test_jump_results_do_not_depend_on_call_grouping():
    """The opening C' of a step continues the closing C' stream of the step
    before from an index kept per atom, so splitting a run into calls changes
    nothing: positions, velocities and accepted events are identical."""
    sy, sp = water_small()
    pa = S.water_params()
    pa.log_events = 1
    a, b = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    a.step_jump(6)
    for n in (1, 2, 3):
        b.step_jump(n)
    xa, va = a.state()
    xb, vb = b.state()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(a.events(), b.events())
    assert len(a.events()) > 0
    pa.respa_inner = 3
    a, b = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    a.step_jump_respa(4)
    for n in (1, 3):
        b.step_jump_respa(n)
    np.testing.assert_array_equal(a.state()[1], b.state()[1])
    np.testing.assert_array_equal(a.events(), b.events())


def test_newton_third_law():
    sy, sp = water_small()
    o = _oracle(sy, sp, S.water_params())
    me = (sy.mass / sy.accel_factor)[:, None]
    for kind in (O.F_SHORT, O.F_FULL, O.F_BONDED):
        f = o.accel(kind) * me
        assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).sum()


def test_forces_are_minus_energy_gradient():
    sy, sp = water_small()
    o = _oracle(sy, sp, S.water_params())
    me = (sy.mass / sy.accel_factor)
    af, ab, ash = o.accel(O.F_FULL), o.accel(O.F_BONDED), o.accel(O.F_SHORT)
    x0, v0 = o.state()
    h = 1e-6
    for i, c in [(0, 0), (1, 2), (5, 1), (200, 0), (374, 2)]:
        e = []
        for sgn in (1, -1):
            x = x0.copy()
            x[i, c] += sgn * h
            o.set_state(pos=x)
            e.append(o.energies())
        o.set_state(pos=x0)
        full = lambda d: d["pe_short"] + d["pe_long"]
        fd_full = -(full(e[0]) - full(e[1])) / (2 * h)
        fd_b = -(e[0]["pe_bonded"] - e[1]["pe_bonded"]) / (2 * h)
        fd_s = -(e[0]["pe_short"] - e[1]["pe_short"]) / (2 * h)
        assert abs(fd_full - af[i, c] * me[i]) < 1e-5 * max(1.0, abs(fd_full))
        assert abs(fd_b - ab[i, c] * me[i]) < 1e-5 * max(1.0, abs(fd_b))
        assert abs(fd_s - ash[i, c] * me[i]) < 1e-5 * max(1.0, abs(fd_s))


def test_energy_split_sums_to_full_potential():
    """U_short + U_long = U pair by pair: total from the oracle against a plain
    numpy sum over all pairs of the full potential."""
    sy, sp = water_small()
    o = _oracle(sy, sp, S.water_params())
    e = o.energies()
    x = sy.pos
    L = sy.box
    tot = 0.0
    excl = set()
    for i in range(sy.n_atoms):
        for j in sy.excl_j[sy.excl_ptr[i]:sy.excl_ptr[i + 1]]:
            excl.add((i, int(j)))
    for i in range(sy.n_atoms):
        d = x[i + 1:] - x[i]
        d -= L * np.rint(d / L)
        r = np.sqrt((d * d).sum(1))
        for k, rr in enumerate(r):
            j = i + 1 + k
            if rr >= sp.r_c or (i, j) in excl:
                continue
            ti, tj = sy.type[i], sy.type[j]
            t = O.pair_terms(rr, sy.lj_eps[ti * 2 + tj], sy.lj_sigma[ti * 2 + tj], sy.charge[i] * sy.charge[j],
                             sy.coulomb_k, sp.coulomb_alpha, sp.r_s, sp.switch_width, sp.r_c)
            tot += t[0] + t[2]
    assert abs(e["pe_short"] + e["pe_long"] - tot) < 1e-9 * max(1.0, abs(tot))


# ------------------------------------------------------------------- lists
@pytest.mark.parametrize("case", ["lj", "water"])
def test_candidate_rows_brute_force(case):
    sy, sp = lj_small() if case == "lj" else water_small(n_rings=4)
    pa = S.lj_params() if case == "lj" else S.water_params()
    o = _oracle(sy, sp, pa)
    o.build_lists()
    rlo = sp.r_s - sp.switch_width
    rin, rout = rlo - sp.skin, sp.r_c + sp.skin
    nr = sp.n_rings
    rw = sp.ring_width if nr > 1 else rout - rin
    excl = {}
    if sy.excl_ptr is not None:
        for i in range(sy.n_atoms):
            excl[i] = set(sy.excl_j[sy.excl_ptr[i]:sy.excl_ptr[i + 1]].tolist())
    for i in range(0, sy.n_atoms, 7):
        d = sy.pos - sy.pos[i]
        d -= sy.box * np.rint(d / sy.box)
        r = np.sqrt((d * d).sum(1))
        keep = [j for j in range(sy.n_atoms) if j != i and j not in excl.get(i, ()) and rin <= r[j] < rout]
        ring = [min(nr - 1, max(0, int(np.floor((r[j] - rin) / rw)))) for j in keep]
        seg = [int(sy.type[j]) * nr + k for j, k in zip(keep, ring)]
        order = sorted(zip(seg, keep))
        np.testing.assert_array_equal(o.cand_row(i), [j for _, j in order])
        starts = [sum(1 for s_, _ in order if s_ < q) for q in range(o.n_segments + 1)]
        np.testing.assert_array_equal(o.seg_start(i), starts)


def _small_water(n_mol=216, seed=7, r_c=10.0, skin=0.5, n_rings=4):
    """216 waters in an 18.6 A box with r_c = 10 A: edges below 2 (r_c + skin),
    so partners can lie within the cutoff in two periodic images."""
    sy = S.water_box(n_mol, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=r_c, w=1.0, skin=skin, n_rings=n_rings)
    assert sy.box[0] < 2 * (r_c + skin)
    return sy, sp


def _image_pairs(sy, i, cut, lo=0.0):
    """Brute force over every lattice vector n in {-2..2}^3 (a superset of
    the images any cutoff below the edge can reach): (j, n, r) of the images
    x_j + n L with lo <= |x_i - x_j - n L| < cut, j != i."""
    L = sy.box
    out = []
    ns = np.array([(a, b, c) for c in range(-2, 3) for b in range(-2, 3) for a in range(-2, 3)])
    for j in range(sy.n_atoms):
        if j == i:
            continue
        d = (sy.pos[i] - sy.pos[j])[None, :] - ns * L
        r = np.sqrt((d * d).sum(1))
        for n, rr in zip(ns, r):
            if lo <= rr < cut:
                out.append((j, tuple(int(x) for x in n), rr))
    return out


def test_candidate_rows_with_periodic_images_brute_force():
    """In a box below 2 (r_c + skin) a candidate is one periodic image of j:
    the rows hold every image x_j + n L with r_s - w - skin <= r < r_c + skin
    (brute force over n in {-2..2}^3), sorted by (segment, j, image offset
    from the nearest image), with the image's lattice vector n."""
    sy, sp = _small_water()
    o = _oracle(sy, sp, S.water_params())
    o.build_lists()
    rlo = sp.r_s - sp.switch_width
    rin, rout = rlo - sp.skin, sp.r_c + sp.skin
    nr = sp.n_rings
    excl = {i: set(sy.excl_j[sy.excl_ptr[i]:sy.excl_ptr[i + 1]].tolist()) for i in range(sy.n_atoms)}
    n_multi = 0
    for i in range(0, sy.n_atoms, 37):
        cands = [(j, n, r) for j, n, r in _image_pairs(sy, i, rout, rin) if j not in excl[i]]
        keys = []
        for j, n, r in cands:
            ring = min(nr - 1, max(0, int(np.floor((r - rin) / sp.ring_width))))
            m = np.rint((sy.pos[i] - sy.pos[j]) / sy.box).astype(int)
            s = np.array(n) - m
            keys.append((int(sy.type[j]) * nr + ring, j, int((s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1)), n))
        keys.sort()
        jo, no = o.cand_row_images(i)
        np.testing.assert_array_equal(jo, [k[1] for k in keys])
        np.testing.assert_array_equal(no, np.array([k[3] for k in keys]).reshape(-1, 3))
        starts = [sum(1 for k in keys if k[0] < q) for q in range(o.n_segments + 1)]
        np.testing.assert_array_equal(o.seg_start(i), starts)
        js = [k[1] for k in keys]
        n_multi += len(js) - len(set(js))
    assert n_multi > 0   # some partners do appear in two images


def test_energy_and_forces_with_periodic_images():
    """Small box: the non-bonded energy is the sum over every pair and every
    periodic image within r_c (brute force over n in {-2..2}^3 with the pinned
    pair terms), forces are minus its gradient (central differences), and
    they sum to zero."""
    sy, sp = _small_water(n_mol=216, seed=8)
    o = _oracle(sy, sp, S.water_params())
    excl = {i: set(sy.excl_j[sy.excl_ptr[i]:sy.excl_ptr[i + 1]].tolist()) for i in range(sy.n_atoms)}

    def brute(pos):
        tot = 0.0
        s2 = S.System(**{**sy.__dict__, "pos": pos})
        for i in range(sy.n_atoms):
            for j, n, r in _image_pairs(s2, i, sp.r_c):
                if j <= i or j in excl[i]:
                    continue
                ti, tj = sy.type[i], sy.type[j]
                t = O.pair_terms(r, sy.lj_eps[ti * 2 + tj], sy.lj_sigma[ti * 2 + tj], sy.charge[i] * sy.charge[j],
                                 sy.coulomb_k, sp.coulomb_alpha, sp.r_s, sp.switch_width, sp.r_c)
                tot += t[0] + t[2]
        return tot

    e = o.energies()
    ref = brute(sy.pos)
    assert abs(e["pe_short"] + e["pe_long"] - ref) < 1e-9 * abs(ref)
    acc = o.accel(O.F_FULL)
    me = sy.mass / sy.accel_factor
    f = acc * me[:, None]
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).sum()
    h = 1e-5
    for i in (0, 100, 401):
        for c in range(3):
            xp, xm = sy.pos.copy(), sy.pos.copy()
            xp[i, c] += h
            xm[i, c] -= h
            o.set_state(pos=xp)
            ep = o.energies()
            o.set_state(pos=xm)
            em = o.energies()
            fd = -((ep["pe_short"] + ep["pe_long"]) - (em["pe_short"] + em["pe_long"])) / (2 * h)
            assert abs(f[i, c] - fd) < 1e-5 * max(1.0, abs(fd)), (i, c, f[i, c], fd)
    o.set_state(pos=sy.pos)


def test_bounds_dominate_long_gradient():
    """Each ring bound is >= |grad (1-chi) U| on a dense grid of distances the
    ring can reach (sup over [e_k - skin, r_c))."""
    sy, sp = water_small(n_rings=4)
    o = _oracle(sy, sp, S.water_params())
    ljb, cub, qmax = o.bounds(2, 4)
    rlo = sp.r_s - sp.switch_width
    for k in range(4):
        ek = rlo - sp.skin + k * sp.ring_width
        grid = np.linspace(max(ek - sp.skin, 1.0), sp.r_c, 3000)
        for a, b in ((0, 0), (0, 1), (1, 1)):
            g_lj, g_c = [], []
            for r in grid:
                t = O.pair_terms(r, sy.lj_eps[a * 2 + b], sy.lj_sigma[a * 2 + b], 1.0, sy.coulomb_k,
                                 sp.coulomb_alpha, sp.r_s, sp.switch_width, sp.r_c)
                g_lj.append(abs((1 - t[4]) * t[1] - t[5] * t[0]))
                g_c.append(abs((1 - t[4]) * t[3] - t[5] * t[2]))
            assert max(g_lj) <= ljb[a, b, k] * (1 + 1e-12)
            assert max(g_c) <= cub[a, b, k] * (1 + 1e-12)


# ----------------------------------------------------------------- phases
def test_bps_reflection_preserves_speed():
    sy, sp = lj_small()
    o = _oracle(sy, sp, S.lj_params())
    _, v0 = o.state()
    o.phase_j(O.PH_J1, 0.5)
    _, v1 = o.state()
    assert o.atom_stats()["n_acc"].sum() > 20
    np.testing.assert_allclose(np.linalg.norm(v1, axis=1), np.linalg.norm(v0, axis=1), rtol=1e-12)


def test_o_step_gaussian_law():
    sy, sp = lj_small()
    pa = S.lj_params()
    pa.gamma = 50.0
    o = _oracle(sy, sp, pa)
    x0, _ = o.state()
    vals = []
    for k in range(20):
        o.set_state(pos=x0, vel=np.zeros_like(x0), step=k)
        o.phase_o(1.0)
        vals.append(o.state()[1].ravel())
    v = np.concatenate(vals) / np.sqrt(pa.kT * (1 - np.exp(-2 * 50.0)))
    assert abs(v.mean()) < 5 / np.sqrt(len(v))
    assert abs(v.var() - 1) < 5 * np.sqrt(2 / len(v))
    assert st.kstest(v, "norm").pvalue > 1e-3


def test_event_log_and_hash_agree():
    sy, sp = lj_small()
    pa = S.lj_params()
    pa.log_events = 1
    o = _oracle(sy, sp, pa)
    o.step_jump(20)
    ev = o.events()
    stt = o.atom_stats()
    assert len(ev) == stt["n_acc"].sum() > 0
    h = np.full(sy.n_atoms, 0xCBF29CE484222325, dtype=object)
    for step, phase, i, j, k in ev:
        h[i] = event_mix(int(h[i]), int(step), int(phase), int(j))
    np.testing.assert_array_equal(np.array(h, dtype=np.uint64), stt["hash"])
    run = 0xCBF29CE484222325
    for x in stt["hash"]:
        run = fnv1a64(run, int(x).to_bytes(8, "little"))
    assert run == o.event_hash()


# --------------------------------------------------------------- schemes
def test_velocity_verlet_energy_error_scales_as_dt_squared():
    """With gamma = 0 and no jumps, the JUMP scheme is velocity Verlet on the
    smooth (C2-switched) short potential: the energy fluctuation falls 4x
    when dt halves."""
    sy, sp = water_small(n_mol=125)
    flucts = []
    for dt in (0.0004, 0.0002):
        pa = S.water_params(dt=dt, gamma=0.0, jumps=False)
        o = _oracle(sy, sp, pa)
        es = []
        for _ in range(10):
            o.step_jump(int(round(0.002 / dt)))
            e = o.energies()
            es.append(e["ke"] + e["pe_short"] + e["pe_bonded"])
        flucts.append(np.std(es))
    ratio = flucts[0] / flucts[1]
    assert 3.0 < ratio < 5.3, ratio


def test_jump_respa_with_one_inner_step_is_jump():
    """Special case of the JUMP-RESPA composition (Sec. 3.3): with one inner
    step and no bonded terms, the inner bonded kicks vanish and the scheme is
    C' J' A O A J' C' at the same step, so it must reproduce JUMP bit for bit
    (same random streams, same events)."""
    sy, sp = lj_small()
    pa = S.lj_params()
    pa.log_events = 1
    pa.respa_inner = 1
    a, b = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    a.step_jump(30)
    b.step_jump_respa(30)
    (xa, va), (xb, vb) = a.state(), b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert len(a.events()) > 50 and np.array_equal(a.events(), b.events())


def test_baoab_respa_with_one_inner_step_is_baoab():
    """Same reduction for the comparator: one inner step, no bonded terms."""
    sy, sp = lj_small()
    pa = S.lj_params(jumps=False)
    pa.respa_inner = 1
    a, b = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    a.step_baoab(30)
    b.step_baoab_respa(30)
    (xa, va), (xb, vb) = a.state(), b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def _bonds_only(sy):
    """The same molecules with no charges and no LJ: only bonds and angles act."""
    return S.with_(sy, charge=np.zeros(sy.n_atoms), lj_eps=np.zeros_like(sy.lj_eps))


@pytest.mark.parametrize("scheme", ["baoab_respa", "jump_respa"])
def test_respa_inner_loop_is_baoab_on_bonded_water(scheme):
    """Special case of the RESPA compositions (Sec. 2.3.2, Sec. 3.3) on
    molecules with bonds and angles but no non-bonded terms, at gamma = 0:
    the outer non-bonded kicks (or C' with no candidates) add exactly zero
    and O is the identity, so n outer steps of 3 inner steps B_b A O A B_b
    must reproduce 3n BAOAB steps at the inner step bit for bit. A dropped,
    doubled, mistimed or stale inner bonded kick breaks this (BAOAB itself is
    pinned by the dt^2 energy law on bonded water)."""
    sy, sp = water_small()
    sy = _bonds_only(sy)
    pa = S.water_params(gamma=0.0, jumps=(scheme == "jump_respa"))
    pa.respa_inner = 3
    a, b = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    a.step_baoab(60)
    (b.step_jump_respa if scheme == "jump_respa" else b.step_baoab_respa)(20)
    (xa, va), (xb, vb) = a.state(), b.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert rel_err(vb, sy.vel) > 1e-2   # the bonded forces did act


def test_baoab_respa_energy_error_scales_as_step_squared():
    """BAOAB-RESPA at gamma = 0 with all forces on (bonded at the inner step,
    full-range non-bonded at the outer step, Sec. 2.3.2) is a symplectic
    second-order integrator: with the inner count fixed, halving the inner
    (and so the outer) step cuts the total-energy fluctuation about 4x."""
    sy, sp = water_small(n_mol=125)
    flucts = []
    for dt in (0.0002, 0.0001):
        pa = S.water_params(dt=dt, gamma=0.0, jumps=False)
        pa.respa_inner = 3
        o = _oracle(sy, sp, pa)
        es = []
        for _ in range(10):
            o.step_baoab_respa(int(round(0.0024 / (3 * dt))))
            e = o.energies()
            es.append(e["ke"] + e["pe_full"])
        flucts.append(np.std(es))
    ratio = flucts[0] / flucts[1]
    assert 3.0 < ratio < 5.3, ratio


def test_jump_respa_samples_the_bond_length_law():
    """One flexible water molecule under JUMP-RESPA (3 inner steps of
    0.5 fs, gamma 50/ps): the O-H bond length b has the marginal
    b^2 exp(-beta k_b (b - b0)^2 / 2) of the Gibbs measure (the bonded energy
    separates in (b1, b2, theta) with Jacobian b1^2 b2^2 sin(theta)); the
    histogram matches it by quadrature, and <v^2> = kT/m per component."""
    sy = S.water_box(1, density=1.0 / 27000.0, seed=2, jitter=0.02)   # box 30 A
    sp = S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=1)
    pa = S.water_params(dt=0.0005, gamma=50.0)
    pa.respa_inner = 3
    o = _oracle(sy, sp, pa)
    kT, kb, b0 = pa.kT, sy.bond_k[0], sy.bond_r0[0]
    bs, ke = [], []
    for _ in range(12000):
        o.step_jump_respa(40)   # 60 fs
        x, v = o.state()
        bs += [np.linalg.norm(x[1] - x[0]), np.linalg.norm(x[2] - x[0])]
        ke.append((0.5 * sy.mass[:, None] * v * v).sum() / S.ACCEL_KJ)
    bs = np.array(bs)
    sd = np.sqrt(kT / kb)
    edges = b0 + sd * np.array([-3.5, -2.0, -1.2, -0.6, -0.2, 0.2, 0.6, 1.2, 2.0, 3.5])
    dens = lambda b: b * b * np.exp(-0.5 * kb * (b - b0) ** 2 / kT)
    p = np.array([si.quad(dens, lo, hi, epsabs=0)[0] for lo, hi in zip(edges[:-1], edges[1:])])
    sel = bs[(bs >= edges[0]) & (bs < edges[-1])]
    cnt, _ = np.histogram(sel, edges)
    exp = p / p.sum() * len(sel)
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert st.chi2.sf(chi2, len(cnt) - 1) > 1e-3, (cnt, exp.round(1))
    # 9 degrees of freedom: <KE> = 9 kT / 2 within 3 %
    assert abs(np.mean(ke) / (4.5 * kT) - 1.0) < 0.03, np.mean(ke) / (4.5 * kT)


def test_rdf_counts_on_rock_salt_lattice():
    """Pair-count histogram against the coordination shells of a rock-salt
    lattice (6 x 6 x 6 sites, spacing a, alternating types): unlike pairs at
    a, sqrt(3) a, sqrt(5) a (6, 8, 24 per site), like pairs at sqrt(2) a, 2a,
    sqrt(6) a, sqrt(8) a (12, 6, 24, 12 per site), every shell below L/2."""
    a = 1.53
    sy = S.ion_lattice(6, a, jitter=0.0)
    sp = S.Split(r_s=2.0, r_c=3.0, switch_width=0.5, skin=0.3)
    o = _oracle(sy, sp, S.Params(dt=0.001, gamma=1.0, kT=1.0))
    n_half = sy.n_atoms // 2
    r_max, nb = 4.5, 45
    dr = r_max / nb
    for (ta, tb), shells in (((0, 1), {1: 6, 3: 8, 5: 24}), ((0, 0), {2: 12 // 2, 4: 6 // 2, 6: 24 // 2, 8: 12 // 2}),
                             ((1, 1), {2: 12 // 2, 4: 6 // 2, 6: 24 // 2, 8: 12 // 2})):
        want = np.zeros(nb)
        for sq, z in shells.items():
            r = a * np.sqrt(sq)
            assert abs(r / dr - round(r / dr)) > 0.05   # no shell on a bin edge
            want[int(r / dr)] += n_half * z
        np.testing.assert_array_equal(o.rdf_counts(ta, tb, r_max, nb), want)


@pytest.mark.parametrize("coul", [O.JUMP_MRZ_ADAPTIVE, O.JUMP_BPS])
def test_thinning_exact_under_bound_inflation(coul):
    """Poisson thinning does not depend on the bound (Sec. 2.4): inflating all
    bounds x3 leaves the law of the C and J updates unchanged (per-atom means
    of dv over independent streams, chi-square over all atoms and components)."""
    sy, sp = S.water_box(125, seed=4), S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    pa = S.water_params(eps0_per_kcal=0.5)
    pa.jump_coul = coul
    res = []
    K = 150
    for scale in (1.0, 3.0):
        o = _oracle(sy, sp, pa)
        o.set_bound_scale(scale)
        x0, v0 = o.state()
        dv = []
        for k in range(K):
            o.set_state(vel=v0, step=1000 + k)
            o.phase_c(O.PH_C1, 0.002)
            o.phase_j(O.PH_J1, 0.002)
            dv.append((o.state()[1] - v0).ravel())
        dv = np.array(dv)
        res.append((dv.mean(0), dv.var(0, ddof=1), o.atom_stats()["n_prop"].sum()))
    (m1, v1, p1), (m2, v2, p2) = res
    z2 = (m1 - m2) ** 2 / ((v1 + v2) / K + 1e-300)
    dof = z2.size
    assert st.chi2.sf(z2.sum(), dof) > 1e-3
    assert p2 > 2.5 * p1          # inflated bounds propose ~3x more often


@pytest.mark.parametrize("kind", [O.JUMP_MRZ_ADAPTIVE, O.JUMP_MRZ_CONST])
def test_small_eps_limit_is_hamiltonian_drift(kind):
    """eps -> 0: the jump process converges to dv/dt = -F_long/m (Sec. 2.2).
    Two charges in the pure long-range region (chi = 0, no short force)."""
    sy = S.two_charges(L=12.0, r0=4.0, lj_eps=0.0)
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.2, coulomb_alpha=0.2)
    eps = 2e-3 if kind == O.JUMP_MRZ_ADAPTIVE else 1e-3
    pa = S.Params(dt=0.02, gamma=0.0, kT=0.722, jump_coul=kind, eps=eps)
    o = _oracle(sy, sp, pa)
    x0, v0 = o.state()
    t = O.pair_terms(4.0, 0.0, 1.0, 1.0, sy.coulomb_k, 0.2, 3.0, 1.0, 5.0)
    g = (1 - t[4]) * t[3] - t[5] * t[2]           # d/dr of the long part
    h = 0.01
    dv = []
    for k in range(2000):
        o.set_state(vel=v0, step=k)
        o.phase_c(O.PH_C1, h)
        dv.append(o.state()[1][0] - v0[0])
    dv = np.array(dv)
    mean, se = dv.mean(0), dv.std(0, ddof=1) / np.sqrt(len(dv))
    expected = -h * g * np.array([-1.0, 0.0, 0.0])  # atom 0 sits at -x of atom 1
    assert np.all(np.abs(mean - expected) < 4.5 * se + 0.01 * abs(expected[0])), (mean, se, expected)
    assert se[0] < 0.05 * abs(expected[0])          # the test has the power to see a wrong drift


def test_c_step_small_eps_is_kick_with_full_force():
    """In the switch region both parts act: the C step integrates the short
    force as a constant acceleration between proposals and the jumps supply the
    long part, so as eps0 -> 0 the mean velocity change over h is the plain
    kick -h grad U_full / m (Sec. 2.3 step (C) with Sec. 2.2's eps -> 0 limit)."""
    r0 = 2.4
    sy = S.two_charges(L=12.0, r0=r0, lj_eps=0.0)
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.2, coulomb_alpha=0.2)
    pa = S.Params(dt=0.02, gamma=0.0, kT=0.722, jump_coul=O.JUMP_MRZ_ADAPTIVE, eps=2e-3)
    o = _oracle(sy, sp, pa)
    x0, v0 = o.state()
    t = O.pair_terms(r0, 0.0, 1.0, 1.0, sy.coulomb_k, 0.2, 3.0, 1.0, 5.0)
    assert 0.1 < t[4] < 0.9                     # really inside the switch
    h = 0.01
    dv = []
    for k in range(2000):
        o.set_state(vel=v0, step=k)
        o.phase_c(O.PH_C1, h)
        dv.append(o.state()[1][0] - v0[0])
    dv = np.array(dv)
    mean, se = dv.mean(0), dv.std(0, ddof=1) / np.sqrt(len(dv))
    expected = -h * t[3] * np.array([-1.0, 0.0, 0.0])
    assert np.all(np.abs(mean - expected) < 4.5 * se + 0.01 * abs(expected[0])), (mean, se, expected)


@pytest.mark.parametrize("kind", [O.JUMP_MRZ_ADAPTIVE, O.JUMP_MRZ_CONST, O.JUMP_BPS])
def test_c_step_bound_holds_under_strong_acceleration(kind):
    """Starting at rest with a strong short force, the velocity grows during
    the half step; the bound B_v of Alg. 4 must still dominate every rate
    (no acceptance probability above one)."""
    sy = S.two_charges(L=12.0, r0=2.3, lj_eps=0.0)
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.2, coulomb_alpha=0.2)
    pa = S.Params(dt=0.02, gamma=0.0, kT=0.722, jump_coul=kind, eps=0.5)
    o = _oracle(sy, sp, pa)
    x0, _ = o.state()
    for k in range(300):
        o.set_state(vel=np.zeros_like(x0), step=k)
        o.phase_c(O.PH_C1, 0.8)
    st_ = o.atom_stats()
    assert st_["n_prop"].sum() > 1000 and st_["n_acc"].sum() > 100
    assert st_["n_viol"].sum() == 0


def _moment_check(o, phase_fn, h, K, kT, seed=11):
    """Mean velocity change over K independent half steps started from
    Maxwell-Boltzmann velocities, against h * a_full (here the short force is
    exactly zero, so the jumps alone must supply -grad U_long / m on average:
    the rate/kernel pair reproduces the missing force in the generator,
    Sec. 2.1-2.2, up to O(h^2)). Returns (chi2 of the mismatch, chi2 of the
    signal against zero, degrees of freedom)."""
    x0, v0 = o.state()
    expected = h * o.accel(O.F_FULL)
    assert np.abs(o.accel(O.F_SHORT)).max() == 0.0
    rng = np.random.default_rng(seed)
    dv = []
    for k in range(K):
        v = rng.standard_normal(v0.shape) * np.sqrt(kT)
        o.set_state(vel=v, step=k)
        phase_fn(h)
        dv.append(o.state()[1] - v)
    dv = np.array(dv)
    m, se = dv.mean(0), dv.std(0, ddof=1) / np.sqrt(K)
    still = se == 0.0                            # atoms that never jump (neutral): no drift either
    assert np.all(m[still] == 0.0) and np.all(np.abs(expected[still]) < 1e-15)
    z, z0 = (m - expected)[~still] / se[~still], m[~still] / se[~still]
    return float((z * z).sum()), float((z0 * z0).sum()), int(z.size)


@pytest.mark.parametrize("kind", [O.JUMP_MRZ_ADAPTIVE, O.JUMP_BPS])
def test_c_step_mean_kick_equals_long_force(kind):
    """Ions on a jittered lattice (+/- charges and neutral sites, 3 rings, all
    pairs beyond r_s): averaged over Maxwell-Boltzmann velocities, the C step
    (adaptive MRZ, or the BPS bounces) changes v by -h grad U_long / m. Detects
    a biased choice of proposal part, segment or index, a wrong floor count,
    jump size or sign."""
    sy = S.ion_lattice(4, 3.3, jitter=0.1, neutral_every=5)   # neutral third type: segments with l = 0
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.3, coulomb_alpha=0.2, n_rings=3,
                 ring_width=(5.3 - 1.7) / 3)
    pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_coul=kind, eps=0.3)
    o = _oracle(sy, sp, pa)
    chi2, signal, dof = _moment_check(o, lambda h: o.phase_c(O.PH_C1, h), 0.05, 20000, pa.kT)
    assert signal > 10 * dof                      # the drift is resolved
    assert st.chi2.sf(chi2, dof) > 1e-3, chi2


def _dv_moments(o, h, K, kT, seed=5):
    """Per-atom mean and mean square of the velocity change of one C step over
    K independent streams started from Maxwell-Boltzmann velocities."""
    x0, v0 = o.state()
    rng = np.random.default_rng(seed)
    dv = []
    for k in range(K):
        v = rng.standard_normal(v0.shape) * np.sqrt(kT)
        o.set_state(vel=v, step=k)
        o.phase_c(O.PH_C1, h)
        dv.append(o.state()[1] - v)
    dv = np.array(dv).reshape(K, -1)
    return dv.mean(0), (dv * dv).mean(0), dv.var(0, ddof=1), (dv * dv).var(0, ddof=1)


def test_mrz_large_eps_has_the_law_of_bps():
    """Sec. 2.2: the MRZ family interpolates between Hamiltonian drift (eps ->
    0) and the BPS bounces (eps -> infinity). With constant eps = 1e3 the mean
    and the mean square of the C-step velocity change match the BPS kernel's
    (two-sample chi-square over atoms and components); with eps = 0.3 the
    mean square differs (the test can tell the kernels apart)."""
    sy = S.ion_lattice(4, 3.3, jitter=0.1)
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=1.0, skin=0.3, coulomb_alpha=0.2, n_rings=3,
                 ring_width=(5.3 - 1.7) / 3)
    K, h = 4000, 0.05
    mom = {}
    for name, kind, eps in (("bps", O.JUMP_BPS, 0.0), ("big", O.JUMP_MRZ_CONST, 1e3),
                            ("small", O.JUMP_MRZ_CONST, 0.3)):
        pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_coul=kind, eps=eps)
        mom[name] = _dv_moments(_oracle(sy, sp, pa), h, K, pa.kT)

    def chi2_sf(a, b):
        m1, s1, vm1, vs1 = a
        m2, s2, vm2, vs2 = b
        zm = (m1 - m2) ** 2 / ((vm1 + vm2) / K)
        zs = (s1 - s2) ** 2 / ((vs1 + vs2) / K)
        z = np.concatenate([zm, zs])
        return st.chi2.sf(z.sum(), z.size)

    assert chi2_sf(mom["bps"], mom["big"]) > 1e-3
    assert chi2_sf(mom["bps"], mom["small"]) < 1e-6


def test_j_step_mean_kick_equals_long_lj_force():
    """Same identity for the BPS J step on the LJ long part (Sec. 3.2)."""
    sy = S.ion_lattice(4, 3.7, q=0.0, lj_eps=5.0, lj_sigma=2.0, jitter=0.1)
    sp = S.Split(r_s=3.5, r_c=6.0, switch_width=1.0, skin=0.3, n_rings=3, ring_width=(6.3 - 2.2) / 3)
    pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_lj=O.JUMP_BPS)
    o = _oracle(sy, sp, pa)
    chi2, signal, dof = _moment_check(o, lambda h: o.phase_j(O.PH_J1, h), 0.1, 10000, pa.kT)
    assert signal > 4 * dof
    assert st.chi2.sf(chi2, dof) > 1e-3, chi2


@pytest.mark.parametrize("kind", [O.JUMP_MRZ_ADAPTIVE, O.JUMP_BPS])
def test_c_step_with_lj_in_c_mean_kick_equals_whole_long_force(kind):
    """LJ long part in the C step (jump_lj IN_C): one chain per atom over the
    long part of the whole pair potential with the Coulomb kernel (bound
    l_LJ + l_Coulomb, floor over every candidate with l > 0). Averaged over
    Maxwell-Boltzmann velocities the C step changes v by -h grad U_long / m
    of both parts, on charged LJ ions where either part alone would miss;
    the Coulomb-only C step misses it."""
    sy = S.ion_lattice(4, 3.7, q=1.0, lj_eps=5.0, lj_sigma=2.0, jitter=0.1)
    sp = S.Split(r_s=3.5, r_c=6.0, switch_width=1.0, skin=0.3, coulomb_alpha=0.2, n_rings=3,
                 ring_width=(6.3 - 2.2) / 3)
    pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_lj=O.JUMP_IN_C, jump_coul=kind, eps=0.3)
    o = _oracle(sy, sp, pa)
    chi2, signal, dof = _moment_check(o, lambda h: o.phase_c(O.PH_C1, h), 0.1, 10000, pa.kT)
    assert signal > 4 * dof
    assert st.chi2.sf(chi2, dof) > 1e-3, chi2
    pa_c = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_coul=kind, eps=0.3)
    o2 = _oracle(sy, sp, pa_c)
    chi2_c, _, _ = _moment_check(o2, lambda h: o2.phase_c(O.PH_C1, h), 0.1, 10000, pa.kT)
    assert st.chi2.sf(chi2_c, dof) < 1e-6


def test_bounce_j_step_mean_kick_equals_whole_long_force():
    """BOUNCE (Sec. 3: bounces on the Coulomb part too, in the J step): one
    BPS chain per atom over the long part of the whole pair potential (LJ +
    Coulomb, bound l_LJ + l_Coulomb). Averaged over Maxwell-Boltzmann
    velocities the J step changes v by -h grad U_long / m of both parts;
    checked on charged LJ ions, where either part alone would miss."""
    sy = S.ion_lattice(4, 3.7, q=1.0, lj_eps=5.0, lj_sigma=2.0, jitter=0.1)
    sp = S.Split(r_s=3.5, r_c=6.0, switch_width=1.0, skin=0.3, coulomb_alpha=0.2, n_rings=3,
                 ring_width=(6.3 - 2.2) / 3)
    pa = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_lj=O.JUMP_BPS, jump_coul=O.JUMP_BOUNCE)
    o = _oracle(sy, sp, pa)
    chi2, signal, dof = _moment_check(o, lambda h: o.phase_j(O.PH_J1, h), 0.1, 10000, pa.kT)
    assert signal > 4 * dof
    assert st.chi2.sf(chi2, dof) > 1e-3, chi2
    # the Coulomb part matters here: the LJ chain alone misses its share of the force
    pa_lj = S.Params(dt=0.01, gamma=0.0, kT=1.0, jump_lj=O.JUMP_BPS)
    o2 = _oracle(sy, sp, pa_lj)
    chi2_lj, _, _ = _moment_check(o2, lambda h: o2.phase_j(O.PH_J1, h), 0.1, 10000, pa.kT)
    assert st.chi2.sf(chi2_lj, dof) < 1e-6


def test_bounce_thinning_exact_under_bound_inflation():
    """BOUNCE's J chain on water: inflating every bound x3 leaves the law of
    the velocity update unchanged (Sec. 2.4)."""
    sy, sp = S.water_box(125, seed=4), S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=0.5, n_rings=3)
    pa = S.water_params()
    pa.jump_coul = O.JUMP_BOUNCE
    res = []
    K = 150
    for scale in (1.0, 3.0):
        o = _oracle(sy, sp, pa)
        o.set_bound_scale(scale)
        x0, v0 = o.state()
        dv = []
        for k in range(K):
            o.set_state(vel=v0, step=1000 + k)
            o.phase_j(O.PH_J1, 0.0005)
            dv.append((o.state()[1] - v0).ravel())
        dv = np.array(dv)
        res.append((dv.mean(0), dv.var(0, ddof=1), o.atom_stats()["n_prop"].sum()))
    (m1, v1, p1), (m2, v2, p2) = res
    z2 = (m1 - m2) ** 2 / ((v1 + v2) / K + 1e-300)
    assert st.chi2.sf(z2.sum(), z2.size) > 1e-3
    assert p2 > 2.5 * p1


# ------------------------------------------------------------ Gibbs marginal
def _gibbs_reference(sy, sp, kT, edges):
    def u(r):
        t = O.pair_terms(r, sy.lj_eps[0], sy.lj_sigma[0], sy.charge[0] * sy.charge[1], sy.coulomb_k,
                         sp.coulomb_alpha, sp.r_s, sp.switch_width, sp.r_c)
        return t[0] + t[2]
    dens = lambda r: r * r * np.exp(-u(r) / kT)
    p = np.array([si.quad(dens, a, b, epsabs=1e-12)[0] for a, b in zip(edges[:-1], edges[1:])])
    return p / p.sum()


@pytest.mark.parametrize("scheme", ["jump", "jump_bps", "jump_respa", "baoab", "bounce", "jump_lj_in_c"])
def test_two_particle_gibbs_marginal(scheme):
    """Two charged LJ particles: the distance histogram (r < L/2) of a long run
    matches p(r) ~ r^2 exp(-beta U(r)) by quadrature, and <v^2> = kT/m.
    JUMP uses BPS for the LJ long part and adaptive MRZ (jump_bps: BPS
    bounces) for the Coulomb one; jump_respa runs them at the outer step of
    JUMP-RESPA with three inner steps (Sec. 3.3)."""
    sy = S.two_charges()
    sp = S.Split(r_s=3.0, r_c=5.0, switch_width=0.5, skin=0.3, coulomb_alpha=0.2)
    pa = S.Params(dt=0.005, gamma=2.0, kT=0.722, seed=3,
                  jump_lj={"baoab": 0, "jump_lj_in_c": O.JUMP_IN_C}.get(scheme, O.JUMP_BPS),
                  jump_coul={"jump": O.JUMP_MRZ_ADAPTIVE, "jump_bps": O.JUMP_BPS, "jump_respa": O.JUMP_MRZ_ADAPTIVE,
                             "baoab": 0, "bounce": O.JUMP_BOUNCE,
                             "jump_lj_in_c": O.JUMP_MRZ_ADAPTIVE}[scheme], eps=0.5)
    pa.respa_inner = 3
    o = _oracle(sy, sp, pa)
    L = sy.box[0]
    rs, v2 = [], []
    for _ in range(6000):
        if scheme == "jump_respa":
            o.step_jump_respa(34)
        else:
            (o.step_baoab if scheme == "baoab" else o.step_jump)(100)
        x, v = o.state()
        d = x[1] - x[0]
        d -= L * np.rint(d / L)
        rs.append(np.linalg.norm(d))
        v2.append((v * v).mean())
    rs = np.array(rs)
    edges = np.array([0.9, 1.1, 1.3, 1.6, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0])
    rsel = rs[rs < edges[-1]]
    cnt, _ = np.histogram(rsel, edges)
    p = _gibbs_reference(sy, sp, pa.kT, edges)
    exp = p * len(rsel)
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert st.chi2.sf(chi2, len(cnt) - 1) > 1e-3, (cnt, exp.round(1))
    assert abs(np.mean(v2) - pa.kT) < 0.03 * pa.kT
    if scheme != "baoab":   # the jumps act (BPS accepts only on approach, so far fewer)
        assert o.atom_stats()["n_acc"].sum() > (200 if scheme in ("jump_bps", "bounce") else 1000)


# ------------------------------------------------------------------- Ewald
MADELUNG_NACL = 1.747564594633182   # rock-salt Madelung constant (nearest-neighbour distance)


def test_ewald_madelung_constant_of_rock_salt():
    """Ewald electrostatics (damped shifted-force real part + reciprocal sum +
    self term) on a perfect rock-salt lattice of 512 unit charges, nearest
    neighbours at distance 1: the energy per ion is -M/2 k_e q^2 / a with the
    rock-salt Madelung constant M (real part converged: erfc(alpha r_c) ~ 1e-13;
    reciprocal sum converged: exp(-k^2 / 4 alpha^2) ~ 1e-13 at kmax)."""
    sy = S.ion_lattice(8, 1.0, q=1.0, coulomb_k=1.0, jitter=0.0)
    sp = S.Split(r_s=2.0, r_c=3.5, switch_width=0.5, skin=0.1, coulomb_alpha=1.5, coulomb_kind=1, ewald_kmax=21)
    e = _oracle(sy, sp, S.Params(dt=0.01, gamma=0.0, kT=1.0)).energies()
    per_ion = e["pe_full"] / sy.n_atoms
    assert abs(per_ion + MADELUNG_NACL / 2) < 1e-9, per_ion
    assert e["pe_recip"] != 0.0


@pytest.mark.parametrize("coul", ["mrz", "none"])
def test_jump_with_ewald_and_no_long_pairs_is_baoab(coul):
    """JUMP with Ewald electrostatics: the C' acceleration (or, without
    Coulomb jumps, the kick) carries the reciprocal-space forces, re-evaluated
    every step. Two charges 3.5 apart, the switch confined to [4.85, 4.9] =
    r_c: no pair or candidate reaches the long part, so C' J' A O A J' C' is
    B A O A B with the same forces and JUMP follows BAOAB to rounding. A
    dropped, doubled or stale reciprocal term fails (the reciprocal forces
    are a sizeable part of the total)."""
    sy = S.two_charges(L=10.0776, r0=3.5)
    sp = S.Split(r_s=4.9, r_c=4.9, switch_width=0.05, skin=0.3, coulomb_alpha=0.6, coulomb_kind=1, ewald_kmax=8)
    pa = S.Params(dt=0.005, gamma=2.0, kT=0.722, seed=5, jump_lj=O.JUMP_BPS,
                  jump_coul=O.JUMP_MRZ_ADAPTIVE if coul == "mrz" else 0, eps=0.5)
    o1, o2 = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    fr, ff = o1.accel(O.F_RECIP), o1.accel(O.F_FULL)
    assert np.abs(fr).max() > 0.05 * np.abs(ff).max()
    o1.step_baoab(40)
    o2.step_jump(40)
    x1, v1 = o1.state()
    x2, v2 = o2.state()
    assert rel_err(x2, x1) < 1e-12 and rel_err(v2, v1) < 1e-12
    assert o2.atom_stats()["n_prop"].sum() == 0


def _ewald_water(alpha, kmax, seed=9):
    sy = S.water_box(125, seed=seed, jitter=0.05)
    sp = S.water_split(r_s=5.0, r_c=7.5, w=1.0, skin=0.3, alpha=alpha, n_rings=3)
    sp.coulomb_kind, sp.ewald_kmax = 1, kmax
    return sy, sp


def test_ewald_sum_independent_of_alpha():
    """The Ewald total energy and forces do not depend on the splitting
    parameter alpha once both sums have converged. On water (bonded
    molecules whose intramolecular pairs are excluded) this also pins the
    excluded-pair correction and the self term: without them the reciprocal
    sum would count the excluded pairs by an alpha-dependent amount."""
    out = []
    for alpha, kmax in ((0.72, 19), (0.86, 23)):
        sy, sp = _ewald_water(alpha, kmax)
        o = _oracle(sy, sp, S.water_params())
        e = o.energies()
        f = o.accel(O.F_FULL) + o.accel(O.F_RECIP)
        out.append((e["pe_full"] - e["pe_bonded"], f, e["pe_recip"]))
    (e1, f1, r1), (e2, f2, r2) = out
    assert abs(r1 - r2) > 1.0                       # the split moved energy between the parts
    assert abs(e1 - e2) < 1e-9 * abs(e1), (e1, e2)
    assert rel_err(f1, f2) < 1e-8


def _spme_water(grid, order, alpha=0.3, seed=9):
    sy, sp = _ewald_water(alpha, 0, seed)
    sp.coulomb_kind, sp.pme_grid, sp.pme_order = O.COUL_SPME, grid, order
    return sy, sp


def test_spme_converges_to_the_ewald_sum():
    """Smooth particle-mesh Ewald approximates the plain reciprocal sum (its
    own pins above) by B-spline interpolation of the structure factor: on
    125 waters the reciprocal energy and forces agree with the converged
    plain sum to 1e-7 on a 32^3 grid with order 8, and the error falls as
    the grid and the order grow (16^3, order 4: about 1 %)."""
    sy, sp = _ewald_water(0.3, 12)
    ref = _oracle(sy, sp, S.water_params())
    e0, f0 = ref.energies()["pe_recip"], ref.accel(O.F_RECIP)
    errs = []
    for grid, order in (((16, 16, 16), 4), ((32, 32, 32), 8)):
        sy2, sp2 = _spme_water(grid, order)
        o = _oracle(sy2, sp2, S.water_params())
        e, f = o.energies()["pe_recip"], o.accel(O.F_RECIP)
        errs.append((abs(e - e0) / abs(e0), rel_err(f, f0)))
    assert errs[1][0] < 1e-7 and errs[1][1] < 5e-8, errs
    assert errs[0][0] > 100 * errs[1][0] and errs[0][1] > 100 * errs[1][1], errs


def test_spme_forces_are_minus_energy_gradient():
    """SPME forces (B-spline derivatives on the transformed grid) are minus
    the gradient of the SPME energy (central differences), on a grid that is
    not cubic."""
    sy, sp = _spme_water((16, 32, 16), 6)
    o = _oracle(sy, sp, S.water_params())
    me = sy.mass / sy.accel_factor
    fr = o.accel(O.F_RECIP) * me[:, None]
    h = 1e-5
    for i in (0, 1, 200):
        for c in range(3):
            xp, xm = sy.pos.copy(), sy.pos.copy()
            xp[i, c] += h
            xm[i, c] -= h
            o.set_state(pos=xp)
            ep = o.energies()["pe_recip"]
            o.set_state(pos=xm)
            em = o.energies()["pe_recip"]
            fd = -(ep - em) / (2 * h)
            assert abs(fr[i, c] - fd) < 1e-6 * max(1.0, abs(fd)), (i, c, fr[i, c], fd)


def test_ewald_forces_are_minus_energy_gradient():
    """Reciprocal-space forces (with the excluded-pair correction) and the
    real-space forces are minus the gradient of the total energy (central
    differences), at an alpha where the two parts are of similar size."""
    sy, sp = _ewald_water(0.3, 8)
    o = _oracle(sy, sp, S.water_params())
    me = sy.mass / sy.accel_factor
    f = (o.accel(O.F_FULL) + o.accel(O.F_RECIP)) * me[:, None]
    fr = o.accel(O.F_RECIP) * me[:, None]
    assert np.abs(fr).max() > 0.1 * np.abs(f).max()
    h = 1e-5
    for i in (0, 1, 200):
        for c in range(3):
            xp, xm = sy.pos.copy(), sy.pos.copy()
            xp[i, c] += h
            xm[i, c] -= h
            o.set_state(pos=xp)
            ep = o.energies()
            o.set_state(pos=xm)
            em = o.energies()
            fd = -((ep["pe_full"] - ep["pe_bonded"]) - (em["pe_full"] - em["pe_bonded"])) / (2 * h)
            assert abs(f[i, c] - fd) < 1e-5 * max(1.0, abs(fd)), (i, c, f[i, c], fd)
    o.set_state(pos=sy.pos)
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).sum()


def test_baoab_respa1_with_single_steps_is_baoab():
    """BAOAB-RESPA1 with one inner and one middle step per outer step is BAOAB
    with the same forces (bonded + short + long real part + reciprocal),
    split over several kicks: trajectories agree to rounding."""
    sy, sp = _ewald_water(0.3, 6)
    pa = S.water_params(jumps=False)
    pa.gamma = 1.0
    o1, o2 = _oracle(sy, sp, pa), _oracle(sy, sp, pa)
    o1.step_baoab(15)
    o2.step_baoab_respa1(15)
    x1, v1 = o1.state()
    x2, v2 = o2.state()
    assert rel_err(x2, x1) < 1e-12 and rel_err(v2, v1) < 1e-11
