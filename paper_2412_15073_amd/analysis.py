"""Post-processing of quantities produced on the GPU (pair histograms from
md_rdf, unwrapped position snapshots from md_get_state): radial distribution
functions, mean-square displacement and the Einstein diffusion constant
(Sec. 4 of the paper compares RDF, temperature and diffusion constants of
JUMP against BAOAB)."""
import numpy as np


def rdf_from_counts(counts, n_a, n_b, volume, r_max, same_type, n_frames=1):
    """Normalise a pair histogram over [0, r_max) into g(r).

    counts: summed over n_frames; unordered pairs when same_type."""
    counts = np.asarray(counts, float)
    nb = len(counts)
    edges = np.linspace(0.0, r_max, nb + 1)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    pairs = n_a * (n_a - 1) / 2.0 if same_type else n_a * n_b
    ideal = pairs * shell / volume
    r = 0.5 * (edges[1:] + edges[:-1])
    return r, counts / (ideal * n_frames)


def rdf_l2(g1, g2):
    """RMS difference of two g(r) curves on the same bins."""
    g1, g2 = np.asarray(g1), np.asarray(g2)
    return float(np.sqrt(np.mean((g1 - g2) ** 2)))


def msd(frames, stride_origins=1):
    """Mean-square displacement of unwrapped positions, averaged over atoms
    and time origins. frames: [T, N, 3]. Returns msd[lag] for lag = 0..T-1."""
    X = np.asarray(frames, float)
    T = X.shape[0]
    out = np.zeros(T)
    cnt = np.zeros(T)
    for t0 in range(0, T, stride_origins):
        d = X[t0:] - X[t0]
        out[: T - t0] += (d * d).sum(-1).mean(-1)
        cnt[: T - t0] += 1
    return out / np.maximum(cnt, 1)


def diffusion_constant(msd_curve, dt_frame, t_fit=(0.2, 0.8), blocks=None):
    """Einstein relation D = slope(MSD)/6 fitted over a fraction window of the
    lags; returns D (length^2/time)."""
    m = np.asarray(msd_curve)
    T = len(m)
    a, b = int(t_fit[0] * (T - 1)), int(t_fit[1] * (T - 1))
    t = np.arange(T) * dt_frame
    slope = np.polyfit(t[a:b + 1], m[a:b + 1], 1)[0]
    return slope / 6.0


def block_diffusion(frames, dt_frame, n_blocks=4, t_fit=(0.2, 0.8)):
    """D from each of n_blocks consecutive segments: mean and standard error."""
    X = np.asarray(frames)
    L = X.shape[0] // n_blocks
    ds = [diffusion_constant(msd(X[k * L:(k + 1) * L]), dt_frame, t_fit) for k in range(n_blocks)]
    ds = np.array(ds)
    return float(ds.mean()), float(ds.std(ddof=1) / np.sqrt(n_blocks))
