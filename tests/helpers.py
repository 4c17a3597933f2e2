"""Shared test helpers: small seeded workloads and comparison utilities."""
import numpy as np

from paper_2412_15073_amd import systems as S


def lj_small(seed=1):
    """256 LJ atoms (fcc 4x4x4x4), box 6.72 sigma; split 2.0 / 3.0 sigma."""
    return S.lj_fcc(4, seed=seed, jitter=0.08), S.Split(r_s=2.0, r_c=3.0, switch_width=0.5, skin=0.3)


def lj_c1(seed=1, n_rings=1):
    """864 LJ atoms, the full LJ workload: split 3.0 / 5.0 sigma, skin 0.3."""
    sp = S.lj_split(skin=0.3, n_rings=n_rings,
                    ring_width=0.0 if n_rings == 1 else (5.3 - 2.2) / n_rings)
    return S.lj_fcc(6, seed=seed), sp


def water_small(n_mol=125, seed=3, n_rings=3, skin=0.5, jitter=0.05):
    """125 flexible waters (box 15.5 A), geometry jittered by 0.05 A; split 5 / 7 A, switch 1 A."""
    return (S.water_box(n_mol, seed=seed, jitter=jitter),
            S.water_split(r_s=5.0, r_c=7.0, w=1.0, skin=skin, n_rings=n_rings))


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def event_mix(h, step, phase, j):
    """Per-atom fingerprint update for one accepted jump (step, phase, partner):
    h <- (h xor key) * C, then h xor (h >> 29), all modulo 2^64."""
    m = 0xFFFFFFFFFFFFFFFF
    key = (step * 0x9E3779B97F4A7C15 + (phase & 0xFFFFFFFF) * 0xC2B2AE3D27D4EB4F + (j & 0xFFFFFFFF)) & m
    h = ((h ^ key) * 0xFF51AFD7ED558CCD) & m
    return h ^ (h >> 29)


def fnv1a64(h, data: bytes):
    for c in data:
        h ^= c
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h
