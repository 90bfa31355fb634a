"""Comparison helpers for the GPU parity tests (test-side only)."""
import numpy as np


def f16(bits: np.ndarray) -> np.ndarray:
    return np.asarray(bits, np.uint16).view(np.float16).astype(np.float64)


def ulp16(x: np.ndarray) -> np.ndarray:
    """Spacing of binary16 numbers at |x| (2^-24 in the subnormal range)."""
    a = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))
    return np.ldexp(1.0, (e - 10).astype(int))


def excess_fp32(got, lo, hi, rel=1e-4, floor_frac=1e-3):
    """Largest violation of lo <= got <= hi, relative to the texel's
    magnitude (dark texels use floor_frac of the map's largest value)."""
    got = np.asarray(got, np.float64)
    scale = max(float(np.abs(hi).max()), 1e-30)
    den = np.maximum(np.maximum(np.abs(lo), np.abs(hi)), floor_frac * scale)
    ex = np.maximum(np.maximum(lo - got, got - hi), 0.0) / den
    return float(ex.max()), ex


def excess_fp16_ulps(got_bits, lo, hi):
    """Violation of lo <= got <= hi in binary16 ulps of the bound."""
    g = f16(got_bits)
    ex = np.maximum(np.maximum(lo - g, g - hi), 0.0) / ulp16(np.maximum(np.abs(lo), np.abs(hi)))
    return float(ex.max()), ex


def ulps_from(got_bits, ref):
    g = f16(got_bits)
    return np.abs(g - ref) / ulp16(np.maximum(np.abs(g), np.abs(ref)))


def fold_consistent(tiles: np.ndarray) -> bool:
    """Every guard texel equals the interior texel the octahedral fold puts
    next to it (property of a tile set [P, C, N+2, N+2])."""
    N = tiles.shape[-1] - 2
    T = tiles
    ok = True
    for x in range(1, N + 1):
        ok &= np.array_equal(T[..., 0, x], T[..., 1, N + 1 - x])
        ok &= np.array_equal(T[..., N + 1, x], T[..., N, N + 1 - x])
    for y in range(1, N + 1):
        ok &= np.array_equal(T[..., y, 0], T[..., N + 1 - y, 1])
        ok &= np.array_equal(T[..., y, N + 1], T[..., N + 1 - y, N])
    ok &= np.array_equal(T[..., 0, 0], T[..., N, N])
    ok &= np.array_equal(T[..., 0, N + 1], T[..., N, 1])
    ok &= np.array_equal(T[..., N + 1, 0], T[..., 1, N])
    ok &= np.array_equal(T[..., N + 1, N + 1], T[..., 1, 1])
    return bool(ok)


def hit_agreement(gpu_hits, rays):
    """(fraction equal to the oracle's nominal hit, fraction inside the
    oracle's accepted set)."""
    nom = rays["hit"]
    eq = gpu_hits == nom
    cand = rays["cand"]
    ok = eq.copy()
    for c in range(cand.shape[-1]):
        ok |= (cand[..., c] == gpu_hits) & (c < rays["ncand"])
    return float(eq.mean()), float(ok.mean())
