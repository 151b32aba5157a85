"""Pins of the multipole oracle (Eq. 4, complete basis, and its (p+1)^2 reduction).

The oracle's sums are checked against facts that do not depend on how it loops:
  * M^{000} is the cell's particle count (numpy bincount of numpy floors);
  * every complete term equals numpy's product of powers of the displacement
    from the cell centre, taken from the positions (not from the binned offsets)
    on a dyadic grid where both are exact;
  * the expansion sum (-1)^n M^{abc}/(a!b!c!) d^{abc}(1/r) reproduces the direct
    potential sum_q 1/|r - x_q| at a distant point within the truncation bound,
    with the derivatives of 1/r built exactly as integer polynomials;
  * the reduced values give the same potential as the complete ones;
  * mirror symmetry zeroes the odd moments, and doubling the box scales an
    order-n term by 2^n exactly.
"""
import math
from functools import lru_cache

import numpy as np
import pytest

import brute
import oracle
from paper_2110_11392_amd import synth


def complete_indices(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def reduced_indices(p):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a)
            for c in range(min(1, p - a - b) + 1)]


# ---- exact derivatives of 1/r: d^{abc}(1/r) = P_{abc}(x, y, z) / r^(2n+1) ----

def _poly_mul(p, q):
    out = {}
    for (i, j, k), u in p.items():
        for (l, m, n), v in q.items():
            key = (i + l, j + m, k + n)
            out[key] = out.get(key, 0) + u * v
    return {k: v for k, v in out.items() if v}


def _poly_add(p, q, s=1):
    out = dict(p)
    for k, v in q.items():
        out[k] = out.get(k, 0) + s * v
    return {k: v for k, v in out.items() if v}


def _poly_diff(p, axis):
    out = {}
    for e, v in p.items():
        if e[axis]:
            f = list(e)
            f[axis] -= 1
            out[tuple(f)] = out.get(tuple(f), 0) + v * e[axis]
    return out


R2 = {(2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1}
UNIT = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


@lru_cache(maxsize=None)
def deriv_poly(a, b, c):
    """P with d^a/dx^a d^b/dy^b d^c/dz^c (1/r) = P / r^(2(a+b+c)+1), integer coefficients."""
    if a == b == c == 0:
        return ((((0, 0, 0), 1),),)[0]
    if a:
        prev, axis, n = deriv_poly(a - 1, b, c), 0, a - 1 + b + c
    elif b:
        prev, axis, n = deriv_poly(a, b - 1, c), 1, b - 1 + c
    else:
        prev, axis, n = deriv_poly(a, b, c - 1), 2, c - 1
    P = dict(prev)
    # d/dx [P r^-(2n+1)] = [r^2 dP/dx - (2n+1) x P] r^-(2n+3)
    term1 = _poly_mul(R2, _poly_diff(P, axis))
    term2 = _poly_mul({UNIT[axis]: 2 * n + 1}, P)
    return tuple(sorted(_poly_add(term1, term2, -1).items()))


def deriv(a, b, c, r):
    x, y, z = r
    rr = math.sqrt(x * x + y * y + z * z)
    val = sum(float(v) * x ** i * y ** j * z ** k for (i, j, k), v in deriv_poly(a, b, c))
    return val / rr ** (2 * (a + b + c) + 1)


def expansion(moments, indices, r):
    return sum((-1) ** (a + b + c) * m / (math.factorial(a) * math.factorial(b) * math.factorial(c))
               * deriv(a, b, c, r) for m, (a, b, c) in zip(moments, indices))


def test_derivative_polynomials_are_harmonic():
    """Sanity of the exact derivatives: the Laplacian of every d^{abc}(1/r) vanishes."""
    r = (0.37, -0.81, 0.52)
    for (a, b, c) in complete_indices(5):
        lap = deriv(a + 2, b, c, r) + deriv(a, b + 2, c, r) + deriv(a, b, c + 2, r)
        assert abs(lap) <= 1e-10 * max(abs(deriv(a + 2, b, c, r)), 1.0)


# ---- pins -------------------------------------------------------------------

def dyadic_positions(n, seed, bits=18):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2 ** bits, size=(n, 3)) / 2 ** bits).astype(np.float32)


def test_terms_count():
    for p in range(0, 12):
        assert oracle.multipole_terms(p) == (p + 3) * (p + 2) * (p + 1) // 6
        assert oracle.multipole_terms(p, reduced=True) == (p + 1) ** 2
        assert len(complete_indices(p)) == oracle.multipole_terms(p)
        assert len(reduced_indices(p)) == oracle.multipole_terms(p, reduced=True)


@pytest.mark.parametrize("p", [0, 3, 8])
def test_monopole_is_the_cell_count(p):
    pos = synth.clustered(3000, 7, 6, 201)
    M = oracle.multipoles(pos, 1.0, 6, p)
    c = brute.cells(pos, 1.0, 6)
    counts = np.bincount((c[:, 0] * 6 + c[:, 1]) * 6 + c[:, 2], minlength=216)
    assert np.array_equal(M[:, 0], counts.astype(np.float64))


@pytest.mark.parametrize("p,K,box", [(8, 5, 1.0), (4, 7, 2.0)])
def test_every_term_matches_numpy_powers(p, K, box):
    pos = (dyadic_positions(1500, 202 + K) * np.float32(box)).astype(np.float32)
    M = oracle.multipoles(pos, box, K, p)
    w = box / K
    x = pos.astype(np.float64)
    cu = np.floor(x / w)
    disp = x - (cu + 0.5) * w            # exact on this dyadic grid
    c = np.mod(cu.astype(np.int64), K)
    cell = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    for k, (a, b, cc) in enumerate(complete_indices(p)):
        mono = disp[:, 0] ** a * disp[:, 1] ** b * disp[:, 2] ** cc
        ref = np.bincount(cell, weights=mono, minlength=K ** 3)
        scale = np.bincount(cell, weights=np.abs(mono), minlength=K ** 3) + 1e-300
        assert np.all(np.abs(M[:, k] - ref) <= 1e-13 * scale), (a, b, cc)


@pytest.mark.parametrize("p", [4, 8])
def test_expansion_reproduces_the_potential(p):
    """Complete and reduced multipoles both reproduce sum 1/|r - x_q| outside
    the cell to the order-p truncation error."""
    K = 4
    w = 1.0 / K
    pos = synth.clustered(600, 3, K, 203 + p)
    M = oracle.multipoles(pos, 1.0, K, p)
    Rm = oracle.multipoles(pos, 1.0, K, p, reduced=True)
    c = brute.cells(pos, 1.0, K)
    cell = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    target = int(np.argmax(M[:, 0]))
    members = pos[cell == target].astype(np.float64)
    cx, cy, cz = target // (K * K), (target // K) % K, target % K
    centre = (np.array([cx, cy, cz]) + 0.5) * w
    disp = members - centre
    disp -= np.rint(disp)                 # the cell's own image
    for direction in ([1.0, 0.3, -0.2], [-0.4, 0.9, 0.7], [0.1, -0.2, -1.0]):
        u = np.array(direction) / np.linalg.norm(direction)
        r = 6.0 * w * u
        direct = float(np.sum(1.0 / np.linalg.norm(r - disp, axis=1)))
        full = expansion(M[target], complete_indices(p), tuple(r))
        red = expansion(Rm[target], reduced_indices(p), tuple(r))
        rho = np.sqrt(3) / 2 * w
        bound = disp.shape[0] / np.linalg.norm(r) * (rho / np.linalg.norm(r)) ** (p + 1) / (
            1 - rho / np.linalg.norm(r))
        assert abs(full - direct) <= bound
        assert red == pytest.approx(full, rel=1e-12, abs=1e-12 * abs(direct))


def test_mirror_symmetry_zeroes_odd_moments():
    K, p = 4, 6
    w = 1.0 / K
    base = (dyadic_positions(100, 204, bits=12) * np.float32(w)).astype(np.float32)
    base = base[base[:, 0] > 0]           # its mirror 2c - x then stays inside cell (0, 0, 0)
    mirrored = base.copy()
    mirrored[:, 0] = np.float32(w) - base[:, 0]
    pos = np.concatenate([base, mirrored]).astype(np.float32)
    assert np.all((pos >= 0) & (pos < w))
    M = oracle.multipoles(pos, 1.0, K, p)
    for k, (a, b, c) in enumerate(complete_indices(p)):
        if a % 2:
            assert abs(M[0, k]) <= 1e-15 * np.abs(M[0]).max(), (a, b, c)


def test_doubling_the_box_scales_order_n_by_2n():
    pos = dyadic_positions(800, 205)
    p = 8
    M1 = oracle.multipoles(pos, 1.0, 5, p)
    M2 = oracle.multipoles((pos * np.float32(2.0)).astype(np.float32), 2.0, 5, p)
    n = np.array([a + b + c for (a, b, c) in complete_indices(p)])
    assert np.array_equal(M2, M1 * 2.0 ** n[None, :])


def test_multipoles_reject_bad_order():
    with pytest.raises(oracle.OracleError):
        oracle.multipoles(synth.uniform(10, 1), 1.0, 4, -1)
