"""Pins of the oracle's explicit MPS operators (Section 2, MPS subsection):
the weight (eq. mpsw), the particle number density (eq. mpspnd), the
gradient (eq. mpsgrad), the Laplacian (eqs. mpslap, mpslambda) and the
two-criteria free-surface test (eqs. mpsni, mpsisgmai1, mpssigmai2).

* Continuum limits derived here: n0 l0^3 -> (2 pi / 3) r_e^3 and
  lambda0 -> 0.3 r_e^2 (the ratio of int r^4 w dr to int r^2 w dr).
* On a full cubic lattice, at interior points: the density equals n0, the
  Laplacian of |r|^2 is 2 dim = 6 (this is what lambda0 normalises), the
  Laplacian of a linear field is 0, the gradient of a linear field is exact
  (cubic symmetry makes the second moment isotropic), sigma is 0.
* The free-surface test flags a block's top layer, not its interior, and not
  an interior particle that has lost one neighbour (its density drops below
  beta1 n0 but the centroid barely moves).
"""
import math

import numpy as np
import pytest

from paper_2306_01959_amd import scene

RE_K = 2.1           # r_e = 2.1 l0 (the paper's MPS runs)
BETA1, RHO1 = 0.98, 0.2


def test_weight_values(oracle_lib):
    orc = oracle_lib
    re = 0.021
    assert orc.mps_weight(re / 2, re) == pytest.approx(1.0, rel=1e-15)
    assert orc.mps_weight(re, re) == 0.0
    assert orc.mps_weight(1.5 * re, re) == 0.0
    assert orc.mps_weight(0.0, re) == 0.0            # coincident particles left out
    r = np.linspace(0.01, 0.99, 50) * re
    w = np.array([orc.mps_weight(v, re) for v in r])
    assert np.all(np.diff(w) < 0) and np.all(w > 0)


def test_lattice_constants_continuum_limit(oracle_lib):
    orc = oracle_lib
    errs = []
    for k in (4.0, 8.0, 16.0):
        n0, lam = orc.mps_lattice(1.0, k)
        errs.append((abs(n0 / (2.0 * math.pi / 3.0 * k ** 3) - 1), abs(lam / (0.3 * k * k) - 1)))
    errs = np.array(errs)
    assert np.all(np.diff(errs, axis=0) < 0)           # converging
    assert np.all(errs[-1] < 0.01), errs
    n0a, lama = orc.mps_lattice(0.01, RE_K * 0.01)
    n0b, lamb = orc.mps_lattice(1.0, RE_K)
    assert n0a == pytest.approx(n0b, rel=1e-12)        # scale free
    assert lama == pytest.approx(lamb * 1e-4, rel=1e-12)


def _block(n, l0, corner=(0.1, 0.1, 0.1)):
    k = np.arange(n)
    zz, yy, xx = np.meshgrid(k, k, k, indexing="ij")
    return (corner[0] + xx.ravel() * l0, corner[1] + yy.ravel() * l0,
            corner[2] + zz.ravel() * l0)


def _grid(l0):
    re = RE_K * l0
    return scene.make_params(l0, h_factor=re / (2 * l0), lo=(0.0, 0.0, 0.0), hi=(0.5,) * 3)


def test_operators_on_full_lattice(oracle_lib):
    orc = oracle_lib
    l0 = 2.0 ** -7                     # exact lattice coordinates
    re = RE_K * l0
    n0, lam = orc.mps_lattice(l0, re)
    prm = _grid(l0)
    p = orc.par(prm)
    x, y, z = _block(12, l0, corner=(0.125, 0.125, 0.125))
    c = np.array([0.125 + 5.5 * l0] * 3)
    inner = np.max(np.abs(np.stack([x, y, z], 1) - c), axis=1) < 2.0 * l0
    assert inner.sum() == 64
    # |r - c|^2: Laplacian 6
    phi = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    pnd, lap, grad, sig, surf = orc.mps_operators(p, x, y, z, phi, re, n0, lam, BETA1, RHO1, l0)
    assert np.allclose(pnd[inner], n0, rtol=1e-13)
    assert np.allclose(lap[inner], 6.0, rtol=1e-11)
    assert np.all(sig[inner] < 1e-12 * l0) and not surf[inner].any()
    # linear field: Laplacian 0, gradient exact
    a = np.array([0.3, -1.2, 2.5])
    phi = a[0] * x + a[1] * y + a[2] * z
    _, lap, grad, _, _ = orc.mps_operators(p, x, y, z, phi, re, n0, lam, BETA1, RHO1, l0)
    assert np.abs(lap[inner]).max() < 1e-9 * np.abs(a).max() / l0
    for k in range(3):
        assert np.allclose(grad[k][inner], a[k], rtol=1e-12, atol=1e-12)


def test_free_surface_two_criteria(oracle_lib):
    orc = oracle_lib
    l0 = 2.0 ** -7
    re = RE_K * l0
    n0, lam = orc.mps_lattice(l0, re)
    p = orc.par(_grid(l0))
    x, y, z = _block(10, l0, corner=(0.125, 0.125, 0.125))
    top = z == z.max()
    deep = (np.minimum.reduce([x - x.min(), y - y.min(), z - z.min(),
                               x.max() - x, y.max() - y, z.max() - z]) >= 3 * l0 - 1e-12)
    pnd, _, _, sig, surf = orc.mps_operators(p, x, y, z, None, re, n0, lam, BETA1, RHO1, l0)
    assert surf[top].all()
    assert not surf[deep].any() and deep.sum() > 0
    # the top layer's centroid is pulled down: sigma along -z, well above 0.2 l0
    assert np.all(sig[top] > RHO1 * l0)
    # an interior particle that lost one neighbour at distance l0: its density
    # drops below beta1 n0, its centroid moves by 1.1 l0 / (n0 - 1.1) only
    c = np.argmin((x - x.mean()) ** 2 + (y - y.mean()) ** 2 + (z - z.mean()) ** 2)
    gone = np.argmin((x - x[c] - l0) ** 2 + (y - y[c]) ** 2 + (z - z[c]) ** 2)
    keep = np.arange(x.size) != gone
    xs, ys, zs = x[keep], y[keep], z[keep]
    c2 = c - (1 if gone < c else 0)
    pnd2, _, _, sig2, surf2 = orc.mps_operators(p, xs, ys, zs, None, re, n0, lam, BETA1, RHO1,
                                               l0)
    assert pnd2[c2] == pytest.approx(n0 - 1.1, rel=1e-12)
    assert pnd2[c2] < BETA1 * n0
    assert sig2[c2] == pytest.approx(1.1 * l0 / (n0 - 1.1), rel=1e-12)
    assert surf2[c2] == 0
