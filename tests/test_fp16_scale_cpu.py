"""The automatic FP16 storage scales the headers state (k = 10 on D2Q9, 11 on D3Q19, 8 on
D3Q27), recomputed by brute force: the largest |S (f_i^eq - w_i rho0)| over a grid of
states with 0 < rho <= 2 rho0 and |u| <= 0.5 (velocities on spheres of several radii in
many directions, plus each lattice direction itself), with the oracle's lattice tables,
must fit 2^k times into half of FP16's largest finite value, and not 2^(k+1) times."""
import itertools

import numpy as np
import pytest

from oracle import binding as o2
from oracle import binding3d as o3

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _max_dev(c, w, S, rho0=1.0):
    d = c.shape[1]
    rng = np.random.default_rng(3)
    dirs = rng.normal(size=(4000, d))
    dirs = np.vstack([dirs, c[np.abs(c).sum(1) > 0]]).astype(float)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    m = 0.0
    for r in np.linspace(0.0, 0.5, 11):
        u = r * dirs
        cu = u @ c.T.astype(float)
        h = 1.0 + 3.0 * cu + 4.5 * cu**2 - 1.5 * (u * u).sum(1, keepdims=True)
        for rho in np.linspace(1e-3, 2.0, 41) * rho0:
            m = max(m, np.abs(S * (rho * w * h - w * rho0)).max())
    return m


@pytest.mark.parametrize("name,k", [("D2Q9", 10), ("D3Q19", 11), ("D3Q27", 8)])
def test_automatic_scale_matches_the_stated_bound(name, k):
    if name == "D2Q9":
        cx, cy, w, _ = o2.lattice()
        c, S = np.stack([cx, cy], 1), 36.0
    else:
        q = int(name[3:])
        cx, cy, cz, w, _ = o3.lattice(q)
        c, S = np.stack([cx, cy, cz], 1), 36.0 if q == 19 else 216.0
    m = _max_dev(c, w, S)
    half = 65504.0 / 2
    assert m * 2.0**k <= half < m * 2.0 ** (k + 1)
    # the bound scales with rho0
    assert _max_dev(c, w, S, rho0=4.0) == pytest.approx(4.0 * m, rel=1e-12)
