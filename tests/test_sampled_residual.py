"""The single-site oracle residual used to check solutions of lattices too
large for the whole-lattice oracle, against that whole-lattice oracle on a
small lattice (every site, boundary sites in t included)."""
import numpy as np

from gen import fields
from oracle import evenodd
from tests.gpu_common import residual_at


def test_residual_at_matches_whole_lattice():
    dims = (6, 4, 2, 6)
    u = fields.gauge_field(dims, "haar", fields.SEED_GAUGE + 7)
    x = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 7)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 8)
    kappa, csw = 0.13, 1.3
    ref = b - evenodd.WilsonClover(u, kappa, csw).M(x)
    lx, ly, lz, lt = dims
    worst = 0.0
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for xx in range(lx):
                    r = residual_at(u, kappa, csw, x, b, (xx, y, z, t))
                    worst = max(worst, float(np.abs(r - ref[t, z, y, xx]).max()))
    assert worst < 1e-12, worst


def test_residual_at_periodic_t():
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "haar", fields.SEED_GAUGE + 8)
    x = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 9)
    b = np.zeros_like(x)
    ref = b - evenodd.WilsonClover(u, 0.12, 1.0, antiperiodic_t=False).M(x)
    for site in [(0, 0, 0, 0), (3, 1, 2, 3), (1, 3, 0, 0)]:
        r = residual_at(u, 0.12, 1.0, x, b, site, antiperiodic_t=False)
        assert np.abs(r - ref[site[3], site[2], site[1], site[0]]).max() < 1e-12
