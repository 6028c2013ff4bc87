"""Shared helpers of the GPU parity tests (seeded inputs, tolerances)."""
import functools

import numpy as np

from gen import fields
from oracle import evenodd

# Relative 2-norm tolerances of the Dslash/clover/Schur parity against the
# FP64 oracle applied to the unrounded FP64 input.
TOL = {0: 1e-12, 1: 1e-6, 2: 5e-3}
PREC_NAME = {0: "f64", 1: "f32", 2: "f16"}


def rel(a, b):
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


def site_rel_max(a, b):
    """Largest per-site relative error max_x |a_x - b_x| / |b_x| over the sites
    (12 complex components per site, the trailing (4, 3) axes), skipping sites
    whose reference is below 1e-12 of the largest site norm."""
    a = a.reshape(-1, 12)
    b = b.reshape(-1, 12)
    nb = np.linalg.norm(b, axis=1)
    keep = nb > 1e-12 * nb.max()
    return float(np.max(np.linalg.norm(a - b, axis=1)[keep] / nb[keep]))


def log_errors(label, got, ref):
    """Log the relative 2-norm error and the largest per-site relative error
    of a GPU result against the oracle; returns the former."""
    err = rel(got, ref)
    say(f"  {label}: relative error {err:.3e}, largest per-site relative error "
        f"{site_rel_max(got, ref):.3e}")
    return err


@functools.lru_cache(maxsize=4)
def case(dims, kind="smooth", seed=0):
    """Seeded gauge field, full Gaussian spinor and its even/odd halves
    (cached: the 32^3x64 links take tens of seconds to generate)."""
    u = fields.gauge_field(dims, kind, fields.SEED_GAUGE + seed)
    psi = fields.gaussian_spinor(dims, fields.SEED_SOURCE + seed)
    e, o = evenodd.split(psi, dims)
    return u, psi, e, o


def say(msg):
    print(msg, flush=True)


def residual_at(u, kappa, csw, x, b, site, antiperiodic_t=True):
    """(b - M x)(site) from the oracle, at one site of a lattice too large for
    the oracle's whole-lattice operator.  The clover term at a site depends
    only on links within one step of it, so it is taken from the oracle's
    clover matrix of the periodic 4^4 window of links starting one step below
    the site (every leaf at window index 1 stays inside the window); the
    hopping term is the oracle's single-site hop_at."""
    from oracle import clover as oclover
    from oracle import dirac
    lt, lz, ly, lx = u.shape[:4]
    ext = (lx, ly, lz, lt)
    idx = [[(site[d] - 1 + k) % ext[d] for k in range(4)] for d in range(4)]
    win = u[np.ix_(idx[3], idx[2], idx[1], idx[0])]
    a = oclover.clover_matrix(win, kappa, csw)[1, 1, 1, 1]
    xs = x[site[3], site[2], site[1], site[0]]
    mx = oclover.apply_site_matrix(a, xs) - kappa * dirac.hop_at(u, x, site,
                                                                  antiperiodic_t=antiperiodic_t)
    return b[site[3], site[2], site[1], site[0]] - mx
