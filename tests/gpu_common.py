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
