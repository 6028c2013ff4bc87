"""Pins of the oracle's preconditioner net: Neumann identity, finite
differences of the loss, gauge equivariance."""
import numpy as np

from gen import fields
from oracle import dirac, evenodd, net
from tests.test_oracle_dirac import gauge_rotate


def test_neumann_initialisation_is_truncated_series():
    dims = (4, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 201)
    psi = fields.gaussian_spinor(dims, 202)
    kappa = 0.12
    w = net.neumann_weights(kappa)
    y = net.forward(u, w, psi)[-1]
    # sum_{n=0..4} (kappa H)^n psi from the hopping term itself
    term = psi.copy()
    ref = psi.copy()
    for _ in range(4):
        term = kappa * dirac.hop(u, term)
        ref = ref + term
    assert dirac.norm(y - ref) <= 1e-13 * dirac.norm(ref)


def test_single_layer_with_projector_weights_is_wilson():
    """W0 = 1, Wp = -kappa (1 - g), Wm = -kappa (1 + g) is M_W = 1 - kappa H."""
    dims = (2, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 211)
    psi = fields.gaussian_spinor(dims, 212)
    w = np.zeros((1, 9, 4, 4), dtype=np.complex128)
    w[0, 0] = np.eye(4)
    for mu in range(4):
        w[0, 1 + 2 * mu] = -0.1 * (np.eye(4) - dirac.GAMMA[mu])
        w[0, 2 + 2 * mu] = -0.1 * (np.eye(4) + dirac.GAMMA[mu])
    y = net.forward(u, w, psi)[-1]
    assert dirac.norm(y - dirac.wilson(u, psi, 0.1)) <= 1e-14 * dirac.norm(y)


def random_weights(seed, nl=4, scale=0.3):
    g = fields.rng(seed)
    return fields.complex_gaussian(g, (nl, 9, 4, 4)) * scale


def test_loss_gradient_finite_differences():
    dims = (4, 4, 4, 4)
    u = fields.gauge_field(dims, "smooth", 221)
    w = random_weights(222)
    srcs = [evenodd.split(fields.gaussian_spinor(dims, 223 + i), dims)[0] for i in range(2)]
    tgts = [evenodd.split(fields.gaussian_spinor(dims, 233 + i), dims)[0] for i in range(2)]
    loss, g = net.loss_and_grad(u, w, srcs, tgts, dims)
    rng = fields.rng(240)
    h = 1e-5
    for _ in range(8):
        l, k, s, t = (int(rng.integers(4)), int(rng.integers(9)),
                      int(rng.integers(4)), int(rng.integers(4)))
        for part, unit in (("re", 1.0), ("im", 1j)):
            wp = w.copy()
            wm = w.copy()
            wp[l, k, s, t] += h * unit
            wm[l, k, s, t] -= h * unit
            lp, _ = net.loss_and_grad(u, wp, srcs, tgts, dims)
            lm, _ = net.loss_and_grad(u, wm, srcs, tgts, dims)
            fd = (lp - lm) / (2 * h)
            an = 2 * (g[l, k, s, t].real if part == "re" else g[l, k, s, t].imag)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (l, k, s, t, part, fd, an)


def test_input_gradient_finite_differences():
    dims = (2, 4, 2, 4)
    u = fields.gauge_field(dims, "haar", 251)
    w = random_weights(252)
    psi = fields.gaussian_spinor(dims, 253)
    tgt = fields.gaussian_spinor(dims, 254)

    def loss_of(p):
        y = net.forward(u, w, p)[-1]
        return float(np.vdot(y - tgt, y - tgt).real)

    acts = net.forward(u, w, psi)
    _, gin = net.backward(u, w, acts, acts[-1] - tgt)
    rng = fields.rng(255)
    # the loss is quadratic in psi: central differences are exact up to rounding
    h = 1e-3
    flat = psi.reshape(-1)
    for _ in range(6):
        j = int(rng.integers(flat.size))
        for unit in (1.0, 1j):
            e = np.zeros_like(flat)
            e[j] = h * unit
            fd = (loss_of((flat + e).reshape(psi.shape))
                  - loss_of((flat - e).reshape(psi.shape))) / (2 * h)
            gj = gin.reshape(-1)[j]
            an = 2 * (gj.real if unit == 1.0 else gj.imag)
            assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_net_gauge_equivariance():
    dims = (4, 2, 4, 4)
    u = fields.gauge_field(dims, "haar", 261)
    g = fields.gauge_transform(dims, 262)
    w = random_weights(263)
    psi = fields.gaussian_spinor(dims, 264)
    lhs = net.forward(gauge_rotate(u, g), w, dirac.colour_mul(g, psi))[-1]
    rhs = dirac.colour_mul(g, net.forward(u, w, psi)[-1])
    assert dirac.norm(lhs - rhs) <= 1e-13 * dirac.norm(rhs)
