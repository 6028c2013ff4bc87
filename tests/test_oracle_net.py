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


def test_adam_constant_gradient_closed_form():
    """With the same gradient at every step the bias-corrected moments are
    exactly g and g^2, so every step moves each real parameter by
    lr * |g| / (|g| + eps) against the sign of its gradient, for any t (a
    missing or wrong bias correction changes the steps with t)."""
    g = np.array([[0.3 - 2.0j, -1e-3 + 0.7j]])
    w0 = np.array([[1.0 + 1.0j, -0.5 + 0.25j]])
    lr, eps = 0.01, 1e-8
    opt = net.Adam(w0.shape, lr=lr, beta1=0.9, beta2=0.999, eps=eps)
    w = w0.copy()
    for t in range(1, 8):
        w = opt.step(w, g)
        gr, gi = 2 * g.real, 2 * g.imag
        ref = w0 - t * lr * (gr / (np.abs(gr) + eps) + 1j * gi / (np.abs(gi) + eps))
        assert np.max(np.abs(w - ref)) <= 1e-14, t


def test_adam_two_steps_are_weighted_means():
    """After gradients g1, g2 the bias-corrected moments are the normalised
    weighted means (b1 g1 + g2) / (1 + b1) and (b2 g1^2 + g2^2) / (1 + b2)
    of the real gradients; the second step is lr times their quotient."""
    rng = fields.rng(270)
    g1 = fields.complex_gaussian(rng, (2, 3))
    g2 = fields.complex_gaussian(rng, (2, 3))
    w0 = fields.complex_gaussian(rng, (2, 3))
    b1, b2, lr, eps = 0.8, 0.95, 0.05, 1e-8
    opt = net.Adam(w0.shape, lr=lr, beta1=b1, beta2=b2, eps=eps)
    w1 = opt.step(w0, g1)
    w2 = opt.step(w1, g2)
    for part, unit in ((np.real, 1.0), (np.imag, 1j)):
        a1, a2 = 2 * part(g1), 2 * part(g2)
        step1 = lr * a1 / (np.abs(a1) + eps)
        mhat = (b1 * a1 + a2) / (1 + b1)
        vhat = (b2 * a1 * a1 + a2 * a2) / (1 + b2)
        step2 = lr * mhat / (np.sqrt(vhat) + eps)
        assert np.max(np.abs(part(w2) - (part(w0) - step1 - step2))) <= 1e-14
    # the moments are rescaled by their bias factors, not carried raw
    assert opt.t == 2


def test_adam_is_invariant_to_gradient_scale():
    """Adam's steps do not depend on a positive scale of the gradients (up to
    eps): 1e3 g and g give the same trajectory."""
    rng = fields.rng(271)
    gs = [fields.complex_gaussian(rng, (4,)) for _ in range(5)]
    w0 = fields.complex_gaussian(rng, (4,))
    a = net.Adam(w0.shape, lr=0.02, eps=1e-12)
    b = net.Adam(w0.shape, lr=0.02, eps=1e-12)
    wa, wb = w0.copy(), w0.copy()
    for g in gs:
        wa = a.step(wa, g)
        wb = b.step(wb, 1e3 * g)
    assert np.max(np.abs(wa - wb)) <= 1e-12
