"""Gauge-covariant linear preconditioner net (FP64 oracle, test infrastructure).

The paper uses a flexible outer Krylov method (FGCR, equal to FGMRES) because
it tolerates a preconditioner that is not a fixed linear operator (section
5); it does not describe a learned preconditioner.  The net here is a
stack of linear, gauge-covariant nearest-neighbour layers:

    psi_{l+1}(x) = W0 psi_l(x)
                   + sum_mu [ Wp_mu U_mu(x) psi_l(x+mu) + Wm_mu U_mu(x-mu)^dagger psi_l(x-mu) ],

each W a complex 4x4 matrix acting on spin only (colour-acting weights would
break gauge covariance), with the fermion boundary conditions of the
hopping term.  No bias and no nonlinearity.  Weight index k per layer:
0 = W0, 1 + 2 mu = Wp_mu, 2 + 2 mu = Wm_mu (9 matrices, 144 complex numbers).

On the even-odd system the net acts as N_e = P_e N E_e: embed an even
field with zeros on odd sites, apply, keep the even sites.

Neumann initialisation: W0 = 1, Wp_mu = -(kappa/w_l)(1 - gamma_mu),
Wm_mu = -(kappa/w_l)(1 + gamma_mu), w_l = exp(2 pi i l / 5), l = 1..4, makes
layer l equal to 1 - (kappa/w_l) H and the net equal to
sum_{n=0..4} (kappa H)^n.

Gradients use the Wirtinger convention: for y = sum_k W_k T_k psi and an
upstream g = dL/d conj(y),
    dL/d conj(W_k) = sum_{x, colour} g(x) (T_k psi)(x)^dagger,
    dL/d conj(psi) = sum_k T_k^dagger W_k^dagger g,
and the real gradients are dL/dRe W = 2 Re(dL/d conj W), dL/dIm W = 2 Im(...).

Training uses Adam (Kingma and Ba's published rule) on the real parameters
(Re W, Im W) with the real gradient above: first and second moment averages
with decay rates beta1, beta2, both divided by their bias factors
(1 - beta^t) at step t, and the step lr * m_hat / (sqrt(v_hat) + eps).

Pins (CPU tests): the Neumann identity against the hopping term; central
finite differences of the loss; gauge equivariance N[U'](g psi) = g N[U] psi;
Adam against its closed forms (a constant gradient gives steps of exactly
lr * |g| / (|g| + eps) at every t; two steps give the bias-corrected weighted
means (beta g1 + g2) / (1 + beta) of the gradients and of their squares).
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, ONE4, colour_mul, colour_mul_dag, shift, spin_mul
from . import evenodd as _eo

NK = 9


def transports(u, psi, antiperiodic_t=True):
    """[T_0 psi, T_{0+} psi, T_{0-} psi, ..., T_{3-} psi]."""
    out = [psi]
    for mu in range(4):
        u_mu = u[..., mu, :, :]
        out.append(colour_mul(u_mu, shift(psi, mu, +1, antiperiodic_t)))
        out.append(shift(colour_mul_dag(u_mu, psi), mu, -1, antiperiodic_t))
    return out


def transports_adjoint(u, g, antiperiodic_t=True):
    """[T_0^dagger g, T_{0+}^dagger g, ...]; T_{mu+}^dagger = T_{mu-} and vice versa."""
    t = transports(u, g, antiperiodic_t)
    out = [t[0]]
    for mu in range(4):
        out.append(t[2 + 2 * mu])
        out.append(t[1 + 2 * mu])
    return out


def layer_forward(u, w, psi, antiperiodic_t=True):
    ts = transports(u, psi, antiperiodic_t)
    return sum(spin_mul(w[k], ts[k]) for k in range(NK))


def forward(u, weights, psi, antiperiodic_t=True):
    """Returns the list of activations [psi_0, psi_1, ..., psi_L]."""
    acts = [psi]
    for w in weights:
        acts.append(layer_forward(u, w, acts[-1], antiperiodic_t))
    return acts


def backward(u, weights, acts, g_out, antiperiodic_t=True):
    """Given g_out = dL/d conj(psi_L), return (dL/d conj(W) per layer, dL/d conj(psi_0))."""
    grads = np.zeros_like(weights)
    g = g_out
    for l in range(len(weights) - 1, -1, -1):
        ts = transports(u, acts[l], antiperiodic_t)
        for k in range(NK):
            grads[l, k] = np.einsum("nsa,nta->st", g.reshape(-1, 4, 3),
                                         ts[k].conj().reshape(-1, 4, 3))
        wg = [spin_mul(weights[l, k].conj().T, g) for k in range(NK)]
        adj = [transports_adjoint(u, wg[k], antiperiodic_t)[k] for k in range(NK)]
        g = sum(adj)
    return grads, g


def neumann_weights(kappa, nlayers=4):
    w = np.zeros((nlayers, NK, 4, 4), dtype=np.complex128)
    for l in range(nlayers):
        om = np.exp(2j * np.pi * (l + 1) / (nlayers + 1))
        w[l, 0] = ONE4
        for mu in range(4):
            w[l, 1 + 2 * mu] = -(kappa / om) * (ONE4 - GAMMA[mu])
            w[l, 2 + 2 * mu] = -(kappa / om) * (ONE4 + GAMMA[mu])
    return w


def apply_even(u, weights, x_e, dims, antiperiodic_t=True):
    """N_e x_e = P_e N E_e x_e on half-lattice (V/2, 4, 3) fields."""
    full = _eo.join(x_e, None, dims)
    y = forward(u, weights, full, antiperiodic_t)[-1]
    return _eo.split(y, dims)[_eo.EVEN]


def loss_and_grad(u, weights, sources_e, targets_e, dims, antiperiodic_t=True):
    """L = mean_i ||N_e b_i - x_i||^2 / ||x_i||^2 and dL/d conj(W)."""
    n = len(sources_e)
    loss = 0.0
    grads = np.zeros_like(weights)
    for b, x in zip(sources_e, targets_e):
        full = _eo.join(b, None, dims)
        acts = forward(u, weights, full, antiperiodic_t)
        y_e = _eo.split(acts[-1], dims)[_eo.EVEN]
        xn = float(np.vdot(x, x).real)
        d = y_e - x
        loss += float(np.vdot(d, d).real) / xn / n
        g_full = _eo.join(d / (xn * n), None, dims)
        gw, _ = backward(u, weights, acts, g_full, antiperiodic_t)
        grads += gw
    return loss, grads


class Adam:
    """Adam on complex weights W, taken as the real parameters (Re W, Im W).

    step(w, g) takes the Wirtinger gradient g = dL/d conj(W); the real
    gradient is (2 Re g, 2 Im g).  Moments start at zero, the step counter at
    0; step t (1, 2, ...) divides the moments by (1 - beta1^t) and
    (1 - beta2^t)."""

    def __init__(self, shape, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros(shape + (2,))
        self.v = np.zeros(shape + (2,))
        self.t = 0

    def step(self, w, g):
        gr = np.stack([2.0 * g.real, 2.0 * g.imag], axis=-1)
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * gr
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * gr * gr
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        d = self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return w - (d[..., 0] + 1j * d[..., 1])
