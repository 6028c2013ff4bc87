"""GPU parity of the learned preconditioner (forward, adjoint, loss and
weight gradients, Adam) against the FP64 oracle of the net, and the
flexible solvers that use it, checked by the oracle's residual of the full
system.

The net computes in FP32 (weights, activations) with FP64 gradient sums;
the tolerances below are FP32 rounding of four layers of nine terms each.
Trained weights are not unique, so training is checked through its loss
curve and through what the trained net gains in the solver, not weight by
weight.
"""
import numpy as np
import pytest

from gen import fields
from oracle import dirac, evenodd
from oracle import net as onet
from tests.gpu_common import case, log_errors, rel, say

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.135, 1.0


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def random_weights(nl, seed, scale=0.25):
    r = fields.rng(seed)
    w = (r.standard_normal((nl, onet.NK, 4, 4)) + 1j * r.standard_normal((nl, onet.NK, 4, 4)))
    return scale * w


def even_fields(dims, n, seed):
    full = fields.gaussian_spinor(dims, fields.SEED_SOURCE + seed, nrhs=n)
    return np.stack([evenodd.split(full[i], dims)[0] for i in range(n)])


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 2, 2), (8, 4, 4, 8)])
@pytest.mark.parametrize("init", ["random", "neumann"])
def test_net_forward_parity(lq, dims, init):
    say(f"net forward dims={dims} init={init}")
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    w = random_weights(4, 11) if init == "random" else onet.neumann_weights(KAPPA, 4)
    net = lq.Net(lat, 4)
    net.set_weights(w)
    assert np.allclose(net.get_weights(), w.astype(np.complex64), rtol=0, atol=1e-7)
    x = even_fields(dims, 1, 3)[0]
    dx = lat.to_device(x, lq.EVEN, lq.F32)
    dy = lat.new_field(lq.EVEN, lq.F32)
    net.apply(dy, dx)
    got = lat.to_host(dy, lq.EVEN, lq.F32)
    ref = onet.apply_even(u, w, x, dims)
    err = log_errors("net FP32 forward", got, ref)
    assert err <= 2e-5, err


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 4, 8)])
@pytest.mark.parametrize("layers", [1, 2, 4])
def test_net_forward_fp16(lq, dims, layers):
    """The solvers' form of the net (FP16 links and activations with per-site
    scales, FP32 accumulation; even-only first layer, even output of the
    last layer only): FP16 rounding of links and activations, a few 1e-3."""
    say(f"net forward fp16 dims={dims} layers={layers}")
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    w = random_weights(layers, 15)
    net = lq.Net(lat, layers)
    net.set_weights(w)
    x = even_fields(dims, 1, 3)[0]
    dx = lat.to_device(x, lq.EVEN, lq.F32)
    dy = lat.new_field(lq.EVEN, lq.F32)
    for adj in (False, True):
        net.apply(dy, dx, adjoint=adj, fp16=True)
        got = lat.to_host(dy, lq.EVEN, lq.F32)
        if not adj:
            ref = onet.apply_even(u, w, x, dims)
        else:
            acts = onet.forward(u, w, evenodd.join(x, None, dims))
            ref = evenodd.split(onet.backward(u, w, acts, evenodd.join(x, None, dims))[1],
                                dims)[0]
        err = log_errors(f"net FP16 adjoint {int(adj)}", got, ref)
        assert err <= 5e-3, (adj, err)


def test_init_neumann_matches_oracle(lq):
    """The library's Neumann start (its own gamma matrices) equals the
    oracle's, FP32-rounded."""
    dims = (4, 4, 4, 4)
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    for nl in (1, 4, 5):
        net = lq.Net(lat, nl)
        net.init_neumann(KAPPA)
        ref = onet.neumann_weights(KAPPA, nl)
        assert np.max(np.abs(net.get_weights() - ref)) <= 1e-7, nl


def test_neumann_net_is_hopping_series(lq):
    """Neumann weights: the GPU net equals sum_{n<=4} (kappa H)^n on the
    embedded even field, with H the oracle's hopping term."""
    dims = (6, 4, 4, 6)
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    net = lq.Net(lat, 4)
    net.set_weights(onet.neumann_weights(KAPPA, 4))
    x = even_fields(dims, 1, 4)[0]
    dy = lat.new_field(lq.EVEN, lq.F32)
    net.apply(dy, lat.to_device(x, lq.EVEN, lq.F32))
    full = evenodd.join(x, None, dims)
    acc, term = full.copy(), full.copy()
    for _ in range(4):
        term = KAPPA * dirac.hop(u, term)
        acc = acc + term
    ref = evenodd.split(acc, dims)[0]
    assert rel(lat.to_host(dy, lq.EVEN, lq.F32), ref) <= 2e-5


def test_net_adjoint(lq):
    dims = (4, 4, 4, 4)
    u, _, _, _ = case(dims, "haar", 2)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    w = random_weights(3, 12)
    net = lq.Net(lat, 3)
    net.set_weights(w)
    a, b = even_fields(dims, 2, 5)
    da, db = lat.to_device(a, lq.EVEN, lq.F32), lat.to_device(b, lq.EVEN, lq.F32)
    na, ntb = lat.new_field(lq.EVEN, lq.F32), lat.new_field(lq.EVEN, lq.F32)
    net.apply(na, da)
    net.apply(ntb, db, adjoint=True)
    lhs = lat.dot(db, na, lq.EVEN, lq.F32)      # <b, N a>
    rhs = lat.dot(ntb, da, lq.EVEN, lq.F32)     # <N^+ b, a>
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    # against the oracle's backward pass (N^+ applied to the embedded field)
    full = evenodd.join(b, None, dims)
    acts = onet.forward(u, w, evenodd.join(a, None, dims))
    _, gin = onet.backward(u, w, acts, full)
    ref = evenodd.split(gin, dims)[0]
    assert rel(lat.to_host(ntb, lq.EVEN, lq.F32), ref) <= 2e-5


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 2, 4)])
def test_net_loss_grad_parity(lq, dims):
    say(f"net loss/grad dims={dims}")
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    w = random_weights(4, 13, scale=0.2)
    net = lq.Net(lat, 4)
    net.set_weights(w)
    b = even_fields(dims, 3, 6)
    x = even_fields(dims, 3, 7)
    db, dx = lat.to_device(b, lq.EVEN, lq.F32), lat.to_device(x, lq.EVEN, lq.F32)
    loss, grad = net.loss_grad(db, dx, 3)
    # the oracle on the inputs the GPU saw (FP32-rounded sources, targets, weights)
    w32 = w.astype(np.complex64).astype(np.complex128)
    b32 = b.astype(np.complex64).astype(np.complex128)
    x32 = x.astype(np.complex64).astype(np.complex128)
    rloss, rgrad = onet.loss_and_grad(u, w32, list(b32), list(x32), dims)
    assert abs(loss - rloss) <= 1e-5 * rloss, (loss, rloss)
    assert rel(grad, rgrad) <= 1e-4, rel(grad, rgrad)


def test_adam_step(lq):
    """Three consecutive GPU Adam steps (moments accumulated, bias factors at
    t = 1, 2, 3) against the oracle's Adam fed the same gradients."""
    dims = (4, 4, 4, 4)
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    w = random_weights(2, 14, scale=0.2)
    net = lq.Net(lat, 2)
    net.set_weights(w)
    b, x = even_fields(dims, 2, 8), even_fields(dims, 2, 9)
    db, dx = lat.to_device(b, lq.EVEN, lq.F32), lat.to_device(x, lq.EVEN, lq.F32)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    opt = onet.Adam(w.shape, lr=lr, beta1=b1, beta2=b2, eps=eps)
    ref = net.get_weights()
    for t in range(3):
        # alternate the pair so that the gradients differ from step to step
        _, g = net.loss_grad(db, dx, 2) if t % 2 == 0 else net.loss_grad(db, dx, 1)
        ref = opt.step(ref, g)
        net.adam_step(lr, b1, b2, eps)
        got = net.get_weights()
        assert np.max(np.abs(got - ref)) <= 2e-6, t
        ref = got  # continue from the FP32 weights the GPU holds


def oracle_residual(u, kappa, csw, x, b):
    wc = evenodd.WilsonClover(u, kappa, csw)
    return dirac.norm(b - wc.M(x.reshape(b.shape))) / dirac.norm(b)


@pytest.mark.parametrize("solver", ["fgmres", "fcg"])
def test_net_solvers(lq, solver):
    dims, tol = (8, 8, 8, 8), 1e-10
    say(f"net solver {solver} dims={dims}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 21)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    net = lq.Net(lat, 4)
    net.set_weights(onet.neumann_weights(KAPPA, 4))
    kind = lq.FGMRES_NET if solver == "fgmres" else lq.FCG_NET
    x, rep = net.solve(b, KAPPA, CSW, tol, solver=kind)
    res = oracle_residual(u, KAPPA, CSW, x, b)
    say(f"  iterations={rep[0].iterations} restarts={rep[0].reliable_updates} "
        f"fallback={rep[0].fallback} dslash={rep[0].dslash_calls} res={res:.2e}")
    assert res <= tol, res
    assert rep[0].fallback == 0
    assert abs(rep[0].true_residual - res) <= 0.1 * res + 1e-14


def test_net_solver_falls_back(lq):
    """A net that maps everything to zero breaks FGMRES down at once; the
    plain mixed CG then finishes the solve."""
    dims, tol = (4, 4, 4, 4), 1e-10
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 22)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    net = lq.Net(lat, 2)  # zero weights
    x, rep = net.solve(b, KAPPA, CSW, tol, solver=lq.FGMRES_NET)
    assert rep[0].fallback == 1
    assert oracle_residual(u, KAPPA, CSW, x, b) <= tol


def make_pairs(lq, lat, u, dims, n, seed):
    """Training pairs (b_e, x_e = Mhat^-1 b_e): solve M x = (b_e, 0) with the
    library's FP64 solver and keep the even half of x."""
    bs = even_fields(dims, n, seed)
    xs = []
    for i in range(n):
        full = evenodd.join(bs[i], None, dims)
        x, _ = lat.solve(full, KAPPA, CSW, 1e-10, inner_prec=lq.F64)
        xs.append(evenodd.split(x, dims)[0])
    return bs, np.stack(xs)


def test_training_gain(lq):
    """Train from the Neumann initialisation on pairs the solver generated,
    keeping after every epoch the weights that need the fewest flexible-CG
    iterations on a held-out source (the Neumann start counts as epoch 0;
    the benchmark's rule).  The loss falls; on a fresh source the kept net
    needs far fewer iterations than no net (identity weights) and strictly
    fewer than its Neumann start (on this 8^4 system the first epochs of
    training help; longer training raises the count again while the loss
    keeps falling, which is what the selection guards against)."""
    dims = (8, 8, 8, 8)
    u = fields.gauge_field(dims, "smooth", fields.SEED_TRAIN_FIELD)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    say("training pairs")
    bs, xs = make_pairs(lq, lat, u, dims, 32, 40)
    db, dx = lat.to_device(bs, lq.EVEN, lq.F32), lat.to_device(xs, lq.EVEN, lq.F32)
    held = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 42)
    fresh = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 41)
    probe = lq.Net(lat, 4)

    def iterations(w, b):
        probe.set_weights(w)
        x, rep = probe.solve(b, KAPPA, CSW, 1e-10, solver=lq.FCG_NET)
        assert oracle_residual(u, KAPPA, CSW, x, b) <= 1e-10
        assert rep[0].fallback == 0
        return rep[0].iterations

    net = lq.Net(lat, 4)
    w0 = onet.neumann_weights(KAPPA, 4)
    net.set_weights(w0)
    l0, _ = net.loss_grad(db, dx, 32)
    kept, kept_its = w0, iterations(w0, held)
    per_epoch = [kept_its]
    for e in range(6):
        net.train(db, dx, 32, epochs=5, batch=4, lr=2e-3, seed=1 if e == 0 else 0)
        w = net.get_weights()
        its = iterations(w, held)
        per_epoch.append(its)
        if its < kept_its:
            kept, kept_its = w, its
    l1, _ = net.loss_grad(db, dx, 32)
    say(f"  loss {l0:.4f} -> {l1:.4f}; held-out iterations per 5 epochs {per_epoch}")
    assert l1 < 0.8 * l0
    assert kept_its <= per_epoch[0]
    identity = np.concatenate([np.eye(4)[None, None].repeat(4, 0), np.zeros((4, 8, 4, 4))], axis=1)
    its = {"kept": iterations(kept, fresh), "neumann": iterations(w0, fresh),
           "identity": iterations(identity, fresh)}
    say(f"  fresh-source flexible-CG iterations {its}")
    assert its["kept"] * 1.5 < its["identity"]
    assert kept is not w0
    assert its["kept"] < its["neumann"]


@pytest.mark.parametrize("m,k", [(16, 4), (24, 8)])
def test_net_fgmres_dr(lq, m, k):
    """FGMRES with deflated restarts and the net (Neumann start) on the
    right: the solution meets the tolerance by the oracle's residual without
    falling back."""
    dims, tol = (8, 8, 8, 8), 1e-10
    say(f"net FGMRES-DR m={m} k={k}")
    u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 1)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 23)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    net = lq.Net(lat, 4)
    net.set_weights(onet.neumann_weights(KAPPA, 4))
    x, rep = net.solve(b, KAPPA, CSW, tol, solver=lq.FGMRES_NET, restart=m, deflate=k)
    res = oracle_residual(u, KAPPA, CSW, x, b)
    say(f"  iterations={rep[0].iterations} restarts={rep[0].reliable_updates} "
        f"fallback={rep[0].fallback} res={res:.2e}")
    assert res <= tol
    assert rep[0].fallback == 0


def test_checkpoint_resume_matches_uninterrupted_training(lq, tmp_path):
    """Four epochs in one go against two epochs, a checkpoint, a fresh net
    loaded from it, and two more epochs continuing the shuffle generator:
    the weights agree bit for bit, and so does the loss history."""
    dims = (4, 4, 4, 4)
    u, _, _, _ = case(dims, "smooth", 1)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    b, x = even_fields(dims, 6, 30), even_fields(dims, 6, 31)
    db, dx = lat.to_device(b, lq.EVEN, lq.F32), lat.to_device(x, lq.EVEN, lq.F32)
    w0 = onet.neumann_weights(KAPPA, 3)
    full = lq.Net(lat, 3)
    full.set_weights(w0)
    h_full = full.train(db, dx, 6, epochs=4, batch=2, lr=5e-3, seed=5)
    part = lq.Net(lat, 3)
    part.set_weights(w0)
    h1 = part.train(db, dx, 6, epochs=2, batch=2, lr=5e-3, seed=5)
    path = tmp_path / "net.ckpt"
    part.save(path)
    head = open(path, "rb").readline().decode()
    assert '"format": "lq-net-checkpoint"' in head and '"layers": 3' in head
    resumed = lq.Net(lat, 3)
    resumed.load(path)
    h2 = resumed.train(db, dx, 6, epochs=2, batch=2, lr=5e-3, seed=0)
    assert np.array_equal(resumed.get_weights(), full.get_weights())
    assert np.array_equal(np.concatenate([h1, h2]), h_full)
    # a net of another depth, and a damaged file, are refused
    with pytest.raises(lq.LQError):
        lq.Net(lat, 2).load(path)
    data = open(path, "rb").read()
    bad = tmp_path / "bad.ckpt"
    open(bad, "wb").write(data[: len(data) // 2])
    with pytest.raises(lq.LQError):
        lq.Net(lat, 3).load(bad)
