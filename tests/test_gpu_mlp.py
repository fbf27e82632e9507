"""GPU tests of the learned-initial-weights network through the C ABI:
forward pass and gradients against the bfloat16-emulating numpy reference,
the Adam update, training, the feature/target rows of converged tables, the
proposal of initial weights, and the gain over flat initial weights."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_ref as R

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")
L = pytest.importorskip("paper_1401_4076_amd.learned")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(a, dt=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def blocks(v):
    return [b.ravel() for b in R.unpack(v)]


@pytest.fixture
def net():
    n = M.Mlp(4096)
    yield n
    n.close()


def test_forward_matches_bf16_reference(net):
    p = W.mlp_init_params(11)
    X, _ = W.mlp_synthetic_rows(1000, 12)
    net.set_params(p)
    Y = torch.zeros(len(X), device="cuda")
    net.forward(dev(X), Y)
    y_ref, _ = R.forward(p.astype(np.float64), X, "bf16")
    y = Y.cpu().numpy()
    scale = np.abs(y_ref).max()
    assert np.abs(y - y_ref).max() <= 1e-2 * scale, np.abs(y - y_ref).max()
    assert np.array_equal(net.get_params(), p)


@pytest.mark.parametrize("rows", [1, 17, 700])
def test_gradient_matches_bf16_reference(net, rows):
    p = W.mlp_init_params(13)
    X, T = W.mlp_synthetic_rows(rows, 14)
    net.set_params(p)
    g = torch.zeros(net.nparams, device="cuda")
    loss = torch.zeros(1, device="cuda")
    net.gradient(dev(X), dev(T), g, loss)
    l_ref, g_ref = R.loss_and_grad(p.astype(np.float64), X, T, "bf16")
    assert abs(loss.item() - l_ref) <= 1e-3 * max(1.0, l_ref)
    gg = g.cpu().numpy().astype(np.float64)
    for a, b in zip(blocks(gg), blocks(g_ref)):
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-7
    assert np.dot(gg, g_ref) / np.linalg.norm(gg) / np.linalg.norm(g_ref) > 0.9995
    assert np.array_equal(net.get_params(), p)  # gradient leaves parameters unchanged


def test_adam_step_applies_the_update(net):
    p = W.mlp_init_params(15)
    X, T = W.mlp_synthetic_rows(300, 16)
    net.set_params(p)
    g = torch.zeros(net.nparams, device="cuda")
    net.gradient(dev(X), dev(T), g)
    lr = 1e-3
    net.train_step(dev(X), dev(T), lr)
    got = net.get_params().astype(np.float64)
    want, _, _ = R.adam_step(p.astype(np.float64), g.cpu().numpy().astype(np.float64),
                             np.zeros(p.size), np.zeros(p.size), 1, lr)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-7)


def test_training_reduces_the_loss(net):
    X, T = W.mlp_synthetic_rows(2000, 17)
    net.set_params(W.mlp_init_params(18))
    hist = L.train(net, dev(X), dev(T), 800, lr=3e-3, lr_end=3e-4, log_every=100)
    say("loss history", hist)
    assert hist[-1][1] < 0.05 * hist[0][1]
    Y = torch.zeros(len(X), device="cuda")
    net.forward(dev(X), Y)
    resid = Y.cpu().numpy() - T
    assert abs(np.mean(resid * resid) - hist[-1][1]) < 0.5 * hist[-1][1] + 1e-4


def test_table_rows_and_proposed_weights(net):
    groups = [(2, 8, 16, 2), (3, 6, 11, 2), (2, 12, 20, 3, -30, 0)]
    ctx = M.Context(groups, 1)
    lnW = W.random_lnW(ctx.total_bins, seed=3, scale=1.0)
    glnW = dev(lnW, torch.float64)
    net.set_params(W.mlp_init_params(19))
    for g, (d, Lg, N, *_rest) in enumerate(groups):
        lo, hi, off = ctx.window(g)
        nb = hi - lo + 1
        X = torch.zeros((nb, 4), device="cuda")
        T = torch.zeros(nb, device="cuda")
        M.mucaMlpTableRows(ctx, g, glnW, X, T)
        E = np.arange(lo, hi + 1)
        want = np.stack([np.full(nb, (d - 2.5) * 2), np.full(nb, Lg / 64),
                         np.full(nb, 10 * N / Lg ** d), E / lo], axis=1).astype(np.float32)
        np.testing.assert_allclose(X.cpu().numpy(), want, rtol=1e-6)
        np.testing.assert_allclose(T.cpu().numpy(), (lnW[off:off + nb] - lnW[off]) / N,
                                   rtol=1e-6, atol=1e-6)
        # proposal: lnW = N y shifted so that lnW(e_hi) = 0
        Y = torch.zeros(nb, device="cuda")
        net.forward(X, Y)
        out = torch.zeros(ctx.total_bins, dtype=torch.float64, device="cuda")
        net.predict_weights(ctx, g, out)
        y = Y.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(out.cpu().numpy()[off:off + nb], N * y - N * y[-1],
                                   rtol=1e-6, atol=1e-6)


# Training lattices (converged by the iteration itself) and a held-out one.
TRAIN = [(2, L_, W.particles(2, L_, r), 128) for L_ in (8, 12, 16, 20) for r in (0.1, 0.2)] + \
        [(3, L_, W.particles(3, L_, r), 128) for L_ in (6, 8) for r in (0.05, 0.1)]
HELD_OUT = [(2, 14, W.particles(2, 14, 0.15), 128), (2, 18, W.particles(2, 18, 0.12), 128),
            (3, 7, W.particles(3, 7, 0.08), 128)]


def test_learned_initial_weights_reach_flatness_sooner(net):
    tables = L.converge(TRAIN, seed=1, sweeps=100, max_iters=300)
    say("training tables: iterations", tables["iters"], "flat", tables["flat"])
    done = [g for g, f in enumerate(tables["flat"]) if f]
    assert len(done) >= 0.8 * len(TRAIN)
    X, T = L.table_rows(tables["ctx"], tables["lnW"], done)  # converged tables only
    net.set_params(W.mlp_init_params(20))
    hist = L.train(net, X, T, 3000, log_every=500)
    say("training loss", hist)
    res = L.compare(net, HELD_OUT, seed=2, sweeps=100, max_iters=300, prod_sweeps=3000)
    say("held-out comparison", res)
    assert all(res["plain"]["flat"]) and all(res["learned"]["flat"])
    # fewer iterations to a flat histogram in total, and on the largest lattice
    assert sum(res["learned"]["iters"]) < sum(res["plain"]["iters"])
    assert res["learned"]["iters"][1] < res["plain"]["iters"][1]
    # both arms estimate the same density of states (production-run statistics)
    assert max(res["ln_omega_max_abs_diff"]) < 0.5
