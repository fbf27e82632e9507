"""GPU tests of the learned-initial-weights network through the C ABI:
forward pass and gradients against the bfloat16-emulating numpy reference,
entry by entry within the tolerances derived in tests/mlp_envelope.py; the
Adam update, training, the feature/target rows of converged tables, the
proposal of initial weights, and the gain over flat initial weights."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import mlp_ref as R

import mlp_envelope as E

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")
L = pytest.importorskip("paper_1401_4076_amd.learned")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(a, dt=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


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
    y = Y.cpu().numpy().astype(np.float64)
    tol = E.output_tolerance(p, X, np.zeros(len(X)), y_ref)
    assert np.all(np.abs(y - y_ref) <= tol), np.max(np.abs(y - y_ref) / tol)
    assert np.array_equal(net.get_params(), p)


def check_gradient(net, p, X, T):
    """GPU loss and gradient vs the reference, every entry within the
    tolerance of tests/mlp_envelope.py."""
    net.set_params(p)
    g = torch.zeros(net.nparams, device="cuda")
    loss = torch.zeros(1, device="cuda")
    net.gradient(dev(X), dev(T), g, loss)
    l_ref, g_ref = R.loss_and_grad(p.astype(np.float64), X, T, "bf16")
    assert abs(loss.item() - l_ref) <= 1e-3 * max(1.0, l_ref)
    gg = g.cpu().numpy().astype(np.float64)
    tol = E.grad_tolerance(p, X, T, g_ref)
    bad = np.abs(gg - g_ref) > tol
    worst = np.argmax(np.abs(gg - g_ref) / tol)
    assert not bad.any(), (int(bad.sum()), int(worst), gg[worst], g_ref[worst], tol[worst])
    say(f"gradient rows={len(X)}: max |g - g_ref| / tol = "
        f"{np.max(np.abs(gg - g_ref) / tol):.3g}, entries with |g_ref| > 2 tol: "
        f"{np.mean(np.abs(g_ref) > 2 * tol):.4f}")
    assert np.array_equal(net.get_params(), p)  # gradient leaves parameters unchanged


@pytest.mark.parametrize("rows", [1, 17, 700])
def test_gradient_matches_bf16_reference(net, rows):
    p = W.mlp_init_params(13)
    X, T = W.mlp_synthetic_rows(rows, 14)
    check_gradient(net, p, X, T)


def ref_table_rows(d, L, N, lo, lnW_group):
    """Features and targets of a converged table, computed on the host from
    the oracle's weights with the definitions of mucaMlpTableRows."""
    f = np.float32
    E_ = np.arange(lo, 0 + 1)
    nb = len(E_)
    X = np.stack([np.full(nb, (f(d) - f(2.5)) * f(2.0), dtype=f),
                  np.full(nb, f(L) / f(64.0), dtype=f),
                  np.full(nb, f(10.0) * f(N) / f(L ** d), dtype=f),
                  (E_.astype(f) / f(lo)).astype(f)], axis=1)
    T = ((lnW_group - lnW_group[0]) / float(N)).astype(f)
    return X, T


def test_gradient_on_converged_table_rows(net):
    """Rows of a table the iteration converged (mucaMlpTableRows on the GPU;
    the oracle's own run, bit-identical, gives the reference rows)."""
    groups = [(2, 8, 16, 64), (3, 6, 11, 64)]
    seed, sweeps = 1, 1000
    ctx = M.Context(groups, seed)
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device="cuda")
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device="cuda")
    rc, it, fl = ctx.run(lnW, P, H, sweeps, 40, M.MUCA_RULE_BERG, True)
    ref = O.RefContext(groups, seed)
    rlnW, rP = ref.zeros_lnW(), ref.zeros_lnW()
    rrc, _, rit, rfl = ref.run(rlnW, rP, sweeps, 40, 0, True)
    say("converged tables: iterations", list(it), "flat", list(fl))
    assert all(fl) and list(it) == list(rit) and list(fl) == list(rfl)
    assert np.array_equal(lnW.cpu().numpy().view(np.int64), rlnW.view(np.int64))
    p = W.mlp_init_params(23)
    for g, (d, Lg, N, _w) in enumerate(groups):
        lo, hi, off = ctx.window(g)
        nb = hi - lo + 1
        Xg = torch.zeros((nb, 4), device="cuda")
        Tg = torch.zeros(nb, device="cuda")
        M.mucaMlpTableRows(ctx, g, lnW, Xg, Tg)
        X, T = ref_table_rows(d, Lg, N, lo, rlnW[off:off + nb])
        assert np.array_equal(Xg.cpu().numpy(), X)
        assert np.array_equal(Tg.cpu().numpy(), T)
        check_gradient(net, p, X, T)
    ctx.close()


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
