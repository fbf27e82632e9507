"""Checkpoint and resume through the C ABI (mucaStateBytes, mucaSaveState,
mucaLoadState): a run split by a saved and reloaded state image, in a
second context, continues bit for bit as the uninterrupted run and as one
oracle run of the same total length; malformed or foreign images are
refused and leave the context unchanged."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"
# small groups that flatten and tunnel within a few iterations, and one 3D
# group of L = 32 whose walker state keeps the bricked bit layout
GROUPS = [(2, 4, 5, 64, -5, 0), (2, 6, 10, 16, 0, 0), (3, 4, 4, 16, -4, 0),
          (3, 32, 983, 4, 0, 0)]


def say(*a):
    print(*a, flush=True)


def same_f64(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return np.array_equal(a.view(np.int64), b.view(np.int64))


def zeros(ctx, dtype):
    return torch.zeros(ctx.total_bins, dtype=dtype, device=DEV)


def walkers_equal(a, b):
    for w in range(a.nwalkers):
        assert a.read_walker(w) == b.read_walker(w), w
    assert a.tunnel() == b.tunnel()


@pytest.mark.parametrize("stop", [M.MUCA_STOP_FLAT, M.MUCA_STOP_TUNNEL], ids=["flat", "tunnel"])
def test_reloaded_state_resumes_the_run(stop):
    seed, S, K1, K2 = 21, 20, 2, 6
    say("checkpoint run", GROUPS, "stop", stop, "sweeps", S, "iterations", K1, "+", K2)
    a = M.Context(GROUPS, seed)
    a.set_tunnel_target(3)
    lnW, P, H = zeros(a, torch.float64), zeros(a, torch.float64), zeros(a, torch.int32)
    a.run(lnW, P, H, S, K1, stop=stop)
    image = a.save_state()
    assert len(image) == a.state_bytes()
    lnW1, P1, H1 = lnW.clone(), P.clone(), H.clone()  # caller-owned, not in the image
    rcA, itA, flA = a.run(lnW, P, H, S, K2, stop=stop, resume=True)

    b = M.Context(GROUPS, seed)  # default tunnelling target: the image sets 3
    b.load_state(image)
    assert bytes(b.save_state()) == bytes(image)
    lnWb, Pb, Hb = lnW1, P1, H1  # a stopped group's histogram stays as it was
    rcB, itB, flB = b.run(lnWb, Pb, Hb, S, K2, stop=stop, resume=True)
    assert (rcA, itA, flA) == (rcB, itB, flB)
    assert torch.equal(H, Hb)
    assert same_f64(lnW.cpu().numpy(), lnWb.cpu().numpy())
    assert same_f64(P.cpu().numpy(), Pb.cpu().numpy())
    walkers_equal(a, b)

    # one oracle run of K1 + K2 iterations
    ref = O.RefContext(GROUPS, seed)
    rlnW, rP = np.zeros(ref.total_bins), np.zeros(ref.total_bins)
    rrc, rH, rit, rfl = ref.run(rlnW, rP, S, K1 + K2, 0, stop == M.MUCA_STOP_FLAT,
                                tunnel_target=3 if stop == M.MUCA_STOP_TUNNEL else None)
    assert rcB == rrc and list(itB) == list(rit) and list(flB) == list(rfl)
    assert np.array_equal(Hb.cpu().numpy(), rH)
    assert same_f64(lnWb.cpu().numpy(), rlnW) and same_f64(Pb.cpu().numpy(), rP)
    last, trips = b.tunnel()
    rlast, rtrips = ref.tunnel()
    assert np.array_equal(np.array(last, dtype=np.uint32), rlast)
    assert np.array_equal(np.array(trips, dtype=np.uint32), rtrips)
    for w in (0, 70, b.nwalkers - 1):
        bits, pos, E, t = b.read_walker(w)
        _, rpos, rE, rt = ref.walker(w)
        assert (E, t) == (rE, rt) and np.array_equal(np.array(pos, dtype=np.uint32), rpos), w


def test_reloaded_state_resumes_sweeps():
    """Without a run: sweeps after a reload equal sweeps after the save, and
    a resumed run is refused (no run was started before the save)."""
    seed = 8
    a = M.Context(GROUPS, seed)
    lnW = torch.tensor(W.random_lnW(a.total_bins, seed=9, scale=0.8), device=DEV)
    H = zeros(a, torch.int32)
    a.sweep(lnW, 3, H)
    image = a.save_state()
    a.sweep(lnW, 5, H)
    b = M.Context(GROUPS, seed)
    b.load_state(image)
    Hb = zeros(b, torch.int32)
    b.sweep(lnW, 5, Hb)
    torch.cuda.synchronize()
    assert torch.equal(H, Hb)
    walkers_equal(a, b)
    P = zeros(b, torch.float64)
    with pytest.raises(M.MucaError) as e:
        b.run(lnW.clone(), P, Hb, 1, 1, resume=True)
    assert e.value.code == M.MUCA_EINVAL


def test_foreign_and_damaged_images_are_refused():
    seed = 4
    a = M.Context(GROUPS, seed)
    H = zeros(a, torch.int32)
    a.sweep(zeros(a, torch.float64), 2, H)
    image = bytes(a.save_state())
    b = M.Context(GROUPS, seed)
    before = bytes(b.save_state())

    def refused(ctx, img):
        with pytest.raises(M.MucaError) as e:
            ctx.load_state(img)
        assert e.value.code == M.MUCA_EINVAL

    flipped = bytearray(image)
    flipped[len(image) // 2] ^= 1  # inside the walker state: checksum
    magic = bytearray(image)
    magic[0] ^= 1
    for img in (image[:-1], image[:40], bytes(flipped), bytes(magic)):
        refused(b, img)
    refused(M.Context(GROUPS, seed + 1), image)
    refused(M.Context(GROUPS, seed, first_id=5), image)
    refused(M.Context(GROUPS[:3], seed), image)
    refused(M.Context(GROUPS[:3] + [(3, 32, 983, 5, 0, 0)], seed), image)
    assert bytes(b.save_state()) == before

    n = a.state_bytes()
    small = (ctypes.c_char * n)()
    assert M.lib().mucaSaveState(a.handle, small, n - 1) == M.MUCA_EINVAL
    assert M.lib().mucaSaveState(a.handle, None, n) == M.MUCA_EINVAL
    assert M.lib().mucaLoadState(a.handle, None, n) == M.MUCA_EINVAL
