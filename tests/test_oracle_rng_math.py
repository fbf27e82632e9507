"""Pins of the oracle's random numbers and IEEE-only exp/log.

* Philox4x32-10 against rocRAND's independent implementation (host build of
  its header), with the counter/key convention matched: key = 64-bit seed,
  counter words 0-1 = block index (offset / 4), words 2-3 = subsequence.
* exp(x) on [-23, 0) and ln(h) on integers against mpmath at 50 digits.
* The acceptance threshold floor(exp(x) 2^32) of the Metropolis rule
  min(1, W(E_n)/W(E_o)) (paper Sec. 2) against mpmath.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("probe") / "philox_probe")
    src = os.path.join(HERE, "rocrand_philox_probe.cpp")
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available to build the rocRAND probe")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O1", src, "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(12345)
    cases = []
    for _ in range(400):
        # rocRAND takes the block index as a 64-bit offset of 4 words per block
        block = int(rng.integers(0, 2**62, dtype=np.uint64))
        ctr = [block & 0xFFFFFFFF, block >> 32]
        sub = int(rng.integers(0, 2**32, dtype=np.uint64)) if rng.random() < 0.5 else int(
            rng.integers(0, 8))
        key = [int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        cases.append((ctr, sub, key))
    # extreme counters and keys
    cases += [([0, 0], 0, [0, 0]), ([2**32 - 1, 2**30 - 1], 1, [2**32 - 1, 2**32 - 1]),
              ([1, 0], 0, [1, 1]), ([0, 1], 2**32 - 1, [0, 2**31])]
    lines = []
    for ctr, sub, key in cases:
        seed = key[0] | (key[1] << 32)
        block = ctr[0] | (ctr[1] << 32)
        lines.append(f"{seed} {sub} {4 * block}")
    out = subprocess.run([rocrand_probe], input="\n".join(lines) + "\n", text=True,
                         capture_output=True, check=True).stdout.split("\n")
    for (ctr, sub, key), line in zip(cases, out):
        want = [int(v) for v in line.split()]
        got = O.philox([ctr[0], ctr[1], sub & 0xFFFFFFFF, sub >> 32], key)
        assert list(got) == want, (ctr, sub, key)


def test_philox_output_is_uniform():
    # 2^16 blocks of one stream: byte frequencies pass a chi-square test.
    words = np.concatenate([O.philox([i, 0, 0, 0], [7, 1]) for i in range(1 << 14)])
    b = words.view(np.uint8)
    counts = np.bincount(b, minlength=256)
    exp = b.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 400  # 255 dof, p ~ 1e-7


mp = pytest.importorskip("mpmath")
mp.mp.dps = 50


def _ulp_err(got, exact):
    return abs(mp.mpf(got) - exact) / mp.mpf(np.spacing(abs(float(exact))))


def test_exp_within_two_ulp():
    rng = np.random.default_rng(1)
    xs = list(-23.0 * rng.random(20000)) + [-23.0, -1e-300, -5e-324, -0.5, -np.log(2),
                                             -1e-17, -22.999999]
    worst = 0
    for x in xs:
        e = _ulp_err(O.exp(x), mp.exp(mp.mpf(float(x))))
        worst = max(worst, e)
    assert worst <= 2.0, worst


def test_log_within_two_ulp():
    rng = np.random.default_rng(2)
    hs = list(rng.integers(1, 2**31, size=20000)) + list(range(1, 2000)) + [2**31 - 1, 2**30,
                                                                            3, 46341]
    worst = 0
    for h in hs:
        h = int(h)
        got = O.log(h)
        if h == 1:
            assert got == 0.0
            continue
        worst = max(worst, _ulp_err(got, mp.log(h)))
    assert worst <= 2.0, worst


def test_accept_threshold_boundaries():
    # accept iff u < floor(exp(x) 2^32): check the two integers around the
    # threshold computed at 50 digits, away from rounding ties.
    rng = np.random.default_rng(3)
    checked = 0
    for x in -23.0 * rng.random(4000):
        t = mp.exp(mp.mpf(float(x))) * 2**32
        v = int(mp.floor(t))
        if t - v < 1e-6 or v + 1 - t < 1e-6 or v >= 2**32 - 1:
            continue
        assert O.accept(x, v - 1) if v >= 1 else True
        assert not O.accept(x, v)
        assert not O.accept(x, 2**32 - 1)
        checked += 1
    assert checked > 3000


def test_accept_special_cases():
    for u in (0, 1, 2**31, 2**32 - 1):
        assert O.accept(0.0, u)
        assert O.accept(3.5, u)
        assert not O.accept(-23.5, u)
        assert not O.accept(-1e6, u)
    # exp(-1e-18) rounds to 1: always accepted, also for the largest u
    assert O.accept(-1e-18, 2**32 - 1)
    # x = -ln 2: P(accept) = 1/2 exactly
    x = float(-mp.log(2))
    t = mp.exp(mp.mpf(x)) * 2**32
    v = int(mp.floor(t))
    assert O.accept(x, v - 1) and not O.accept(x, v)
