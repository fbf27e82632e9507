"""Host logic of the run driver (paper_1401_4076_amd/run.py): group specs,
per-group metrics of a histogram, checkpoint files and their checks."""
import json

import numpy as np
import pytest

from paper_1401_4076_amd import run as R


def test_parse_groups():
    assert R.parse_groups("3:48:3318:16384") == [(3, 48, 3318, 16384)]
    assert R.parse_groups("2:8:16:64,3:6:11:8") == [(2, 8, 16, 64), (3, 6, 11, 8)]
    with pytest.raises(ValueError):
        R.parse_groups("2:8:16")


def test_group_metrics():
    h = np.array([0, 4, 0, 8, 2, 0], dtype=np.int32)  # bins E = -10 ... -5
    m = R.group_metrics(h, -10)
    assert m == {"visited": 0.5, "lowest_e": -9, "highest_e": -6, "bottom": False,
                 "top": False, "min_over_max": 0.25}
    m = R.group_metrics(np.array([1, 0, 3], dtype=np.int32), -2)
    assert (m["bottom"], m["top"], m["lowest_e"], m["highest_e"]) == (True, True, -2, 0)
    m = R.group_metrics(np.zeros(4, dtype=np.int32), -3)
    assert m["visited"] == 0.0 and m["lowest_e"] is None


def test_checkpoint_file_round_trip(tmp_path):
    path = str(tmp_path / "ck.npz")
    image = bytes(range(256)) * 3
    lnW, P = np.linspace(-3, 0, 7), np.arange(7, dtype=np.float64)
    H = np.arange(7, dtype=np.int32)
    meta = {"version": R.CHECKPOINT_VERSION, "groups": [[2, 8, 16, 64]], "seed": 1,
            "sweeps": 10, "rule": "berg", "stop": "flat", "tunnel_target": 30,
            "iterations": 3, "iters": [3], "flat": [0], "stopped": False}
    R.save_checkpoint(path, image, lnW, P, H, meta)
    img, l2, p2, h2, m2 = R.load_checkpoint(path)
    assert img == image and m2 == meta
    assert np.array_equal(l2.view(np.int64), lnW.view(np.int64))
    assert np.array_equal(p2, P) and np.array_equal(h2, H) and h2.dtype == np.int32
    with np.load(path, allow_pickle=False) as z:  # nothing in it needs unpickling
        assert sorted(z.files) == ["H", "P", "image", "lnW", "meta"]
    R.check_meta(m2, dict(meta, iterations=9))  # progress keys are not compared
    for k, v in (("seed", 2), ("sweeps", 11), ("groups", [[2, 8, 16, 32]]), ("stop", "none"),
                 ("rule", "simple"), ("tunnel_target", 3)):
        with pytest.raises(ValueError, match=k):
            R.check_meta(m2, dict(meta, **{k: v}))
    R.save_checkpoint(path, image, lnW, P, H, dict(meta, version=99))
    with pytest.raises(ValueError, match="version"):
        R.load_checkpoint(path)


def test_run_config_from_workload_and_groups():
    ap = R.build_parser()
    cfg = R.run_config(ap.parse_args(["--workload", "plain_2d", "--walkers", "16",
                                      "--sweeps", "50"]))
    assert cfg["groups"] == [[2, 8, 16, 16]] and cfg["sweeps"] == 50 and cfg["seed"] == 1
    cfg = R.run_config(ap.parse_args(["--groups", "3:6:11:40,2:8:16:8", "--walkers", "20",
                                      "--seed", "5", "--stop", "tunnel"]))
    assert cfg["groups"] == [[3, 6, 11, 20], [2, 8, 16, 8]] and cfg["seed"] == 5
    assert cfg["workload"] is None and cfg["stop"] == "tunnel"
    json.dumps(cfg)


def test_bad_arguments_exit_before_any_device_work():
    for argv in (["--resume"], ["--max-iters", "0"], ["--checkpoint-every", "-1"]):
        with pytest.raises(SystemExit) as e:
            R.main(argv)
        assert e.value.code == 2
