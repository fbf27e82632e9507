"""Python binding of libmuca (include/muca.h): argument marshalling only.

Every step of the MUCA iteration runs in the HIP kernels of libmuca.so;
this module passes device pointers of torch tensors and the current HIP
stream through ctypes.  PyTorch is used for device memory and streams only.
The functions keep the C names (mucaInit, mucaSweep, ...) and raise
MucaError on a negative status.  There is no fallback: if libmuca.so is not
built, loading fails with an ImportError.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that libmuca shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmuca.so")

MUCA_OK = 0
MUCA_NOT_CONVERGED = 1
MUCA_EINVAL = -1
MUCA_EOVERFLOW = -2
MUCA_ENOMEM = -3
MUCA_EHIP = -4
MUCA_ENONFINITE = -5
MUCA_RULE_BERG = 0
MUCA_RULE_SIMPLE = 1
MUCA_STOP_NONE = 0
MUCA_STOP_FLAT = 1
MUCA_STOP_TUNNEL = 2
MUCA_LAYOUT_AUTO = 0
MUCA_LAYOUT_LANE = 1
MUCA_LAYOUT_SUB16 = 2
MUCA_LAYOUT_SUB64 = 3
MUCA_LAYOUT_LOOK4 = 4
MUCA_LAYOUT_SUB16X2 = 5
MUCA_LAYOUT_SUB16X1 = 6
MUCA_LAYOUT_SUB16MIX = 7
MUCA_NUM_LAYOUTS = 8
MUCA_NOALLOC_WORKSPACE_BYTES = 4194304
LAYOUTS = (MUCA_LAYOUT_LANE, MUCA_LAYOUT_SUB16, MUCA_LAYOUT_SUB64, MUCA_LAYOUT_LOOK4,
           MUCA_LAYOUT_SUB16X2, MUCA_LAYOUT_SUB16X1, MUCA_LAYOUT_SUB16MIX)

# C ABI: name -> (restype, argtypes)
_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
SIGNATURES = {
    "mucaInit": (ctypes.c_int, [_P(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_uint64]),
    "mucaInitGroups": (ctypes.c_int, [_P(_vp), _vp, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint32]),
    "mucaDefaultWindow": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _P(_i32),
                                         _P(_i32)]),
    "mucaDestroy": (ctypes.c_int, [_vp]),
    "mucaLastError": (ctypes.c_char_p, []),
    "mucaNumGroups": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "mucaNumWalkers": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "mucaTotalBins": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "mucaGetWindow": (ctypes.c_int, [_vp, ctypes.c_int, _P(_i32), _P(_i32), _P(_i32)]),
    "mucaSetLayout": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mucaGetLayout": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "mucaGetPlacement": (ctypes.c_int, [_vp, _P(ctypes.c_int), _P(ctypes.c_int)]),
    "mucaAutotune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _P(ctypes.c_int),
                                    _P(ctypes.c_double), _vp]),
    "mucaSetLdsLimit": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "mucaSetGraph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mucaSetResidentLimit": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "mucaGetResidentLimit": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "mucaThresholdEntries": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "mucaBuildThresholds": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mucaSweep": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "mucaSweepActive": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp]),
    "mucaSweepNoAlloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "mucaUpdateWeights": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "mucaIsFlat": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mucaRun": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, _P(_i32), _P(_i32), _vp]),
    "mucaReadWalker": (ctypes.c_int, [_vp, ctypes.c_int, _P(ctypes.c_uint32),
                                      _P(ctypes.c_uint32), _P(_i32), _P(ctypes.c_uint64)]),
    "mucaStatus": (ctypes.c_int, [_vp, _vp]),
    "mucaStateBytes": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "mucaSaveState": (ctypes.c_int, [_vp, _vp, ctypes.c_int64]),
    "mucaLoadState": (ctypes.c_int, [_vp, _vp, ctypes.c_int64]),
    "mucaSetTunnelTarget": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mucaCalibrateRandomLines": (ctypes.c_int, [_vp, ctypes.c_int64, _vp, ctypes.c_int64,
                                                ctypes.c_int, _P(ctypes.c_double),
                                                _P(ctypes.c_double), _vp]),
    "mucaReweight": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "mucaLargestCluster": (ctypes.c_int, [_vp, _vp, _vp]),
    "mucaMeasureDroplets": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mucaProduction": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "mucaReweightObservable": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "mucaGetTunnel": (ctypes.c_int, [_vp, _P(ctypes.c_uint32), _P(ctypes.c_uint32)]),
    "mucaMlpParamCount": (ctypes.c_int, []),
    "mucaMlpCreate": (ctypes.c_int, [_P(_vp), ctypes.c_int]),
    "mucaMlpDestroy": (ctypes.c_int, [_vp]),
    "mucaMlpSetParams": (ctypes.c_int, [_vp, _P(ctypes.c_float), ctypes.c_int]),
    "mucaMlpGetParams": (ctypes.c_int, [_vp, _P(ctypes.c_float), ctypes.c_int]),
    "mucaMlpForward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "mucaMlpGradient": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp]),
    "mucaMlpTrainStep": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp]),
    "mucaMlpTableRows": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "mucaMlpPredictWeights": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
}


class MucaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmuca error {code}: {msg}")
        self.code = code


class muca_group(ctypes.Structure):
    _fields_ = [("d", _i32), ("L", _i32), ("N", _i32), ("walkers", _i32), ("e_lo", _i32),
                ("e_hi", _i32)]


_lib = None


def lib():
    """Load libmuca.so (HIP path).  Raises ImportError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(or python paper_1401_4076_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise MucaError(rc, lib().mucaLastError().decode())
    return rc


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, n, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise TypeError(f"{name} must be a contiguous {dtype} tensor of >= {n} entries")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libmuca context (mucaInitGroups).  groups: list of
    (d, L, N, walkers) or (d, L, N, walkers, e_lo, e_hi)."""

    def __init__(self, groups, seed, first_id=0):
        gs = [tuple(g) + ((0, 0) if len(g) == 4 else ()) for g in groups]
        arr = (muca_group * len(gs))(*[muca_group(*g) for g in gs])
        h = ctypes.c_void_p()
        _check(lib().mucaInitGroups(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(gs),
                                    int(seed), int(first_id)))
        self._h = h
        self.groups = gs
        self.ngroups = self._int(lib().mucaNumGroups)
        self.nwalkers = self._int(lib().mucaNumWalkers)
        self.total_bins = self._int(lib().mucaTotalBins)
        self.threshold_entries = self._int(lib().mucaThresholdEntries)

    def _int(self, f):
        v = ctypes.c_int()
        _check(f(self._h, ctypes.byref(v)))
        return v.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().mucaDestroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def window(self, g):
        lo, hi, off = _i32(), _i32(), _i32()
        _check(lib().mucaGetWindow(self._h, g, ctypes.byref(lo), ctypes.byref(hi),
                                   ctypes.byref(off)))
        return lo.value, hi.value, off.value

    def set_layout(self, layout):
        _check(lib().mucaSetLayout(self._h, int(layout)))

    def layout(self):
        return self._int(lib().mucaGetLayout)

    def placement(self):
        """(walker state in LDS, threshold table in LDS) of the resolved layout."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().mucaGetPlacement(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), bool(b.value)

    def set_lds_limit(self, nbytes):
        _check(lib().mucaSetLdsLimit(self._h, int(nbytes)))

    def set_resident_limit(self, nbytes):
        _check(lib().mucaSetResidentLimit(self._h, int(nbytes)))

    def resident_limit(self):
        v = ctypes.c_int64()
        _check(lib().mucaGetResidentLimit(self._h, ctypes.byref(v)))
        return v.value

    def set_graph(self, enable):
        _check(lib().mucaSetGraph(self._h, 1 if enable else 0))

    def autotune(self, lnW, probe_sweeps=1, stream=None):
        """Returns (chosen layout, [ms per layout index 0..4])."""
        ch = ctypes.c_int()
        ms = (ctypes.c_double * MUCA_NUM_LAYOUTS)()
        _check(lib().mucaAutotune(self._h, _dev(lnW, torch.float64, self.total_bins, "lnW"),
                                  int(probe_sweeps), ctypes.byref(ch), ms, _stream(stream)))
        return ch.value, list(ms)

    def build_thresholds(self, lnW, out=None, stream=None):
        p = _dev(lnW, torch.float64, self.total_bins, "lnW")
        o = None if out is None else _dev(out, torch.int32, self.threshold_entries, "out")
        _check(lib().mucaBuildThresholds(self._h, p, o, _stream(stream)))

    def sweep(self, lnW, sweeps, H, active=None, stream=None):
        p = _dev(lnW, torch.float64, self.total_bins, "lnW")
        h = _dev(H, torch.int32, self.total_bins, "H")
        if active is None:
            _check(lib().mucaSweep(self._h, p, int(sweeps), h, _stream(stream)))
        else:
            a = _dev(active, torch.int32, self.ngroups, "active")
            _check(lib().mucaSweepActive(self._h, p, int(sweeps), h, a, _stream(stream)))

    def sweep_noalloc(self, lnW, sweeps, H, stream=None):
        """mucaSweepNoAlloc: the sweep with its tables in the library's static
        device workspace (no allocation in the call)."""
        p = _dev(lnW, torch.float64, self.total_bins, "lnW")
        h = _dev(H, torch.int32, self.total_bins, "H")
        _check(lib().mucaSweepNoAlloc(self._h, p, int(sweeps), h, _stream(stream)))

    def update_weights(self, H, lnW, P, rule=MUCA_RULE_BERG, stream=None):
        _check(lib().mucaUpdateWeights(self._h, _dev(H, torch.int32, self.total_bins, "H"),
                                       _dev(lnW, torch.float64, self.total_bins, "lnW"),
                                       _dev(P, torch.float64, self.total_bins, "P"), int(rule),
                                       _stream(stream)))

    def is_flat(self, H, flags, stream=None):
        _check(lib().mucaIsFlat(self._h, _dev(H, torch.int32, self.total_bins, "H"),
                                _dev(flags, torch.int32, self.ngroups, "flags"),
                                _stream(stream)))

    def run(self, lnW, P, H, sweeps, max_iters, rule=MUCA_RULE_BERG, stop_on_flat=False,
            stream=None, resume=False, stop=None):
        """Returns (status, iters[list], flat[list]).  stop (a MUCA_STOP_*
        value) overrides stop_on_flat."""
        it = (_i32 * self.ngroups)()
        fl = (_i32 * self.ngroups)()
        rc = _check(lib().mucaRun(self._h, _dev(lnW, torch.float64, self.total_bins, "lnW"),
                                  _dev(P, torch.float64, self.total_bins, "P"),
                                  _dev(H, torch.int32, self.total_bins, "H"), int(sweeps),
                                  int(max_iters), int(rule),
                                  int(stop) if stop is not None else (1 if stop_on_flat else 0),
                                  1 if resume else 0, it, fl, _stream(stream)))
        return rc, list(it), list(fl)

    def reweight(self, lnW, H, beta, out, stream=None):
        """Canonical ln Z, <E>, <E^2>, C per group and beta into out (device
        float64, ngroups x len(beta) x 4); beta is a device float64 tensor."""
        nb = int(beta.numel())
        _check(lib().mucaReweight(self._h, _dev(lnW, torch.float64, self.total_bins, "lnW"),
                                  _dev(H, torch.int32, self.total_bins, "H"),
                                  _dev(beta, torch.float64, nb, "beta"), nb,
                                  _dev(out, torch.float64, self.ngroups * nb * 4, "out"),
                                  _stream(stream)))

    def largest_cluster(self, out, stream=None):
        """Largest nearest-neighbour droplet of every walker into out (device
        int32, nwalkers)."""
        _check(lib().mucaLargestCluster(self._h, _dev(out, torch.int32, self.nwalkers, "out"),
                                        _stream(stream)))

    def measure_droplets(self, osum, ocount, out=None, stream=None):
        """Add every walker's largest droplet to osum (device int64) at its
        energy bin and count it in ocount (device int32)."""
        o = None if out is None else _dev(out, torch.int32, self.nwalkers, "out")
        _check(lib().mucaMeasureDroplets(self._h, _dev(osum, torch.int64, self.total_bins, "osum"),
                                         _dev(ocount, torch.int32, self.total_bins, "ocount"), o,
                                         _stream(stream)))

    def production(self, lnW, sweeps_between, measurements, H, osum, ocount, stream=None):
        """mucaProduction: rounds of sweeps and droplet measurements with
        fixed weights."""
        _check(lib().mucaProduction(self._h, _dev(lnW, torch.float64, self.total_bins, "lnW"),
                                    int(sweeps_between), int(measurements),
                                    _dev(H, torch.int32, self.total_bins, "H"),
                                    _dev(osum, torch.int64, self.total_bins, "osum"),
                                    _dev(ocount, torch.int32, self.total_bins, "ocount"),
                                    _stream(stream)))

    def reweight_observable(self, lnW, ocount, osum, beta, out, stream=None):
        """Canonical average of a measured observable per group and beta into
        out (device float64, ngroups x len(beta))."""
        nb = int(beta.numel())
        _check(lib().mucaReweightObservable(
            self._h, _dev(lnW, torch.float64, self.total_bins, "lnW"),
            _dev(ocount, torch.int32, self.total_bins, "ocount"),
            _dev(osum, torch.int64, self.total_bins, "osum"),
            _dev(beta, torch.float64, nb, "beta"), nb,
            _dev(out, torch.float64, self.ngroups * nb, "out"), _stream(stream)))

    def set_tunnel_target(self, target):
        _check(lib().mucaSetTunnelTarget(self._h, int(target)))

    def tunnel(self):
        """(last window end visited, tunnelling events) per walker: two lists."""
        last = (ctypes.c_uint32 * self.nwalkers)()
        trips = (ctypes.c_uint32 * self.nwalkers)()
        _check(lib().mucaGetTunnel(self._h, last, trips))
        return list(last), list(trips)

    def status(self, stream=None):
        return _check(lib().mucaStatus(self._h, _stream(stream)))

    def state_bytes(self):
        n = ctypes.c_int64()
        _check(lib().mucaStateBytes(self._h, ctypes.byref(n)))
        return n.value

    def save_state(self):
        """mucaSaveState into a new host bytearray (the state image)."""
        n = self.state_bytes()
        buf = bytearray(n)
        _check(lib().mucaSaveState(self._h, (ctypes.c_char * n).from_buffer(buf), n))
        return buf

    def load_state(self, image):
        """mucaLoadState from a bytes-like state image."""
        data = bytes(image)
        _check(lib().mucaLoadState(self._h, data, len(data)))

    def read_walker(self, w):
        """(bits[words] uint32 list, pos[N] list, E, t) of walker w."""
        acc = 0
        for g in self.groups:
            if w < acc + g[3]:
                break
            acc += g[3]
        d, L, N = g[0], g[1], g[2]
        words = (L ** d + 31) // 32
        bits = (ctypes.c_uint32 * words)()
        pos = (ctypes.c_uint32 * N)()
        E = _i32()
        t = ctypes.c_uint64()
        _check(lib().mucaReadWalker(self._h, int(w), bits, pos, ctypes.byref(E), ctypes.byref(t)))
        return list(bits), list(pos), E.value, t.value


def calibrate_random_lines(table, sink, rounds, stream=None):
    """mucaCalibrateRandomLines on a device uint8/int32 table and int32 sink;
    returns (lines read, seconds) of the timed launch."""
    lines, sec = ctypes.c_double(), ctypes.c_double()
    nbytes = table.numel() * table.element_size()
    _check(lib().mucaCalibrateRandomLines(ctypes.c_void_p(table.data_ptr()), int(nbytes),
                                          ctypes.c_void_p(sink.data_ptr()), int(sink.numel()),
                                          int(rounds), ctypes.byref(lines), ctypes.byref(sec),
                                          _stream(stream)))
    return lines.value, sec.value


def mucaDefaultWindow(d, L, N):
    lo, hi = _i32(), _i32()
    _check(lib().mucaDefaultWindow(int(d), int(L), int(N), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def mucaInitGroups(groups, seed, first_id=0):
    return Context(groups, seed, first_id)


def mucaInit(d, L, N, walkers, seed):
    return Context([(d, L, N, walkers)], seed)


def mucaSweep(ctx, lnW, sweeps, H, stream=None):
    ctx.sweep(lnW, sweeps, H, stream=stream)


def mucaSweepNoAlloc(ctx, lnW, sweeps, H, stream=None):
    ctx.sweep_noalloc(lnW, sweeps, H, stream=stream)


def mucaSweepActive(ctx, lnW, sweeps, H, active, stream=None):
    ctx.sweep(lnW, sweeps, H, active=active, stream=stream)


def mucaUpdateWeights(ctx, H, lnW, P, rule=MUCA_RULE_BERG, stream=None):
    ctx.update_weights(H, lnW, P, rule, stream)


def mucaIsFlat(ctx, H, flags, stream=None):
    ctx.is_flat(H, flags, stream)


def mucaBuildThresholds(ctx, lnW, out=None, stream=None):
    ctx.build_thresholds(lnW, out, stream)


def mucaRun(ctx, lnW, P, H, sweeps_per_iter, max_iters, rule=MUCA_RULE_BERG, stop_on_flat=False,
            stream=None, resume=False):
    return ctx.run(lnW, P, H, sweeps_per_iter, max_iters, rule, stop_on_flat, stream, resume)


def mucaReadWalker(ctx, walker):
    return ctx.read_walker(walker)


def mucaSaveState(ctx):
    return ctx.save_state()


def mucaLoadState(ctx, image):
    return ctx.load_state(image)


def mucaDestroy(ctx):
    ctx.close()


class Mlp:
    """The learned-initial-weights network (mucaMlp*).  Tensors are CUDA
    float32 (features rows x 4, targets / outputs rows)."""

    def __init__(self, max_rows):
        h = ctypes.c_void_p()
        _check(lib().mucaMlpCreate(ctypes.byref(h), int(max_rows)))
        self._h = h
        self.max_rows = int(max_rows)
        self.nparams = lib().mucaMlpParamCount()

    def close(self):
        if self._h:
            lib().mucaMlpDestroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().mucaMlpSetParams(self._h, p.ctypes.data_as(_P(ctypes.c_float)), p.size))

    def get_params(self):
        import numpy as np
        p = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().mucaMlpGetParams(self._h, p.ctypes.data_as(_P(ctypes.c_float)), p.size))
        return p

    def forward(self, X, Y, stream=None):
        rows = X.shape[0]
        _check(lib().mucaMlpForward(self._h, _dev(X, torch.float32, rows * 4, "X"), rows,
                                    _dev(Y, torch.float32, rows, "Y"), _stream(stream)))

    def gradient(self, X, T, grad, loss=None, stream=None):
        rows = X.shape[0]
        _check(lib().mucaMlpGradient(self._h, _dev(X, torch.float32, rows * 4, "X"),
                                     _dev(T, torch.float32, rows, "T"), rows,
                                     _dev(grad, torch.float32, self.nparams, "grad"),
                                     None if loss is None else _dev(loss, torch.float32, 1, "loss"),
                                     _stream(stream)))

    def train_step(self, X, T, lr, loss=None, stream=None):
        rows = X.shape[0]
        _check(lib().mucaMlpTrainStep(self._h, _dev(X, torch.float32, rows * 4, "X"),
                                      _dev(T, torch.float32, rows, "T"), rows, float(lr),
                                      None if loss is None else _dev(loss, torch.float32, 1,
                                                                     "loss"),
                                      _stream(stream)))

    def predict_weights(self, ctx, group, lnW, stream=None):
        _check(lib().mucaMlpPredictWeights(self._h, ctx.handle, int(group),
                                           _dev(lnW, torch.float64, ctx.total_bins, "lnW"),
                                           _stream(stream)))


def mucaMlpTableRows(ctx, group, lnW, X, T=None, stream=None):
    lo, hi, _ = ctx.window(group)
    nb = hi - lo + 1
    _check(lib().mucaMlpTableRows(ctx.handle, int(group),
                                  None if lnW is None else _dev(lnW, torch.float64,
                                                                ctx.total_bins, "lnW"),
                                  _dev(X, torch.float32, nb * 4, "X"),
                                  None if T is None else _dev(T, torch.float32, nb, "T"),
                                  _stream(stream)))
