"""ctypes wrapper of the CPU oracle (muca_ref.c).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only tests/, the smoke check in
__graft_entry__.py and the CPU-baseline leg of bench.py may import this
package.  It shares no code with the GPU library paper_1401_4076_amd.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("MUCA_REF_LIB", os.path.join(_HERE, "libmuca_ref.so"))
_lib = None


class RefGroup(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("L", ctypes.c_int32), ("N", ctypes.c_int32),
                ("walkers", ctypes.c_int32), ("e_lo", ctypes.c_int32),
                ("e_hi", ctypes.c_int32)]


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    u32p, i32p, i64p, f64p, u8p, u64p = (P(ctypes.c_uint32), P(ctypes.c_int32),
                                          P(ctypes.c_int64), P(ctypes.c_double),
                                          P(ctypes.c_uint8), P(ctypes.c_uint64))
    vp = ctypes.c_void_p
    sig = {
        "ref_philox": (None, [u32p, u32p, u32p]),
        "ref_exp": (ctypes.c_double, [ctypes.c_double]),
        "ref_log": (ctypes.c_double, [ctypes.c_int64]),
        "ref_accept": (ctypes.c_int, [ctypes.c_double, ctypes.c_uint32]),
        "ref_energy_floor": (ctypes.c_int32, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "ref_brute_dos": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p]),
        "ref_create": (vp, [P(RefGroup), ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32]),
        "ref_destroy": (None, [vp]),
        "ref_num_groups": (ctypes.c_int, [vp]),
        "ref_window": (ctypes.c_int, [vp, ctypes.c_int, i32p, i32p]),
        "ref_total_bins": (ctypes.c_int, [vp]),
        "ref_bin_offset": (ctypes.c_int, [vp, ctypes.c_int]),
        "ref_num_walkers": (ctypes.c_int, [vp]),
        "ref_sweep": (ctypes.c_int, [vp, f64p, ctypes.c_int, i32p, i32p]),
        "ref_update": (ctypes.c_int, [vp, i32p, f64p, f64p, ctypes.c_int, i32p]),
        "ref_flat": (ctypes.c_int, [vp, i32p, i32p]),
        "ref_run": (ctypes.c_int, [vp, f64p, f64p, i32p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, i32p]),
        "ref_get_tunnel": (ctypes.c_int, [vp, u32p, u32p]),
        "ref_get_walker": (ctypes.c_int, [vp, ctypes.c_int, u8p, u32p, i32p, u64p]),
        "ref_set_walker": (ctypes.c_int, [vp, ctypes.c_int, u8p, u32p, ctypes.c_int32,
                                          ctypes.c_uint64]),
        "ref_recount": (ctypes.c_int32, [vp, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox(ctr, key):
    """Philox4x32-10 block for counter (4 words) and key (2 words)."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ref_philox(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                     _ptr(out, ctypes.c_uint32))
    return out


def exp(x):
    return lib().ref_exp(float(x))


def log(h):
    return lib().ref_log(int(h))


def accept(x, u):
    return bool(lib().ref_accept(float(x), int(u)))


def energy_floor(d, L, N):
    return int(lib().ref_energy_floor(d, L, N))


def brute_dos(d, L, N):
    """Exact Omega(E) as a dict {E: count} by enumeration of all configurations."""
    om = np.zeros(d * N + 1, dtype=np.int64)
    rc = lib().ref_brute_dos(d, L, N, _ptr(om, ctypes.c_int64))
    if rc != 0:
        raise ValueError("invalid brute_dos arguments")
    return {-k: int(v) for k, v in enumerate(om) if v}


class RefContext:
    """Oracle state for a list of groups (d, L, N, walkers[, e_lo, e_hi])."""

    def __init__(self, groups, seed, first_id=0):
        gs = []
        for g in groups:
            g = tuple(g)
            if len(g) == 4:
                g = g + (0, 0)
            gs.append(g)
        arr = (RefGroup * len(gs))(*[RefGroup(*g) for g in gs])
        self._groups = gs
        self._h = lib().ref_create(arr, len(gs), int(seed), int(first_id))
        if not self._h:
            raise ValueError("ref_create rejected the groups")
        self.ngroups = lib().ref_num_groups(self._h)
        self.total_bins = lib().ref_total_bins(self._h)
        self.nwalkers = lib().ref_num_walkers(self._h)

    def close(self):
        if self._h:
            lib().ref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def window(self, g):
        lo, hi = ctypes.c_int32(), ctypes.c_int32()
        lib().ref_window(self._h, g, ctypes.byref(lo), ctypes.byref(hi))
        return lo.value, hi.value

    def bin_offset(self, g):
        return lib().ref_bin_offset(self._h, g)

    def bins(self, g):
        lo, hi = self.window(g)
        return hi - lo + 1

    def zeros_lnW(self):
        return np.zeros(self.total_bins, dtype=np.float64)

    def sweep(self, lnW, sweeps, active=None):
        lnW = np.ascontiguousarray(lnW, dtype=np.float64)
        H = np.zeros(self.total_bins, dtype=np.int32)
        act = None
        if active is not None:
            act = np.ascontiguousarray(active, dtype=np.int32)
        rc = lib().ref_sweep(self._h, _ptr(lnW, ctypes.c_double), int(sweeps),
                             _ptr(H, ctypes.c_int32),
                             None if act is None else _ptr(act, ctypes.c_int32))
        if rc != 0:
            raise RuntimeError(f"ref_sweep failed ({rc})")
        return H

    def update(self, H, lnW, P, rule=0, active=None):
        """In-place update of lnW and P (numpy float64 arrays)."""
        H = np.ascontiguousarray(H, dtype=np.int32)
        act = None if active is None else np.ascontiguousarray(active, dtype=np.int32)
        rc = lib().ref_update(self._h, _ptr(H, ctypes.c_int32), _ptr(lnW, ctypes.c_double),
                              _ptr(P, ctypes.c_double), int(rule),
                              None if act is None else _ptr(act, ctypes.c_int32))
        if rc != 0:
            raise RuntimeError(f"ref_update failed ({rc})")

    def flat(self, H):
        H = np.ascontiguousarray(H, dtype=np.int32)
        f = np.zeros(self.ngroups, dtype=np.int32)
        lib().ref_flat(self._h, _ptr(H, ctypes.c_int32), _ptr(f, ctypes.c_int32))
        return f

    def run(self, lnW, P, sweeps, max_iters, rule=0, stop_on_flat=False, tunnel_target=None):
        """In-place run; returns (status, H, iters, flat).  With tunnel_target a
        group stops once its walkers made that many tunnelling events."""
        H = np.zeros(self.total_bins, dtype=np.int32)
        it = np.zeros(self.ngroups, dtype=np.int32)
        fl = np.zeros(self.ngroups, dtype=np.int32)
        stop = 2 if tunnel_target is not None else (1 if stop_on_flat else 0)
        rc = lib().ref_run(self._h, _ptr(lnW, ctypes.c_double), _ptr(P, ctypes.c_double),
                           _ptr(H, ctypes.c_int32), int(sweeps), int(max_iters), int(rule),
                           stop, int(tunnel_target or 0), _ptr(it, ctypes.c_int32),
                           _ptr(fl, ctypes.c_int32))
        if rc < 0:
            raise RuntimeError(f"ref_run failed ({rc})")
        return rc, H, it, fl

    def _group_of(self, w):
        acc = 0
        for gi, g in enumerate(self._groups):
            if w < acc + g[3]:
                return gi
            acc += g[3]
        raise IndexError(w)

    def walker(self, w):
        """(n[V] uint8, pos[N] uint32, E, t) of walker w."""
        g = self._groups[self._group_of(w)]
        V = g[1] ** g[0]
        n = np.zeros(V, dtype=np.uint8)
        pos = np.zeros(g[2], dtype=np.uint32)
        E = ctypes.c_int32()
        t = ctypes.c_uint64()
        lib().ref_get_walker(self._h, w, _ptr(n, ctypes.c_uint8), _ptr(pos, ctypes.c_uint32),
                             ctypes.byref(E), ctypes.byref(t))
        return n, pos, E.value, t.value

    def set_walker(self, w, n, pos, E, t):
        n = np.ascontiguousarray(n, dtype=np.uint8)
        pos = np.ascontiguousarray(pos, dtype=np.uint32)
        lib().ref_set_walker(self._h, w, _ptr(n, ctypes.c_uint8), _ptr(pos, ctypes.c_uint32),
                             int(E), int(t))

    def tunnel(self):
        """(last window end visited, tunnelling events) per walker, uint32 arrays."""
        last = np.zeros(self.nwalkers, dtype=np.uint32)
        trips = np.zeros(self.nwalkers, dtype=np.uint32)
        lib().ref_get_tunnel(self._h, _ptr(last, ctypes.c_uint32), _ptr(trips, ctypes.c_uint32))
        return last, trips

    def recount(self, w):
        return int(lib().ref_recount(self._h, w))
