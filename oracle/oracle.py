"""ctypes view of the reference oracle (test infrastructure only).

The oracle is a plain single-threaded C implementation of replica-exchange
Wang-Landau sampling written from the paper (arXiv:1402.2328, Secs. 2-3 and
Eqs. 1-2, 7-8).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

ISING, POTTS = 0, 1
FP64, FP32C = 0, 1
HALVING, ONE_OVER_T = 0, 1


class Params(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("L", C.c_int32), ("q", C.c_int32),
        ("n_windows", C.c_int32), ("overlap_num", C.c_int32), ("overlap_den", C.c_int32),
        ("walkers_per_window", C.c_int32), ("flat_num", C.c_int32), ("flat_den", C.c_int32),
        ("lnf_init", C.c_double), ("lnf_final", C.c_double),
        ("flips_per_exchange", C.c_int64), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("instance", C.c_int32),
        ("schedule", C.c_int32), ("reserved", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("N", "nbins", "binw", "emin", "h", "m", "W", "max_nb")]


class Status(C.Structure):
    _fields_ = [("done", C.c_int32), ("pad", C.c_int32), ("done_merge", C.c_int64),
                ("merges", C.c_int64), ("rounds", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("REWL_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_new.restype = P
        L.orc_new.argtypes = [C.POINTER(Params), P, P]
        L.orc_free.argtypes = [P]
        L.orc_get_info.argtypes = [P, C.POINTER(Info)]
        L.orc_get_windows.argtypes = [P, P, P]
        L.orc_warm_status.argtypes = [P]
        L.orc_run.restype = C.c_int64
        L.orc_run.argtypes = [P, C.c_int64]
        L.orc_sweep.argtypes = [P, C.c_int64]
        L.orc_merge.argtypes = [P]
        L.orc_exchange.argtypes = [P]
        L.orc_status.argtypes = [P, C.POINTER(Status)]
        L.orc_get_walker.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.orc_get_walker_f32.argtypes = [P, C.c_int32, P, P]
        L.orc_set_walker_lng.argtypes = [P, C.c_int32, P]
        L.orc_get_window.argtypes = [P, C.c_int32, P, P, P, P, P]
        L.orc_get_exchange_stats.argtypes = [P, P, P, P]
        L.orc_join.argtypes = [P, P, P]
        L.orc_join_raw.argtypes = [P, P, P]
        L.orc_jackknife.argtypes = [P, P, P]
        L.orc_get_phase.argtypes = [P, C.c_int32]
        L.orc_get_piece.argtypes = [P, C.c_int32, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_exp_spec.restype = C.c_double
        L.orc_exp_spec.argtypes = [C.c_double]
        L.orc_expf_spec.restype = C.c_float
        L.orc_expf_spec.argtypes = [C.c_float]
        L.orc_exchange_pairing.argtypes = [C.c_uint64, C.c_int32, C.c_uint64, C.c_int32,
                                           C.c_int32, P]
        L.orc_accept64.argtypes = [C.c_uint64, C.c_double]
        L.orc_accept32.argtypes = [C.c_uint32, C.c_float]
        L.orc_energy.restype = C.c_int32
        L.orc_energy.argtypes = [C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_equal_windows.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.orc_stitch.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P]
        L.orc_normalise.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_thermo.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, C.c_int32, P, P]
        for n in ("orc_df_add1", "orc_df_add", "orc_df_div_int"):
            getattr(L, n).restype = None
        L.orc_df_add1.argtypes = [C.c_float, C.c_float, C.c_float, P, P]
        L.orc_df_add.argtypes = [C.c_float, C.c_float, C.c_float, C.c_float, P, P]
        L.orc_df_div_int.argtypes = [C.c_float, C.c_float, C.c_int32, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def make_params(model, L, q=2, n_windows=1, overlap=(3, 4), walkers_per_window=1,
                flat=(4, 5), lnf_init=1.0, lnf_final=1e-8, flips_per_exchange=10000,
                seed=1, precision=FP64, instance=0, schedule=HALVING):
    return Params(model, L, q, n_windows, overlap[0], overlap[1], walkers_per_window,
                  flat[0], flat[1], lnf_init, lnf_final, flips_per_exchange, seed,
                  precision, instance, schedule, 0)


class Sim:
    """One REWL instance run by the oracle."""

    def __init__(self, params=None, windows=None, **kw):
        self.params = params if params is not None else make_params(**kw)
        L = lib()
        if windows is not None:
            lo = np.ascontiguousarray(windows[0], dtype=np.int32)
            hi = np.ascontiguousarray(windows[1], dtype=np.int32)
            self._h = L.orc_new(C.byref(self.params), _p(lo), _p(hi))
        else:
            self._h = L.orc_new(C.byref(self.params), None, None)
        if not self._h:
            raise ValueError("oracle rejected parameters")
        self.info = Info()
        L.orc_get_info(self._h, C.byref(self.info))
        self.lo = np.zeros(self.info.h, np.int32)
        self.hi = np.zeros(self.info.h, np.int32)
        L.orc_get_windows(self._h, _p(self.lo), _p(self.hi))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    @property
    def warm_ok(self):
        return lib().orc_warm_status(self._h) == 0

    def run(self, cycles):
        return lib().orc_run(self._h, cycles)

    def sweep(self, flips):
        return lib().orc_sweep(self._h, flips)

    def merge(self):
        return lib().orc_merge(self._h)

    def exchange(self):
        return lib().orc_exchange(self._h)

    def status(self):
        st = Status()
        lib().orc_status(self._h, C.byref(st))
        return {"done": st.done, "done_merge": st.done_merge, "merges": st.merges,
                "rounds": st.rounds}

    def walker(self, slot):
        w = slot // self.info.m
        nb = int(self.hi[w] - self.lo[w] + 1)
        spins = np.zeros(self.info.N, np.int8)
        H = np.zeros(nb, np.uint32)
        lng = np.zeros(nb, np.float64)
        E = C.c_int32()
        att = C.c_uint64()
        cid = C.c_int32()
        lib().orc_get_walker(self._h, slot, _p(spins), C.byref(E), _p(H), _p(lng),
                             C.byref(att), C.byref(cid))
        out = {"spins": spins, "E": E.value, "H": H, "lng": lng, "attempts": att.value,
               "config": cid.value}
        if self.params.precision == FP32C:
            hi = np.zeros(nb, np.float32)
            lo = np.zeros(nb, np.float32)
            lib().orc_get_walker_f32(self._h, slot, _p(hi), _p(lo))
            out["lng_hi"], out["lng_lo"] = hi, lo
        return out

    def set_lng(self, slot, lng):
        a = np.ascontiguousarray(lng, dtype=np.float64)
        if lib().orc_set_walker_lng(self._h, slot, _p(a)):
            raise ValueError("bad slot")

    def window(self, w):
        nb = int(self.hi[w] - self.lo[w] + 1)
        U = np.zeros(nb, np.uint8)
        sm = np.zeros(64, np.int64)
        lnf = C.c_double()
        stage = C.c_int32()
        frozen = C.c_int32()
        lib().orc_get_window(self._h, w, C.byref(lnf), C.byref(stage), C.byref(frozen),
                             _p(U), _p(sm))
        return {"lnf": lnf.value, "stage": stage.value, "frozen": frozen.value, "U": U,
                "stage_merge": sm, "phase": lib().orc_get_phase(self._h, w)}

    def piece(self, slot):
        w = slot // self.info.m
        out = np.zeros(int(self.hi[w] - self.lo[w] + 1), np.float64)
        if lib().orc_get_piece(self._h, slot, _p(out)):
            raise ValueError("bad slot")
        return out

    def exchange_stats(self):
        t = np.zeros(self.info.h, np.uint64)
        r = np.zeros(self.info.h, np.uint64)
        a = np.zeros(self.info.h, np.uint64)
        lib().orc_get_exchange_stats(self._h, _p(t), _p(r), _p(a))
        return t, r, a

    def jackknife(self):
        mean = np.zeros(self.info.nbins, np.float64)
        err = np.zeros(self.info.nbins, np.float64)
        if lib().orc_jackknife(self._h, _p(mean), _p(err)):
            raise RuntimeError("jackknife needs a finished run with m >= 2")
        return mean, err

    def join(self, normalise=True):
        out = np.zeros(self.info.nbins, np.float64)
        joins = np.zeros(max(self.info.h - 1, 1), np.int32)
        f = lib().orc_join if normalise else lib().orc_join_raw
        rc = f(self._h, _p(out), _p(joins))
        if rc:
            raise RuntimeError("join failed")
        return out, joins[: self.info.h - 1]


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def exchange_pairing(seed, instance, rnd, w, m):
    """Permutation pi of 0..m-1: walker k of window w meets walker pi[k] of
    window w+1 in exchange round `rnd`."""
    pi = np.zeros(m, np.int32)
    if lib().orc_exchange_pairing(int(seed), int(instance), int(rnd), int(w), int(m), _p(pi)):
        raise ValueError("bad pairing arguments")
    return pi


def exp_spec(x):
    return lib().orc_exp_spec(float(x))


def expf_spec(x):
    return lib().orc_expf_spec(float(np.float32(x)))


def accept64(u53, delta):
    return bool(lib().orc_accept64(int(u53), float(delta)))


def accept32(u24, delta):
    return bool(lib().orc_accept32(int(u24), float(np.float32(delta))))


def energy(model, L, q, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    return lib().orc_energy(model, L, q, _p(s))


def equal_windows(nbins, h, on=3, od=4):
    lo = np.zeros(h, np.int32)
    hi = np.zeros(h, np.int32)
    if lib().orc_equal_windows(nbins, h, on, od, _p(lo), _p(hi)):
        raise ValueError("bad window parameters")
    return lo, hi


def stitch(lo, hi, pieces, masks, nbins):
    h = len(lo)
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    pieces = [np.ascontiguousarray(p, dtype=np.float64) for p in pieces]
    masks = [np.ascontiguousarray(m, dtype=np.uint8) for m in masks]
    lp = (C.c_void_p * h)(*[p.ctypes.data for p in pieces])
    mp = (C.c_void_p * h)(*[m.ctypes.data for m in masks])
    R = np.zeros(nbins, np.float64)
    joins = np.zeros(max(h - 1, 1), np.int32)
    lib().orc_stitch(h, _p(lo), _p(hi), C.cast(lp, C.c_void_p), C.cast(mp, C.c_void_p),
                     nbins, _p(R), _p(joins))
    return R, joins[: h - 1]


def normalise(model, N, q, R):
    R = np.array(R, dtype=np.float64)
    if lib().orc_normalise(model, N, q, len(R), _p(R)):
        raise ValueError("normalise failed")
    return R


def thermo(lng, emin, binw, T):
    lng = np.ascontiguousarray(lng, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    Em = np.zeros(len(T))
    Cv = np.zeros(len(T))
    lib().orc_thermo(_p(lng), len(lng), emin, binw, _p(T), len(T), _p(Em), _p(Cv))
    return Em, Cv


def df_add1(ah, al, b):
    rh, rl = C.c_float(), C.c_float()
    lib().orc_df_add1(ah, al, b, C.byref(rh), C.byref(rl))
    return rh.value, rl.value


def df_add(ah, al, bh, bl):
    rh, rl = C.c_float(), C.c_float()
    lib().orc_df_add(ah, al, bh, bl, C.byref(rh), C.byref(rl))
    return rh.value, rl.value


def df_div_int(ah, al, m):
    rh, rl = C.c_float(), C.c_float()
    lib().orc_df_div_int(ah, al, m, C.byref(rh), C.byref(rl))
    return rh.value, rl.value
