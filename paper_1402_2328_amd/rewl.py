"""Thin Python binding of librewl (include/rewl.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies the device workspace (a uint8 tensor) and the stream.  If
the built library is missing, importing this module raises: there is no
fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librewl.so")

ISING, POTTS = 0, 1
FP64, FP32C = 0, 1
HALVING, ONE_OVER_T = 0, 1

ERRORS = {0: "ok", -1: "invalid argument", -2: "workspace or buffer too small",
          -3: "HIP runtime error", -4: "non-finite ln g", -5: "histogram overflow",
          -6: "call not valid in this state", -7: "walker could not reach its window",
          -8: "checkpoint does not match this context"}


class RewlError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {ERRORS.get(code, 'unknown')} ({code})")
        self.code = code


class rewl_params(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("L", C.c_int32), ("q", C.c_int32), ("n_windows", C.c_int32),
        ("overlap_num", C.c_int32), ("overlap_den", C.c_int32),
        ("walkers_per_window", C.c_int32), ("flat_num", C.c_int32), ("flat_den", C.c_int32),
        ("precision", C.c_int32), ("lnf_init", C.c_double), ("lnf_final", C.c_double),
        ("flips_per_exchange", C.c_int64), ("seed", C.c_uint64),
        ("schedule", C.c_int32), ("reserved", C.c_int32),
    ]


class rewl_instance_status(C.Structure):
    _fields_ = [("done", C.c_int32), ("error", C.c_int32), ("done_merge", C.c_int64),
                ("merges", C.c_int64), ("rounds", C.c_uint64), ("attempts", C.c_uint64)]


_lib = None

EXPORTS = ["rewl_workspace_bytes", "rewl_init", "rewl_run_sweeps", "rewl_set_launch",
           "rewl_set_batching",
           "rewl_autotune", "rewl_merge",
           "rewl_exchange", "rewl_run_cycles", "rewl_status", "rewl_running",
           "rewl_get_lng", "rewl_get_geometry", "rewl_get_walker", "rewl_get_walker_f32",
           "rewl_get_visited", "rewl_get_exchange_stats", "rewl_thermo", "rewl_checkpoint",
           "rewl_restore", "rewl_destroy", "rewl_strerror", "rewl_get_schedule",
           "rewl_get_piece", "rewl_jackknife", "rewl_balanced_windows", "rewl_locate_walker",
           "rewl_jackknife_noalloc"]


def lib():
    """Load librewl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.rewl_workspace_bytes.restype = SZ
    L.rewl_workspace_bytes.argtypes = [P, I32, P, P]
    L.rewl_init.argtypes = [P, I32, P, P, P, SZ, P, C.POINTER(C.c_void_p)]
    L.rewl_run_sweeps.argtypes = [P, I64]
    L.rewl_set_launch.argtypes = [P, I32, I32, I32, I32, I32, P]
    L.rewl_set_batching.argtypes = [P, I32, I32, I32, P]
    L.rewl_autotune.argtypes = [P, I64, I32, P]
    L.rewl_merge.argtypes = [P]
    L.rewl_exchange.argtypes = [P]
    L.rewl_run_cycles.argtypes = [P, I64, I64, I32]
    L.rewl_status.argtypes = [P, I32, C.POINTER(rewl_instance_status), P, P, P]
    L.rewl_running.argtypes = [P, C.POINTER(I32)]
    L.rewl_get_lng.argtypes = [P, I32, I32, P, I32, C.POINTER(I32), P]
    L.rewl_get_geometry.argtypes = [P, I32, P, P, P, P, P, P, P, P, P]
    L.rewl_get_walker.argtypes = [P, I32, I32, P, P, P, P, P, P]
    L.rewl_get_walker_f32.argtypes = [P, I32, I32, P, P]
    L.rewl_locate_walker.argtypes = [P, I32, I32, C.POINTER(SZ), C.POINTER(SZ), C.POINTER(SZ),
                                     C.POINTER(I32)]
    L.rewl_get_visited.argtypes = [P, I32, I32, P]
    L.rewl_get_exchange_stats.argtypes = [P, I32, P, P, P]
    L.rewl_thermo.argtypes = [P, I32, P, I32, P, P]
    L.rewl_get_schedule.argtypes = [P, I32, P, P]
    L.rewl_get_piece.argtypes = [P, I32, I32, P]
    L.rewl_jackknife.argtypes = [P, I32, P, P, I32, C.POINTER(I32)]
    L.rewl_jackknife_noalloc.argtypes = [P, I32, P, P, I32, C.POINTER(I32)]
    L.rewl_balanced_windows.argtypes = [I32, I32, I32, I32, I32, P, P, P, C.c_double, P, P]
    L.rewl_checkpoint.argtypes = [P, P, SZ, C.POINTER(SZ)]
    L.rewl_restore.argtypes = [P, P, SZ]
    L.rewl_destroy.argtypes = [P]
    L.rewl_strerror.restype = C.c_char_p
    L.rewl_strerror.argtypes = [C.c_int]
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RewlError(rc, what)


def make_params(model=ISING, L=8, q=2, n_windows=1, overlap=(3, 4), walkers_per_window=1,
                flat=(4, 5), precision=FP64, lnf_init=1.0, lnf_final=1e-8,
                flips_per_exchange=10000, seed=1, schedule=HALVING):
    return rewl_params(model, L, q, n_windows, overlap[0], overlap[1], walkers_per_window,
                       flat[0], flat[1], precision, lnf_init, lnf_final, flips_per_exchange, seed,
                       schedule, 0)


def balanced_windows(nbins, h, pre_lo, pre_hi, pre_steps, overlap=(3, 4), alpha=2.0):
    """Run-time balanced split (rewl_balanced_windows); returns (lo, hi)."""
    pl = np.ascontiguousarray(pre_lo, dtype=np.int32)
    ph = np.ascontiguousarray(pre_hi, dtype=np.int32)
    ps = np.ascontiguousarray(pre_steps, dtype=np.float64)
    if not (len(pl) == len(ph) == len(ps)):
        raise ValueError("pre-run arrays differ in length")
    lo = np.zeros(h, np.int32)
    hi = np.zeros(h, np.int32)
    _check(lib().rewl_balanced_windows(int(nbins), int(h), int(overlap[0]), int(overlap[1]),
                                       len(pl), _p(pl), _p(ph), _p(ps), float(alpha), _p(lo),
                                       _p(hi)), "rewl_balanced_windows")
    return lo, hi


def _window_arrays(windows):
    if windows is None:
        return None, None
    lo = np.ascontiguousarray(np.concatenate([np.asarray(w[0]) for w in windows]), dtype=np.int32)
    hi = np.ascontiguousarray(np.concatenate([np.asarray(w[1]) for w in windows]), dtype=np.int32)
    return lo, hi


def rewl_workspace_bytes(params, windows=None):
    arr = (rewl_params * len(params))(*params)
    lo, hi = _window_arrays(windows)
    return lib().rewl_workspace_bytes(C.cast(arr, C.c_void_p), len(params), _p(lo), _p(hi))


class Context:
    """A batch of REWL instances living in one device workspace.

    Method names follow the C-ABI (rewl_init -> Context(...), rewl_run_sweeps
    -> run_sweeps, ...).  The workspace is a torch uint8 tensor on the current
    device; work goes to torch's current stream unless `stream` is given.
    """

    def __init__(self, params, windows=None, stream=None, device=None):
        import torch

        self.params = list(params)
        self._arr = (rewl_params * len(self.params))(*self.params)
        self._wlo, self._whi = _window_arrays(windows)
        nbytes = rewl_workspace_bytes(self.params, windows)
        if nbytes == 0:
            raise RewlError(-1, "rewl_workspace_bytes")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = C.c_void_p()
        _check(lib().rewl_init(C.cast(self._arr, C.c_void_p), len(self.params), _p(self._wlo),
                               _p(self._whi), C.c_void_p(self.workspace.data_ptr()), nbytes,
                               C.c_void_p(self.stream.cuda_stream), C.byref(self._h)), "rewl_init")
        self.geometry = [self.get_geometry(i) for i in range(len(self.params))]

    def close(self):
        if getattr(self, "_h", None):
            lib().rewl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- hot path ----
    def run_sweeps(self, flips):
        _check(lib().rewl_run_sweeps(self._h, int(flips)), "rewl_run_sweeps")

    CLASSES = ("ising_L<=32", "ising_L<=64", "potts")

    PLAN_WORDS = 21

    @staticmethod
    def _plan(out):
        """Per class present: its launch shape; and, when not the default
        (per-class launches, one launch per sweep), the batching."""
        plan = {}
        for c, name in enumerate(Context.CLASSES):
            if out[6 * c + 3] > 0:
                plan[name] = {"page_bins": int(out[6 * c]), "walkers_per_group": int(out[6 * c + 1]),
                              "lds_bytes": int(out[6 * c + 2]), "workgroups": int(out[6 * c + 3]),
                              "rng_producer": int(out[6 * c + 4]), "potts_nibbles": int(out[6 * c + 5])}
        if out[18] or out[19] != 1:
            plan["batching"] = {"fused": int(out[18]), "splits": int(out[19]), "order": int(out[20])}
        return plan

    def set_launch(self, page_bins=0, walkers_per_group=0, cls=-1, rng_producer=-1,
                   potts_nibbles=-1):
        out = np.zeros(self.PLAN_WORDS, np.int32)
        _check(lib().rewl_set_launch(self._h, int(cls), int(page_bins), int(walkers_per_group),
                                     int(rng_producer), int(potts_nibbles), _p(out)),
               "rewl_set_launch")
        return self._plan(out)

    def set_batching(self, fused=0, splits=1, order=0):
        out = np.zeros(self.PLAN_WORDS, np.int32)
        _check(lib().rewl_set_batching(self._h, int(fused), int(splits), int(order), _p(out)),
               "rewl_set_batching")
        return self._plan(out)

    def autotune(self, flips, repeats=1):
        out = np.zeros(self.PLAN_WORDS, np.int32)
        _check(lib().rewl_autotune(self._h, int(flips), int(repeats), _p(out)), "rewl_autotune")
        return self._plan(out)

    def merge(self):
        _check(lib().rewl_merge(self._h), "rewl_merge")

    def exchange(self):
        _check(lib().rewl_exchange(self._h), "rewl_exchange")

    def run_cycles(self, cycles, flips, use_graph=False):
        _check(lib().rewl_run_cycles(self._h, int(cycles), int(flips), int(bool(use_graph))),
               "rewl_run_cycles")

    # ---- queries (synchronise) ----
    def status(self, instance=0):
        g = self.geometry[instance]
        st = rewl_instance_status()
        stage = np.zeros(g["h"], np.int32)
        frozen = np.zeros(g["h"], np.int32)
        lnf = np.zeros(g["h"], np.float64)
        _check(lib().rewl_status(self._h, instance, C.byref(st), _p(stage), _p(frozen), _p(lnf)),
               "rewl_status")
        return {"done": st.done, "error": st.error, "done_merge": st.done_merge,
                "merges": st.merges, "rounds": st.rounds, "attempts": st.attempts,
                "stage": stage, "frozen": frozen, "lnf": lnf}

    def running(self):
        n = C.c_int32()
        _check(lib().rewl_running(self._h, C.byref(n)), "rewl_running")
        return n.value

    def get_geometry(self, instance=0):
        v = [C.c_int32() for _ in range(7)]
        h = self.params[instance].n_windows
        lo = np.zeros(h, np.int32)
        hi = np.zeros(h, np.int32)
        _check(lib().rewl_get_geometry(self._h, instance, *[C.byref(x) for x in v], _p(lo), _p(hi)),
               "rewl_get_geometry")
        names = ["N", "nbins", "binw", "emin", "h", "m", "first_slot"]
        d = {n: x.value for n, x in zip(names, v)}
        d["lo"], d["hi"] = lo, hi
        return d

    def get_lng(self, instance=0, normalise=True):
        g = self.geometry[instance]
        out = np.zeros(g["nbins"], np.float64)
        joins = np.zeros(max(g["h"] - 1, 1), np.int32)
        nb = C.c_int32()
        _check(lib().rewl_get_lng(self._h, instance, 0 if normalise else 1, _p(out), len(out),
                                  C.byref(nb), _p(joins)), "rewl_get_lng")
        return out, joins[: g["h"] - 1]

    def get_walker(self, instance, slot):
        g = self.geometry[instance]
        w = slot // g["m"]
        nb = int(g["hi"][w] - g["lo"][w] + 1)
        spins = np.zeros(g["N"], np.int8)
        H = np.zeros(nb, np.uint32)
        lng = np.zeros(nb, np.float64)
        E, att, cid = C.c_int32(), C.c_uint64(), C.c_int32()
        _check(lib().rewl_get_walker(self._h, instance, slot, _p(spins), C.byref(E), _p(H),
                                     _p(lng), C.byref(att), C.byref(cid)), "rewl_get_walker")
        out = {"spins": spins, "E": E.value, "H": H, "lng": lng, "attempts": att.value,
               "config": cid.value}
        if self.params[instance].precision == FP32C:
            hi = np.zeros(nb, np.float32)
            lo = np.zeros(nb, np.float32)
            _check(lib().rewl_get_walker_f32(self._h, instance, slot, _p(hi), _p(lo)),
                   "rewl_get_walker_f32")
            out["lng_hi"], out["lng_lo"] = hi, lo
        return out

    def locate_walker(self, instance, slot):
        """Byte offsets of a walker's energy, H row and ln g row in the
        workspace, and its window's bin count."""
        e, h, l, nb = C.c_size_t(), C.c_size_t(), C.c_size_t(), C.c_int32()
        _check(lib().rewl_locate_walker(self._h, instance, slot, C.byref(e), C.byref(h), C.byref(l),
                                        C.byref(nb)), "rewl_locate_walker")
        return {"energy": e.value, "H": h.value, "lng": l.value, "n_bins": nb.value}

    def get_visited(self, instance, window):
        g = self.geometry[instance]
        nb = int(g["hi"][window] - g["lo"][window] + 1)
        mask = np.zeros(nb, np.uint8)
        _check(lib().rewl_get_visited(self._h, instance, window, _p(mask)), "rewl_get_visited")
        return mask

    def get_exchange_stats(self, instance=0):
        h = self.geometry[instance]["h"]
        t, r, a = (np.zeros(h, np.uint64) for _ in range(3))
        _check(lib().rewl_get_exchange_stats(self._h, instance, _p(t), _p(r), _p(a)),
               "rewl_get_exchange_stats")
        return t, r, a

    def get_schedule(self, instance=0):
        """Per window: phase (0 halving, 1 ln f = 1/t) and the merge index at
        which each WL iteration ended ([h, 64], -1 if not reached)."""
        h = self.geometry[instance]["h"]
        phase = np.zeros(h, np.int32)
        sm = np.zeros((h, 64), np.int64)
        _check(lib().rewl_get_schedule(self._h, instance, _p(phase), _p(sm)), "rewl_get_schedule")
        return phase, sm

    def get_piece(self, instance, slot):
        g = self.geometry[instance]
        w = slot // g["m"]
        out = np.zeros(int(g["hi"][w] - g["lo"][w] + 1), np.float64)
        _check(lib().rewl_get_piece(self._h, instance, slot, _p(out)), "rewl_get_piece")
        return out

    def jackknife(self, instance=0):
        """Jackknife mean and error of the normalised joined ln g over the m
        pieces per window."""
        g = self.geometry[instance]
        mean = np.zeros(g["nbins"], np.float64)
        err = np.zeros(g["nbins"], np.float64)
        nb = C.c_int32()
        _check(lib().rewl_jackknife(self._h, instance, _p(mean), _p(err), len(mean), C.byref(nb)),
               "rewl_jackknife")
        return mean, err

    def jackknife_noalloc(self, instance=0):
        """jackknife() through the allocation-free entry point (its scratch
        is the library's per-GPU device array)."""
        g = self.geometry[instance]
        mean = np.zeros(g["nbins"], np.float64)
        err = np.zeros(g["nbins"], np.float64)
        nb = C.c_int32()
        _check(lib().rewl_jackknife_noalloc(self._h, instance, _p(mean), _p(err), len(mean),
                                            C.byref(nb)), "rewl_jackknife_noalloc")
        return mean, err

    def thermo(self, T, instance=0):
        T = np.ascontiguousarray(T, dtype=np.float64)
        Em = np.zeros(len(T))
        Cv = np.zeros(len(T))
        _check(lib().rewl_thermo(self._h, instance, _p(T), len(T), _p(Em), _p(Cv)), "rewl_thermo")
        return Em, Cv

    def checkpoint(self):
        used = C.c_size_t()
        _check(lib().rewl_checkpoint(self._h, None, 0, C.byref(used)), "rewl_checkpoint")
        buf = np.zeros(used.value, np.uint8)
        _check(lib().rewl_checkpoint(self._h, _p(buf), used.value, C.byref(used)), "rewl_checkpoint")
        return buf

    def restore(self, blob):
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(lib().rewl_restore(self._h, _p(blob), len(blob)), "rewl_restore")

    def run_to_convergence(self, flips, cycles_per_check=64, max_cycles=10 ** 9, use_graph=True):
        """Cycle until every instance is finished; returns cycles enqueued."""
        done = 0
        while done < max_cycles:
            n = min(cycles_per_check, max_cycles - done)
            self.run_cycles(n, flips, use_graph=use_graph)
            done += n
            if self.running() == 0:
                break
        return done
