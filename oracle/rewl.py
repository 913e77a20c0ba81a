"""ctypes wrapper of the C oracle (test infrastructure only).

The oracle runs one REWL simulation per ``OracleREWL`` object, exactly as the
paper describes it (Sec. 2): independent WL walkers per overlapping energy
window, each with its own ln g(E,M) and H(E,M); flatness checks; a global
f -> sqrt(f) refinement once every walker is flat; configuration exchange
between adjacent windows with Eq. (2).  With ``sync=1`` each window refines
alone once its own walkers are flat, averaging their ln g first (a common
REWL form the paper cites; not the paper's own runs).  Tables are returned as numpy arrays of
shape (hi - lo + 1, N + 1) indexed by (e - lo, m), with e = (E + 2N)/4 and
m = (M + N)/2.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.or_philox.argtypes = [C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32),
                                C.POINTER(C.c_uint32)]
        L.or_philox.restype = None
        L.or_exp_spec.argtypes = [C.c_double]
        L.or_exp_spec.restype = C.c_double
        L.or_uniform.argtypes = [C.c_uint32]
        L.or_uniform.restype = C.c_double
        L.or_accept.argtypes = [C.c_int64, C.c_uint32, C.c_int]
        L.or_accept.restype = C.c_int
        L.or_window.argtypes = [C.c_int] * 5 + [C.POINTER(C.c_int)] * 2
        L.or_window.restype = None
        L.or_energy.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                C.POINTER(C.c_int)]
        L.or_energy.restype = None
        L.or_create.argtypes = [C.c_int] * 8 + [C.c_int64, C.c_uint64, C.c_int]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_destroy.restype = None
        L.or_init.argtypes = [C.c_void_p, C.c_int64]
        L.or_init.restype = C.c_int
        L.or_sweep.argtypes = [C.c_void_p, C.c_int64]
        L.or_sweep.restype = None
        L.or_is_flat.argtypes = [C.c_void_p, C.c_int]
        L.or_is_flat.restype = C.c_int
        L.or_exchange.argtypes = [C.c_void_p, C.c_int64]
        L.or_exchange.restype = C.c_int64
        L.or_boundary.argtypes = [C.c_void_p]
        L.or_boundary.restype = None
        L.or_run.argtypes = [C.c_void_p, C.c_int64]
        L.or_run.restype = C.c_int64
        L.or_info.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                              C.POINTER(C.c_int64), C.POINTER(C.c_int)]
        L.or_info.restype = None
        L.or_window_of.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int)]
        L.or_window_of.restype = None
        L.or_bins_of_walker.argtypes = [C.c_void_p, C.c_int]
        L.or_bins_of_walker.restype = C.c_int64
        L.or_get_walker.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int)]
        L.or_get_walker.restype = None
        L.or_set_walker.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.or_set_walker.restype = None
        L.or_set_stage.argtypes = [C.c_void_p, C.c_int]
        L.or_set_stage.restype = None
        L.or_set_sync.argtypes = [C.c_void_p, C.c_int]
        L.or_set_sync.restype = C.c_int
        L.or_set_split.argtypes = [C.c_void_p, C.c_int]
        L.or_set_split.restype = C.c_int
        L.or_create_2d.argtypes = [C.c_int] * 11 + [C.c_int64, C.c_uint64, C.c_int]
        L.or_create_2d.restype = C.c_void_p
        L.or_window_rect.argtypes = [C.c_void_p, C.c_int] + [C.POINTER(C.c_int)] * 4
        L.or_window_rect.restype = None
        L.or_n_windows.argtypes = [C.c_void_p]
        L.or_n_windows.restype = C.c_int
        L.or_realizable.argtypes = [C.c_int] * 3
        L.or_realizable.restype = C.c_int
        L.or_set_hist.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_set_hist.restype = None
        L.or_draw_matching.argtypes = [C.c_uint64, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.or_draw_matching.restype = None
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = C.c_int
        L.or_window_state.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
        L.or_window_state.restype = None
        _lib = L
    return _lib


# ---------------------------------------------------------------- primitives
def philox(key, ctr):
    """Philox4x32-10 block for 64-bit key and 4-word counter -> 4 uint32."""
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (C.c_uint32 * 4)()
    lib().or_philox(key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF, c, o)
    return [int(x) for x in o]


def exp_spec(x):
    return lib().or_exp_spec(float(x))


def uniform(word):
    return lib().or_uniform(int(word))


def accept(delta, u_word, K):
    return bool(lib().or_accept(int(delta), int(u_word), int(K)))


def window(N, n, p, q, i):
    lo, hi = C.c_int(), C.c_int()
    lib().or_window(N, n, p, q, i, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def realizable(L, e, m):
    """Whether bin (e, m) holds a state, by the closed-form support (or_realizable)."""
    return bool(lib().or_realizable(int(L), int(e), int(m)))


def set_threads(n):
    """Host threads for the oracle's walker loops (0 = unchanged); returns the count in effect."""
    return int(lib().or_set_threads(int(n)))


def draw_matching(seed, r, w, W):
    """The exchange matching of round r for the window pair with lower window w: walker a of
    the lower window meets walker pi[a] of the upper one."""
    pi = (C.c_int * W)()
    lib().or_draw_matching(seed & 0xFFFFFFFFFFFFFFFF, int(r), int(w), int(W), pi)
    return tuple(pi)


def energy(spins, L):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    E, M = C.c_int(), C.c_int()
    lib().or_energy(s.ctypes.data, L, C.byref(E), C.byref(M))
    return E.value, M.value


# ---------------------------------------------------------------- simulation
class OracleREWL:
    """One 2D-REWL simulation (all windows and walkers of one problem).

    split = 0: the windows split the energy range, every window keeping the
    full magnetization range (the paper's runs, Sec. 3); split = 1: they split
    the magnetization range and keep every energy (the alternative named at
    the end of Sec. 2)."""

    def __init__(self, L, n_windows=1, overlap=(3, 4), walkers_per_window=1,
                 k_final=16, flat=(4, 5), interval=10_000, seed=0, init=0, sync=0, split=0,
                 m_windows=None):
        self.L, self.N = L, L * L
        self.W = walkers_per_window
        self.K, self.X, self.seed = k_final, interval, seed
        self.overlap, self.flat = overlap, flat
        if split == 2:
            # rectangles: n_windows x overlap in e, m_windows = (n, (p, q)) in m;
            # only rectangles that hold states are kept
            n_m, (pm, qm) = m_windows
            h = lib().or_create_2d(L, n_windows, overlap[0], overlap[1], n_m, pm, qm,
                                   walkers_per_window, k_final, flat[0], flat[1],
                                   interval, seed & 0xFFFFFFFFFFFFFFFF, init)
        else:
            h = lib().or_create(L, n_windows, overlap[0], overlap[1],
                                walkers_per_window, k_final, flat[0], flat[1],
                                interval, seed & 0xFFFFFFFFFFFFFFFF, init)
        if not h:
            raise ValueError("invalid REWL problem")
        self._h = h
        self.n_windows = lib().or_n_windows(h)
        self.sync = sync
        if lib().or_set_sync(h, sync) != 0:
            raise ValueError("sync must be 0 (all windows together) or 1 (per window)")
        self.split = split
        if split != 2 and lib().or_set_split(h, split) != 0:
            raise ValueError("split must be 0 (energy), 1 (magnetization) or 2 (both)")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    @property
    def n_walkers(self):
        return self.n_windows * self.W

    def init(self, entry_cap=1 << 40):
        if lib().or_init(self._h, entry_cap) != 0:
            raise RuntimeError("entry walk exceeded its cap")

    def sweep(self, n):
        lib().or_sweep(self._h, n)

    def boundary(self):
        lib().or_boundary(self._h)

    def exchange(self, r):
        return lib().or_exchange(self._h, r)

    def run(self, n_intervals):
        return lib().or_run(self._h, n_intervals)

    def run_to_end(self, max_intervals=1 << 40):
        return self.run(max_intervals)

    def is_flat(self, g):
        return bool(lib().or_is_flat(self._h, g))

    def info(self):
        s, d, r, n = C.c_int(), C.c_int(), C.c_int64(), C.c_int()
        lib().or_info(self._h, C.byref(s), C.byref(d), C.byref(r), C.byref(n))
        return {"stage": s.value, "done": bool(d.value), "boundaries": r.value}

    def window(self, w):
        lo, hi = C.c_int(), C.c_int()
        lib().or_window_of(self._h, w, C.byref(lo), C.byref(hi))
        return lo.value, hi.value

    def window_rect(self, w):
        """(e_lo, e_hi, m_lo, m_hi) of window w."""
        r = [C.c_int() for _ in range(4)]
        lib().or_window_rect(self._h, w, *[C.byref(x) for x in r])
        return tuple(x.value for x in r)

    def window_state(self, w):
        """(stage, done) of window w."""
        s, d = C.c_int(), C.c_int()
        lib().or_window_state(self._h, w, C.byref(s), C.byref(d))
        return s.value, bool(d.value)

    def walker(self, g, tables=True):
        """State of walker g = w * W + a as a dict of numpy arrays / ints."""
        w = g // self.W
        lo, hi = self.window(w)
        elo, ehi, mlo, mhi = self.window_rect(w)
        # rows e - e_lo, columns m - m_lo of the window's rectangle
        shape = (ehi - elo + 1, mhi - mlo + 1)
        lng = np.zeros(shape, np.int64) if tables else None
        H = np.zeros(shape, np.uint64) if tables else None
        sp = np.zeros(self.N, np.int8)
        e, m, fl = C.c_int(), C.c_int(), C.c_int()
        t, te = C.c_int64(), C.c_int64()
        lib().or_get_walker(self._h, g,
                            lng.ctypes.data if tables else None,
                            H.ctypes.data if tables else None,
                            sp.ctypes.data, C.byref(e), C.byref(m), C.byref(t),
                            C.byref(te), C.byref(fl))
        return {"lng": lng, "H": H, "spins": sp.reshape(self.L, self.L),
                "e": e.value, "m": m.value, "t": t.value, "te": te.value,
                "flag": fl.value, "lo": lo, "hi": hi}

    def set_hist(self, g, H):
        """Overwrite walker g's visit histogram (window-table shape, uint64)."""
        a = np.ascontiguousarray(H, np.uint64)
        lib().or_set_hist(self._h, g, a.ctypes.data)

    def set_stage(self, s):
        lib().or_set_stage(self._h, s)

    def set_walker(self, g, lng=None, spins=None):
        la = None if lng is None else np.ascontiguousarray(lng, np.int64)
        sa = None if spins is None else np.ascontiguousarray(spins, np.int8).reshape(-1)
        lib().or_set_walker(self._h, g, None if la is None else la.ctypes.data,
                            None if sa is None else sa.ctypes.data)
