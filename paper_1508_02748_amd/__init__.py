"""MI355X (gfx950) two-dimensional replica-exchange Wang-Landau sampling.

A thin binding of the C ABI in ``include/rewl.h`` (``librewl.so``): argument
marshalling only.  Every step of the sampling and of the reweighting runs in the
library's HIP kernels; PyTorch provides device memory and the stream.  The
library must have been built (``python -m paper_1508_02748_amd.build``); there
is no fallback.

Method: Valentim et al., "Exploring Replica-Exchange Wang-Landau sampling in
higher-dimensional parameter space" (arXiv:1508.02748), Sec. 2: joint density
of states g(E, M) of the periodic L x L Ising model from Wang-Landau walkers in
overlapping energy windows with configuration exchange (Eq. 1, Eq. 2).
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librewl.so")

REWL_OK, REWL_EINVAL, REWL_ENOMEM, REWL_EDEVICE, REWL_ESTATE, REWL_EOVERFLOW, REWL_ENOTREADY = \
    0, -1, -2, -3, -4, -5, -6
FORM_BATCHED, FORM_PLAIN = 0, 1
SYNC_PROBLEM, SYNC_WINDOW = 0, 1
SPLIT_ENERGY, SPLIT_MAGNETIZATION, SPLIT_BOTH = 0, 1, 2
LAYOUT_DENSE, LAYOUT_BAND, LAYOUT_DENSE_PACKED, LAYOUT_BAND_PACKED = 0, 1, 2, 3
LAYOUTS = (LAYOUT_DENSE, LAYOUT_BAND, LAYOUT_DENSE_PACKED, LAYOUT_BAND_PACKED)
NBUF = 3


class RewlError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"rewl status {status}: {message}")
        self.status = status


class _Problem(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_windows", C.c_int32), ("overlap_num", C.c_int32),
                ("overlap_den", C.c_int32), ("walkers_per_window", C.c_int32), ("k_final", C.c_int32),
                ("flat_num", C.c_int32), ("flat_den", C.c_int32), ("interval", C.c_int64),
                ("seed", C.c_uint64), ("init", C.c_int32), ("stage_sync", C.c_int32),
                ("split", C.c_int32), ("m_windows", C.c_int32), ("m_overlap_num", C.c_int32),
                ("m_overlap_den", C.c_int32), ("reserved", C.c_int32)]


class _Tuning(C.Structure):
    _fields_ = [("form", C.c_int32), ("walkers_per_wg", C.c_int32), ("graph_intervals", C.c_int32),
                ("grid_waves_per_cu", C.c_int32), ("profile", C.c_int32), ("walkers_per_wave", C.c_int32),
                ("table_layout", C.c_int32), ("audit_shift", C.c_int32)]


_lib = None


def lib():
    """Load librewl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1508_02748_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        sig = {
            "rewl_plan_create": ([C.POINTER(_Problem), C.c_int32, C.POINTER(_Tuning), C.POINTER(P)], C.c_int),
            "rewl_plan_destroy": ([P], None),
            "rewl_plan_buffer_sizes": ([P, C.POINTER(C.c_size_t)], C.c_int),
            "rewl_plan_bind": ([P, C.POINTER(P), P], C.c_int),
            "rewl_window_bounds": ([P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
            "rewl_plan_counts": ([P, C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
            "rewl_window_rect": ([P, C.c_int32, C.c_int32] + [C.POINTER(C.c_int32)] * 4, C.c_int),
            "rewl_plan_windows": ([P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "rewl_init": ([P], C.c_int),
            "rewl_run": ([P, C.c_int64], C.c_int),
            "rewl_sweep": ([P, C.c_int64], C.c_int),
            "rewl_reduce_lnf": ([P], C.c_int),
            "rewl_exchange": ([P], C.c_int),
            "rewl_query": ([P, P, P, P], C.c_int),
            "rewl_query_windows": ([P, C.c_int32, P, P, P], C.c_int),
            "rewl_read_walker": ([P, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_size_t, P,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
            "rewl_lnz_forward": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int64,
                                  P, P], C.c_int),
            "rewl_lnz_backward": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int64,
                                   P, P, P, P, P, P, C.c_int32, P], C.c_int),
            "rewl_lnz_grid_workspace_size": ([C.c_int32, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)], C.c_int),
            "rewl_lnz_grid_forward": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64,
                                       P, C.c_int64, P, C.c_size_t, P, P], C.c_int),
            "rewl_lnz_grid_forward_noalloc": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P,
                                               C.c_int64, P, C.c_int64, P, P], C.c_int),
            "rewl_lnz_grid_backward": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64,
                                        P, C.c_int64, P, P, P, C.c_size_t, P, P, P, P, P], C.c_int),
            "rewl_lnz_backward2": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int64,
                                    P, P, P, P, P, P, P, P], C.c_int),
            "rewl_lnz_grid_backward2": ([P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64,
                                         P, C.c_int64, P, P, P, P, P, C.c_size_t, P, P, P, P], C.c_int),
            "rewl_sweep_times": ([P, P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "rewl_set_profile": ([P, C.c_int32], C.c_int),
            "rewl_merge_workspace_size": ([P, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
            "rewl_merge_points": ([P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "rewl_set_tuning": ([P, C.POINTER(_Tuning)], C.c_int),
            "rewl_save_size": ([P, C.POINTER(C.c_size_t)], C.c_int),
            "rewl_save": ([P, P, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
            "rewl_load": ([P, P, C.c_size_t], C.c_int),
            "rewl_merge_lng": ([P, C.c_int32, C.c_int32, P, C.c_size_t, P, P, P, P], C.c_int),
            "rewl_last_error": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != REWL_OK:
        raise RewlError(status, lib().rewl_last_error().decode())


@dataclass
class Problem:
    """One REWL simulation (Sec. 2 of the paper; defaults: 80 % flatness).

    stage_sync: SYNC_PROBLEM (all windows refine ln f together, the paper) or
    SYNC_WINDOW (each window averages its walkers' ln g and refines alone).
    split: SPLIT_ENERGY (windows over E, the paper's runs), SPLIT_MAGNETIZATION
    (windows over M with every energy, the alternative of Sec. 2) or SPLIT_BOTH
    (the rectangles of n_windows energy windows x m_windows magnetization windows
    that hold states, the second alternative of Sec. 2); one per plan."""
    L: int
    n_windows: int = 1
    overlap: tuple = (3, 4)
    walkers_per_window: int = 1
    k_final: int = 20
    flat: tuple = (4, 5)
    interval: int = 10_000
    seed: int = 0
    init: int = 0
    stage_sync: int = SYNC_PROBLEM
    split: int = SPLIT_ENERGY
    m_windows: int = 0
    m_overlap: tuple = (0, 0)

    def _c(self):
        return _Problem(self.L, self.n_windows, self.overlap[0], self.overlap[1], self.walkers_per_window,
                        self.k_final, self.flat[0], self.flat[1], self.interval,
                        self.seed & 0xFFFFFFFFFFFFFFFF, self.init, self.stage_sync, self.split,
                        self.m_windows, self.m_overlap[0], self.m_overlap[1], 0)

    @property
    def N(self):
        return self.L * self.L


@dataclass
class Tuning:
    form: int = FORM_BATCHED
    walkers_per_wg: int = 0
    graph_intervals: int = 0
    grid_waves_per_cu: int = 0
    profile: int = 0
    walkers_per_wave: int = 0
    table_layout: int = LAYOUT_DENSE
    audit_shift: int = 0

    def _c(self):
        return _Tuning(self.form, self.walkers_per_wg, self.graph_intervals, self.grid_waves_per_cu,
                       self.profile, self.walkers_per_wave, self.table_layout, self.audit_shift)


def plan_bytes(problems, table_layout=LAYOUT_DENSE):
    """Device bytes a plan of `problems` needs (all three buffers), without binding it."""
    arr = (_Problem * len(problems))(*[p._c() for p in problems])
    h = C.c_void_p()
    _check(lib().rewl_plan_create(arr, len(problems), C.byref(Tuning(table_layout=table_layout)._c()),
                                  C.byref(h)))
    try:
        sizes = (C.c_size_t * NBUF)()
        _check(lib().rewl_plan_buffer_sizes(h, sizes))
        return int(sum(sizes))
    finally:
        lib().rewl_plan_destroy(h)


class Plan:
    """A batch of REWL problems bound to device buffers allocated by PyTorch."""

    def __init__(self, problems, tuning=None, device="cuda:0", stream=None):
        import torch

        self.problems = list(problems)
        arr = (_Problem * len(self.problems))(*[p._c() for p in self.problems])
        h = C.c_void_p()
        self.tuning = tuning if tuning is not None else Tuning()
        tn = None if tuning is None else C.byref(tuning._c())
        _check(lib().rewl_plan_create(arr, len(self.problems), tn, C.byref(h)))
        self._h = h
        sizes = (C.c_size_t * NBUF)()
        _check(lib().rewl_plan_buffer_sizes(h, sizes))
        self.sizes = list(sizes)
        self.device = torch.device(device)
        # uint8 buffers; the caching allocator returns >= 256-byte aligned blocks
        self.buffers = [torch.empty(max(1, s), dtype=torch.uint8, device=self.device) for s in self.sizes]
        # a stream of its own (default priority): graph capture is not possible on
        # the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        torch.cuda.current_stream(self.device).synchronize()
        ptrs = (C.c_void_p * NBUF)(*[b.data_ptr() for b in self.buffers])
        _check(lib().rewl_plan_bind(h, ptrs, C.c_void_p(self.stream.cuda_stream)))
        npb = C.c_int32()
        nw = C.c_int64()
        _check(lib().rewl_plan_counts(h, C.byref(npb), C.byref(nw)))
        self.n_problems, self.n_walkers = npb.value, nw.value
        self.windows_of = []
        for i in range(self.n_problems):
            k = C.c_int32()
            _check(lib().rewl_plan_windows(h, i, C.byref(k)))
            self.windows_of.append(k.value)

    def close(self):
        """Destroy the plan after its stream has drained, then release the buffers.

        The buffers come from the caching allocator on the current stream but
        are written on ``self.stream``; rewl_plan_destroy waits for that stream,
        so no kernel of the plan can still touch a buffer once it is handed
        back to the allocator."""
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rewl_plan_destroy(h)
        self._h = None
        st = getattr(self, "stream", None)
        if st is not None:
            st.synchronize()
        self.buffers = []

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: torch may already be gone
            pass

    # ----- the paper's operations
    def init(self):
        _check(lib().rewl_init(self._h))

    def run(self, n_intervals):
        _check(lib().rewl_run(self._h, int(n_intervals)))

    def sweep(self, n_trials):
        _check(lib().rewl_sweep(self._h, int(n_trials)))

    def reduce_lnf(self):
        _check(lib().rewl_reduce_lnf(self._h))

    def exchange(self):
        _check(lib().rewl_exchange(self._h))

    def query(self):
        n = self.n_problems
        st = np.zeros(n, np.int32)
        dn = np.zeros(n, np.int32)
        tr = np.zeros(n, np.int64)
        _check(lib().rewl_query(self._h, st.ctypes.data, dn.ctypes.data, tr.ctypes.data))
        return {"stage": st, "done": dn.astype(bool), "trials": tr}

    def query_windows(self, prob=0):
        """Per window of problem prob: stage, done, trials per walker."""
        n = self.windows_of[prob]
        st = np.zeros(n, np.int32)
        dn = np.zeros(n, np.int32)
        tr = np.zeros(n, np.int64)
        _check(lib().rewl_query_windows(self._h, prob, st.ctypes.data, dn.ctypes.data, tr.ctypes.data))
        return {"stage": st, "done": dn.astype(bool), "trials": tr}

    def set_tuning(self, tuning):
        self.tuning = tuning
        _check(lib().rewl_set_tuning(self._h, C.byref(tuning._c())))

    def save(self):
        """Checkpoint: bytes holding the problems and the whole device state."""
        n = C.c_size_t()
        _check(lib().rewl_save_size(self._h, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        used = C.c_size_t()
        _check(lib().rewl_save(self._h, buf.ctypes.data, n.value, C.byref(used)))
        return buf[:used.value].tobytes()

    def load(self, blob):
        arr = np.frombuffer(blob, np.uint8)
        _check(lib().rewl_load(self._h, arr.ctypes.data, arr.size))

    def set_profile(self, on):
        _check(lib().rewl_set_profile(self._h, 1 if on else 0))

    def sweep_times(self):
        """Durations (ms) of the sweep kernels of the last profiled rewl_run."""
        cap = 4096
        buf = np.zeros(cap, np.float32)
        n = C.c_int32()
        _check(lib().rewl_sweep_times(self._h, buf.ctypes.data, cap, C.byref(n)))
        return buf[:min(cap, n.value)].astype(np.float64)

    def merge(self, prob=0, norm="ground", with_err=False):
        """Joint ln g(E, M) (device, float64, (N+1) x (N+1)), marginal ln g(E), matching points
        (rewl_merge_points: E_mat list, M_mat list for magnetization windows, per-window E_mat
        then M_mat for windows in both coordinates) [, error bars of the joint table (device,
        NaN below two walkers)]."""
        import torch
        p = self.problems[prob]
        nb = C.c_size_t()
        _check(lib().rewl_merge_workspace_size(self._h, prob, C.byref(nb)))
        npts = C.c_int32()
        _check(lib().rewl_merge_points(self._h, prob, C.byref(npts)))
        ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device=self.device)
        joint = torch.empty((p.N + 1, p.N + 1), dtype=torch.float64, device=self.device)
        marg = torch.empty(p.N + 1, dtype=torch.float64, device=self.device)
        emat = torch.zeros(max(1, npts.value), dtype=torch.int32, device=self.device)
        err = torch.empty_like(joint) if with_err else None
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().rewl_merge_lng(self._h, prob, {"ground": 0, "sum": 1}[norm], C.c_void_p(ws.data_ptr()),
                                    nb.value, C.c_void_p(joint.data_ptr()), C.c_void_p(marg.data_ptr()),
                                    C.c_void_p(emat.data_ptr()), _ptr(err)))
        em = [int(x) for x in emat.cpu()[:npts.value]]
        return (joint, marg, em, err) if with_err else (joint, marg, em)

    def window(self, prob, w):
        lo, hi = C.c_int32(), C.c_int32()
        _check(lib().rewl_window_bounds(self._h, prob, w, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def window_rect(self, prob, w):
        """(e_lo, e_hi, m_lo, m_hi) of window w of problem prob."""
        r = [C.c_int32() for _ in range(4)]
        _check(lib().rewl_window_rect(self._h, prob, w, *[C.byref(x) for x in r]))
        return tuple(x.value for x in r)

    def walker(self, prob, w, a, tables=True):
        """Walker a of window w of problem prob: lng / H tables over the window's rectangle
        (rows e - e_lo, columns m - m_lo), spins, e, m, t."""
        p = self.problems[prob]
        lo, hi = self.window(prob, w)
        elo, ehi, mlo, mhi = self.window_rect(prob, w)
        nb = (ehi - elo + 1) * (mhi - mlo + 1)
        lng = np.zeros(nb, np.int64) if tables else None
        H = np.zeros(nb, np.uint64) if tables else None
        sp = np.zeros(p.N, np.int8)
        e, m, t = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().rewl_read_walker(self._h, prob, w, a,
                                      lng.ctypes.data if tables else None,
                                      H.ctypes.data if tables else None, nb if tables else 0,
                                      sp.ctypes.data, C.byref(e), C.byref(m), C.byref(t)))
        shape = (ehi - elo + 1, mhi - mlo + 1)
        return {"lng": None if lng is None else lng.reshape(shape),
                "H": None if H is None else H.reshape(shape),
                "spins": sp.reshape(p.L, p.L), "e": e.value, "m": m.value, "t": t.value,
                "lo": lo, "hi": hi}


# ------------------------------------------------------------------ reweighting
def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _geom(lng, N, e0, m0):
    nE, nM = lng.shape
    return N, e0, nE, m0, nM


def lnz_forward(lng, beta, h, N, e0=0, m0=0):
    """ln Z(beta, h) on the device for a float64 joint ln g table (-inf = unvisited)."""
    import torch
    assert lng.dtype == torch.float64 and lng.is_cuda and lng.is_contiguous()
    beta = beta.contiguous()
    h = h.contiguous()
    out = torch.empty_like(beta)
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_forward(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta), _ptr(h), beta.numel(),
                                  _ptr(out), C.c_void_p(st)))
    return out


def lnz_moments(lng, beta, h, lnz, N, e0=0, m0=0):
    """(G, 5) float64: <M>, <U>, Var(U), Var(M), Cov(U, M) with U = -E + h M."""
    import torch
    mom = torch.empty((beta.numel(), 5), dtype=torch.float64, device=lng.device)
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_backward(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta.contiguous()),
                                   _ptr(h.contiguous()), beta.numel(), _ptr(lnz.contiguous()), None, None,
                                   None, None, _ptr(mom), 2, C.c_void_p(st)))
    return mom


def _lnz_grads(lng, beta, h, lnz, grad_out, N, e0, m0, want_lng):
    import torch
    gb = torch.empty_like(beta)
    gh = torch.empty_like(beta)
    gl = torch.empty_like(lng) if want_lng else None
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_backward(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta), _ptr(h), beta.numel(),
                                   _ptr(lnz), _ptr(grad_out.contiguous()), _ptr(gb), _ptr(gh), _ptr(gl),
                                   None, 1, C.c_void_p(st)))
    return gb, gh, gl


def lnz_second(lng, beta, h, lnz, grad_out, up_beta, up_h, N, e0=0, m0=0):
    """Backward of (grad_beta, grad_h) = first-order backward of ln Z: (d grad_out, d beta, d h), each (G,)."""
    import torch
    d_go, d_b, d_h = (torch.empty_like(beta) for _ in range(3))
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_backward2(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta.contiguous()),
                                    _ptr(h.contiguous()), beta.numel(), _ptr(lnz.contiguous()),
                                    _ptr(None if grad_out is None else grad_out.contiguous()),
                                    _ptr(None if up_beta is None else up_beta.contiguous()),
                                    _ptr(None if up_h is None else up_h.contiguous()),
                                    _ptr(d_go), _ptr(d_b), _ptr(d_h), C.c_void_p(st)))
    return d_go, d_b, d_h


def _grid_ws(lng, nB, nH):
    import torch
    nb = C.c_size_t()
    _check(lib().rewl_lnz_grid_workspace_size(lng.shape[1], nB, nH, C.byref(nb)))
    return torch.empty(max(1, nb.value), dtype=torch.uint8, device=lng.device), nb.value


def lnz_grid_forward(lng, beta, h, N, e0=0, m0=0):
    """ln Z on the tensor-product grid beta (nB) x h (nH): (nB, nH) float64 on the device."""
    import torch
    assert lng.dtype == torch.float64 and lng.is_cuda and lng.is_contiguous()
    beta = beta.contiguous()
    h = h.contiguous()
    out = torch.empty((beta.numel(), h.numel()), dtype=torch.float64, device=lng.device)
    ws, nb = _grid_ws(lng, beta.numel(), h.numel())
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_grid_forward(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta), beta.numel(), _ptr(h),
                                       h.numel(), _ptr(ws), nb, _ptr(out), C.c_void_p(st)))
    return out


def lnz_grid_forward_noalloc(lng, beta, h, out, N, e0=0, m0=0):
    """ln Z on the grid into the caller's `out` (nB, nH) with no device allocation (the library's
    fixed scratch array); every tensor must already be contiguous float64 on the device."""
    import torch
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_grid_forward_noalloc(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta), beta.numel(),
                                               _ptr(h), h.numel(), _ptr(out), C.c_void_p(st)))
    return out


def lnz_grid_backward(lng, beta, h, lnz, grad_out, N, e0=0, m0=0, want_grads=True, want_lng=False,
                      want_mom=False):
    """(grad_beta (nB), grad_h (nH), grad_lng or None, moments (nB, nH, 5) or None) on the device."""
    import torch
    nB, nH = beta.numel(), h.numel()
    gb = torch.empty(nB, dtype=torch.float64, device=lng.device) if want_grads else None
    gh = torch.empty(nH, dtype=torch.float64, device=lng.device) if want_grads else None
    gl = torch.empty_like(lng) if want_lng else None
    mom = torch.empty((nB, nH, 5), dtype=torch.float64, device=lng.device) if want_mom else None
    go = None if grad_out is None else grad_out.contiguous()
    ws, nb = _grid_ws(lng, nB, nH)
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_grid_backward(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta.contiguous()), nB,
                                        _ptr(h.contiguous()), nH, _ptr(lnz.contiguous()), _ptr(go), _ptr(ws), nb,
                                        _ptr(gb), _ptr(gh), _ptr(gl), _ptr(mom), C.c_void_p(st)))
    return gb, gh, gl, mom


def lnz_grid_second(lng, beta, h, lnz, grad_out, up_beta, up_h, N, e0=0, m0=0):
    """Second order on a grid: (d grad_out (nB, nH), d beta (nB), d h (nH)) on the device."""
    import torch
    nB, nH = beta.numel(), h.numel()
    d_go = torch.empty((nB, nH), dtype=torch.float64, device=lng.device)
    d_b = torch.empty(nB, dtype=torch.float64, device=lng.device)
    d_h = torch.empty(nH, dtype=torch.float64, device=lng.device)
    ws, nb = _grid_ws(lng, nB, nH)
    st = torch.cuda.current_stream(lng.device).cuda_stream
    _check(lib().rewl_lnz_grid_backward2(_ptr(lng), *_geom(lng, N, e0, m0), _ptr(beta.contiguous()), nB,
                                         _ptr(h.contiguous()), nH, _ptr(lnz.contiguous()),
                                         _ptr(None if grad_out is None else grad_out.contiguous()),
                                         _ptr(None if up_beta is None else up_beta.contiguous()),
                                         _ptr(None if up_h is None else up_h.contiguous()),
                                         _ptr(ws), nb, _ptr(d_go), _ptr(d_b), _ptr(d_h), C.c_void_p(st)))
    return d_go, d_b, d_h


def _no_lng_second_order(ctx, name):
    """Second derivatives through ln g are not provided: refuse instead of dropping them."""
    import torch
    if ctx.needs_input_grad[0] and torch.is_grad_enabled():
        raise RuntimeError(f"{name}: second derivatives with respect to ln g are not implemented "
                           "(differentiate twice with respect to beta and h only)")


def _torch_functions():
    import torch

    class _LnZBackward(torch.autograd.Function):
        """(grad_out, beta, h) -> (grad_beta, grad_h) of ln Z, differentiable once more."""

        @staticmethod
        def forward(ctx, grad_out, beta, h, lng, lnz, N, e0, m0):
            gb, gh, _ = _lnz_grads(lng, beta, h, lnz, grad_out, N, e0, m0, False)
            ctx.save_for_backward(grad_out, beta, h, lng, lnz)
            ctx.geo = (N, e0, m0)
            return gb, gh

        @staticmethod
        def backward(ctx, a, b):
            grad_out, beta, h, lng, lnz = ctx.saved_tensors
            N, e0, m0 = ctx.geo
            d_go, d_beta, d_h = lnz_second(lng, beta.detach(), h.detach(), lnz, grad_out.detach(), a, b, N, e0, m0)
            return d_go, d_beta, d_h, None, None, None, None, None

    class LnZ(torch.autograd.Function):
        """ln Z(beta, h) = logsumexp over (E, M) of ln g - beta E + beta h M.

        Gradients: d/d beta = <-E + h M>, d/d h = beta <M>, d/d ln g = p(E, M);
        second derivatives (through a second Function) give Var(E - h M),
        beta^2 Var(M) and the mixed term, i.e. specific heat and susceptibility."""

        @staticmethod
        def forward(ctx, lng, beta, h, N, e0=0, m0=0):
            lnz = lnz_forward(lng, beta, h, N, e0, m0)
            ctx.save_for_backward(lng, beta, h, lnz)
            ctx.geo = (N, e0, m0)
            return lnz

        @staticmethod
        def backward(ctx, grad_out):
            lng, beta, h, lnz = ctx.saved_tensors
            N, e0, m0 = ctx.geo
            _no_lng_second_order(ctx, "LnZ")
            g_lng = None
            if ctx.needs_input_grad[0]:
                _, _, g_lng = _lnz_grads(lng, beta.detach(), h.detach(), lnz, grad_out.detach(), N, e0, m0, True)
            gb, gh = _LnZBackward.apply(grad_out, beta, h, lng.detach(), lnz.detach(), N, e0, m0)
            return g_lng, gb, gh, None, None, None

    class _LnZGridBackward(torch.autograd.Function):
        """(grad_out (nB, nH), beta, h) -> (grad_beta (nB), grad_h (nH)), differentiable once more."""

        @staticmethod
        def forward(ctx, grad_out, beta, h, lng, lnz, N, e0, m0):
            gb, gh, _, _ = lnz_grid_backward(lng, beta, h, lnz, grad_out, N, e0, m0)
            ctx.save_for_backward(grad_out, beta, h, lng, lnz)
            ctx.geo = (N, e0, m0)
            return gb, gh

        @staticmethod
        def backward(ctx, a, b):
            grad_out, beta, h, lng, lnz = ctx.saved_tensors
            N, e0, m0 = ctx.geo
            d_go, d_beta, d_h = lnz_grid_second(lng, beta.detach(), h.detach(), lnz, grad_out.detach(), a, b, N,
                                                e0, m0)
            return d_go, d_beta, d_h, None, None, None, None, None

    class LnZGrid(torch.autograd.Function):
        """ln Z on a tensor-product grid: (lng, beta (nB), h (nH), N) -> (nB, nH).

        Same quantity and derivatives as LnZ at the points (beta_i, h_j),
        computed through the factorisation over M columns."""

        @staticmethod
        def forward(ctx, lng, beta, h, N, e0=0, m0=0):
            lnz = lnz_grid_forward(lng, beta, h, N, e0, m0)
            ctx.save_for_backward(lng, beta, h, lnz)
            ctx.geo = (N, e0, m0)
            return lnz

        @staticmethod
        def backward(ctx, grad_out):
            lng, beta, h, lnz = ctx.saved_tensors
            N, e0, m0 = ctx.geo
            _no_lng_second_order(ctx, "LnZGrid")
            g_lng = None
            if ctx.needs_input_grad[0]:
                _, _, g_lng, _ = lnz_grid_backward(lng, beta.detach(), h.detach(), lnz, grad_out.detach(), N, e0,
                                                   m0, want_grads=False, want_lng=True)
            gb, gh = _LnZGridBackward.apply(grad_out, beta, h, lng.detach(), lnz.detach(), N, e0, m0)
            return g_lng, gb, gh, None, None, None

    return LnZ, LnZGrid


_LnZ = None


def LnZ():
    """The torch.autograd.Function computing ln Z(beta, h) from a joint ln g."""
    global _LnZ
    if _LnZ is None:
        _LnZ = _torch_functions()
    return _LnZ[0]


def LnZGrid():
    """The torch.autograd.Function computing ln Z on a tensor-product (beta, h) grid."""
    global _LnZ
    if _LnZ is None:
        _LnZ = _torch_functions()
    return _LnZ[1]
