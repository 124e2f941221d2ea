"""Python binding of libwpcd (include/wpcd.h): argument marshalling only.

Every step of the hot path runs inside the library (host FP64 C++ and gfx950 HIP kernels).
PyTorch provides device memory (a caching-allocator-backed ``wp_allocator``) and streams
(``torch.cuda.current_stream()``). If ``libwpcd.so`` is missing this module raises on import:
there is no fallback.

The module-level functions carry the names of the C entry points:
``wp_lattice_build``, ``twobody_pseudostates``, ``perm_matrix_build``, ``perm_matrix_export``,
``faddeev_solve``, ``amplitude`` and the ``faddeev_batch_*`` step API. ``Lattice`` wraps them.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwpcd.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1404_5253_amd/build.py`")
_lib = C.CDLL(LIB_PATH)
C = C   # ctypes, re-exported for callers that pass raw stream handles

WP_OK, WP_EINVAL, WP_ENOMEM, WP_EDEVICE, WP_ENOTREADY, WP_ENOCONV, WP_EBUDGET, WP_EINTERNAL = range(8)
WP_P_FP64, WP_P_FP32 = 0, 1
WP_SOLVE_FP64, WP_SOLVE_MIXED, WP_SOLVE_MIXED_SPLIT = 0, 1, 2
WP_WEIGHTS_UNIT, WP_WEIGHTS_ENERGY = 0, 1
WEIGHTS = {"unit": WP_WEIGHTS_UNIT, "energy": WP_WEIGHTS_ENERGY}
SOLVE_MODES = {"fp64": WP_SOLVE_FP64, "mixed": WP_SOLVE_MIXED, "mixed_split": WP_SOLVE_MIXED_SPLIT}
H2M = 41.471


class WpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wpcd status {status}: {msg}")
        self.status = status


class _Alloc(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("release", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


class _LatDesc(C.Structure):
    _fields_ = [("M", C.c_int), ("N", C.c_int), ("grid_kind", C.c_int),
                ("alpha", C.c_double), ("p_max", C.c_double), ("q_max", C.c_double),
                ("p_edges", C.POINTER(C.c_double)), ("q_edges", C.POINTER(C.c_double)),
                ("two_J", C.c_int), ("parity", C.c_int), ("two_T", C.c_int), ("j_max", C.c_int),
                ("swave_only", C.c_int), ("n_x", C.c_int), ("n_phi", C.c_int),
                ("hbar2_over_m", C.c_double)]


class _PotDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("beta", C.c_double), ("lambda_", C.c_double),
                ("V_R", C.c_double), ("mu_R", C.c_double), ("V_A", C.c_double), ("mu_A", C.c_double),
                ("singlet_ratio", C.c_double), ("target_BE", C.c_double), ("tune", C.c_int)]


class _PermStats(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("blocks", C.c_int64), ("candidates", C.c_int64),
                ("bytes", C.c_int64), ("device_ms", C.c_double)]


class _SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("tol", C.c_double), ("accept", C.c_double),
                ("max_iter", C.c_int), ("refine_every", C.c_int), ("graph", C.c_int), ("step_tile", C.c_int),
                ("spmm_cols", C.c_int), ("breakup", C.c_int)]


WP_STEP_AUTO, WP_STEP_MFMA8, WP_STEP_MFMA16, WP_STEP_VALU, WP_STEP_ROWS = 0, 1, 2, 3, 4
STEP_TILES = {"auto": WP_STEP_AUTO, "mfma8": WP_STEP_MFMA8, "mfma16": WP_STEP_MFMA16, "valu": WP_STEP_VALU,
              "rows": WP_STEP_ROWS}


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)

_SIGS = {
    "wp_last_error": (C.c_char_p, []),
    "wp_lattice_build": (C.c_int, [C.POINTER(_LatDesc), C.POINTER(_Alloc), C.POINTER(_P)]),
    "wp_lattice_channels": (C.c_int, [_P, _I, _I]),
    "wp_lattice_info": (C.c_int, [_P, _I, _I]),
    "wp_lattice_weights": (C.c_int, [_P, C.c_int]),
    "wp_lattice_edges": (C.c_int, [_P, _D, _D]),
    "wp_lattice_pseudostates": (C.c_int, [_P, C.c_int, _I, _D, _D, _D]),
    "wp_lattice_resolvent": (C.c_int, [_P, C.c_double, C.c_int, _D]),
    "wp_lattice_resolvent_noalloc": (C.c_int, [_P, C.c_double, C.c_int, _D]),
    "wp_lattice_free": (None, [_P]),
    "twobody_pseudostates": (C.c_int, [_P, C.POINTER(_PotDesc), _D, _D]),
    "perm_matrix_build": (C.c_int, [_P, C.c_int, _P, C.POINTER(_PermStats)]),
    "perm_matrix_export": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _D]),
    "faddeev_solve": (C.c_int, [_P, C.c_int, _D, C.POINTER(_SolveOpts), _P, C.POINTER(_P)]),
    "amplitude": (C.c_int, [_P, C.c_int, _I, _D, _D, _D, _D, _D, _I]),
    "faddeev_series": (C.c_int, [_P, C.c_int, C.c_int, _I, _D]),
    "faddeev_breakup": (C.c_int, [_P, C.c_int, C.c_int, _I, _I, _D]),
    "wp_solution_free": (None, [_P]),
    "nd_sigma_rep": (C.c_int, [C.c_int, C.c_int, _I, _I, _D, _I, _I, _D]),
    "nd_eigenphases": (C.c_int, [C.c_int, _D, _D, _D]),
    "nd_elastic_observables": (C.c_int, [C.c_int, _I, _I, _I, _I, _D, C.c_double, C.c_int, _D, _D, _D]),
    "faddeev_batch_create": (C.c_int, [_P, C.c_int, C.c_size_t, C.POINTER(_SolveOpts), C.POINTER(_P)]),
    "faddeev_batch_admit": (C.c_int, [_P, C.c_double, _I]),
    "faddeev_batch_admit_many": (C.c_int, [_P, C.c_int, _D, _P, _I, _I]),
    "faddeev_batch_slot_bytes": (C.c_int, [_P, C.POINTER(_SolveOpts), C.POINTER(C.c_size_t)]),
    "faddeev_batch_step": (C.c_int, [_P, _P, C.c_int, _I, _I]),
    "faddeev_batch_take": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "faddeev_batch_live": (C.c_int, [_P, _I]),
    "faddeev_batch_free": (None, [_P]),
    "wp_profile_enable": (C.c_int, [C.c_int]),
    "wp_profile_read": (C.c_int, [C.c_int, _I, C.c_char_p, C.POINTER(C.c_int64), _D]),
    "wp_profile_reset": (C.c_int, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(st):
    if st != WP_OK:
        raise WpError(st, _lib.wp_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _iarr(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int32))
    return a, a.ctypes.data_as(_I)


def _carr(S):
    """Complex matrix -> contiguous re/im doubles."""
    a = np.ascontiguousarray(np.asarray(S, dtype=np.complex128))
    return a, a.ctypes.data_as(_D)


def open_channels(channels):
    """(lam, 2I) of a lattice's open elastic channels (deuteron (l, s, j) = (0, 1, 1)), in the order
    of the amplitude matrices."""
    return [(c[3], c[4]) for c in channels if c[0] == 0 and c[1] == 1 and c[2] == 1]


def nd_sigma_rep(two_J, chans, S):
    """(lam, 2 Sigma) channels and S in the channel-spin representation."""
    n = len(chans)
    lam, pl = _iarr([c[0] for c in chans])
    tI, pI = _iarr([c[1] for c in chans])
    Sa, pS = _carr(S)
    ls, pls = _iarr(np.zeros(n))
    ts, pts = _iarr(np.zeros(n))
    out = np.zeros((n, n), dtype=np.complex128)
    _check(_lib.nd_sigma_rep(two_J, n, pl, pI, pS, pls, pts, out.ctypes.data_as(_D)))
    return list(zip(ls.tolist(), ts.tolist())), out


def nd_eigenphases(S):
    """Eigenphases (radians) and the real orthogonal O with S = O diag(exp(2 i delta)) O^T."""
    Sa, pS = _carr(S)
    n = Sa.shape[0]
    d = np.zeros(n)
    O = np.zeros((n, n))
    _check(_lib.nd_eigenphases(n, pS, _dptr(d), _dptr(O)))
    return d, O


def nd_elastic_observables(blocks, k, thetas):
    """dsigma/dOmega (fm^2/sr) and A_y at the angles thetas (radians) from blocks = [(two_J, chans, S)]
    with chans the (lam, 2I) of S's rows (open_channels of the block's lattice)."""
    tJ, ptJ = _iarr([b[0] for b in blocks])
    no, pno = _iarr([len(b[1]) for b in blocks])
    lam, pl = _iarr([c[0] for b in blocks for c in b[1]])
    tI, pI = _iarr([c[1] for b in blocks for c in b[1]])
    Sa, pS = _carr(np.concatenate([np.asarray(b[2], dtype=np.complex128).ravel() for b in blocks]))
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
    ds = np.zeros(len(th))
    ay = np.zeros(len(th))
    _check(_lib.nd_elastic_observables(len(blocks), ptJ, pno, pl, pI, pS, float(k), len(th), _dptr(th), _dptr(ds),
                                       _dptr(ay)))
    return ds, ay


def exported_symbols():
    """Names of the C entry points this binding resolves (all must exist in the library)."""
    return sorted(_SIGS)


# ---------------------------------------------------------------- torch plumbing

class TorchAllocator:
    """wp_allocator backed by torch's caching allocator (device memory stays torch-owned)."""

    def __init__(self, device="cuda"):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.n_alloc = 0   # allocations served so far
        self._a = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)(self._alloc)
        self._r = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)(self._release)
        self.struct = _Alloc(self._a, self._r, None)

    def _alloc(self, nbytes, ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        self.n_alloc += 1
        return p

    def _release(self, ptr, ctx):
        self.live.pop(ptr, None)


def current_stream():
    """torch's current HIP stream as a void* (None when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- C entry points

def wp_lattice_build(M, N, two_J=1, parity=1, j_max=1, swave_only=True, n_x=8, n_phi=8, alpha=1.0,
                     p_max=10.0, q_max=10.0, hbar2_over_m=H2M, p_edges=None, q_edges=None, allocator=None):
    pe = None if p_edges is None else np.ascontiguousarray(p_edges, dtype=np.float64)
    qe = None if q_edges is None else np.ascontiguousarray(q_edges, dtype=np.float64)
    d = _LatDesc(M, N, 1 if pe is not None else 0, alpha, p_max, q_max, _dptr(pe), _dptr(qe),
                 two_J, parity, 1, j_max, 1 if swave_only else 0, n_x, n_phi, hbar2_over_m)
    h = _P()
    _check(_lib.wp_lattice_build(C.byref(d), C.byref(allocator.struct) if allocator else None, C.byref(h)))
    return h


def twobody_pseudostates(lat, kind="mt", beta=1.394, lam=0.0, V_R=1438.72, mu_R=3.11, V_A=0.0, mu_A=1.55,
                         singlet_ratio=0.82, target_BE=2.2246, tune=True):
    k = {"yamaguchi": 0, "mt": 1}[kind]
    p = _PotDesc(k, beta, lam, V_R, mu_R, V_A, mu_A, singlet_ratio, target_BE, 1 if tune else 0)
    eps0, strength = C.c_double(), C.c_double()
    _check(_lib.twobody_pseudostates(lat, C.byref(p), C.byref(eps0), C.byref(strength)))
    return eps0.value, strength.value


def perm_matrix_build(lat, precision=WP_P_FP64, stream=None):
    st = _PermStats()
    _check(_lib.perm_matrix_build(lat, precision, stream, C.byref(st)))
    return dict(nnz=st.nnz, blocks=st.blocks, candidates=st.candidates, bytes=st.bytes, device_ms=st.device_ms)


def faddeev_solve(lat, E_lab, mode=WP_SOLVE_FP64, tol=1e-12, accept=1e-7, max_iter=200, refine_every=0,
                  stream=None, allow_noconv=False, graph=0, step_tile=0, spmm_cols=0, breakup=0):
    E = np.ascontiguousarray(np.atleast_1d(E_lab), dtype=np.float64)
    o = _SolveOpts(mode, tol, accept, max_iter, refine_every, graph, step_tile, spmm_cols, breakup)
    h = _P()
    st = _lib.faddeev_solve(lat, len(E), _dptr(E), C.byref(o), stream, C.byref(h))
    if st == WP_ENOCONV and allow_noconv and h.value:
        return h, False
    if st != WP_OK and h.value:   # the library hands back a solution with WP_ENOCONV; not wanted here
        _lib.wp_solution_free(h)
    _check(st)
    return h, True


def amplitude(sol, e_idx):
    n = C.c_int()
    _check(_lib.amplitude(sol, e_idx, C.byref(n), None, None, None, None, None, None))
    n = n.value
    A = np.zeros(2 * n * n)
    S = np.zeros(2 * n * n)
    dl, et, er = np.zeros(n), np.zeros(n), np.zeros(n)
    it = (C.c_int * n)()
    nn = C.c_int()
    _check(_lib.amplitude(sol, e_idx, C.byref(nn), _dptr(A), _dptr(S), _dptr(dl), _dptr(et), _dptr(er), it))
    return dict(A=(A[0::2] + 1j * A[1::2]).reshape(n, n), S=(S[0::2] + 1j * S[1::2]).reshape(n, n),
                delta=dl, eta=et, err=er, iters=np.array(list(it)))


def faddeev_series(sol, e_idx, initial=0):
    """Series terms a_n of the FP64 path: complex array (n_terms, n_open)."""
    n = C.c_int(0)
    _check(_lib.faddeev_series(sol, e_idx, initial, C.byref(n), None))
    nopen = C.c_int()
    _check(_lib.amplitude(sol, e_idx, C.byref(nopen), None, None, None, None, None, None))
    a = np.zeros(2 * n.value * nopen.value)
    _check(_lib.faddeev_series(sol, e_idx, initial, C.byref(n), _dptr(a)))
    return (a[0::2] + 1j * a[1::2]).reshape(n.value, nopen.value)


def wp_profile_enable(on=True):
    _check(_lib.wp_profile_enable(1 if on else 0))


def wp_profile_reset():
    _check(_lib.wp_profile_reset())


def wp_profile_read():
    """{kernel name: (launches, total ms)} from the HIP events recorded around each launch."""
    n = C.c_int()
    _check(_lib.wp_profile_read(-1, C.byref(n), None, None, None))
    out = {}
    for i in range(n.value):
        buf = C.create_string_buffer(64)
        cnt = C.c_int64()
        ms = C.c_double()
        _check(_lib.wp_profile_read(i, None, buf, C.byref(cnt), C.byref(ms)))
        out[buf.value.decode()] = (cnt.value, ms.value)
    return out


# ---------------------------------------------------------------- convenience wrapper

class Solution:
    def __init__(self, handle, n_E, converged=True):
        self.h = handle
        self.n_E = n_E
        self.converged = converged

    def amplitude(self, e_idx=0):
        return amplitude(self.h, e_idx)

    def series(self, e_idx=0, initial=0):
        return faddeev_series(self.h, e_idx, initial)

    def breakup(self, e_idx=0, initial=0):
        """Breakup cells (n, 3) int array of (channel, pseudostate, q bin) and their complex
        transition elements (faddeev_breakup)."""
        n = C.c_int()
        _check(_lib.faddeev_breakup(self.h, e_idx, initial, C.byref(n), None, None))
        cells = np.zeros(max(n.value, 1) * 3, dtype=np.int32)
        U = np.zeros(max(n.value, 1) * 2)
        _check(_lib.faddeev_breakup(self.h, e_idx, initial, C.byref(n), cells.ctypes.data_as(_I), _dptr(U)))
        return cells[:3 * n.value].reshape(n.value, 3), U[0:2 * n.value:2] + 1j * U[1:2 * n.value:2]

    def __del__(self, _lib=_lib):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.wp_solution_free(self.h)
            self.h = None


class Lattice:
    """One lattice: channels, pseudostates, resident P0 (device memory from torch)."""

    def __init__(self, M, N, two_J=1, parity=1, j_max=1, swave_only=True, n_x=8, n_phi=8, alpha=1.0,
                 p_max=10.0, q_max=10.0, hbar2_over_m=H2M, p_edges=None, q_edges=None, torch_alloc=True,
                 weights="unit"):
        self.alloc = None
        if torch_alloc:
            try:
                import torch
                if torch.cuda.is_available():
                    self.alloc = TorchAllocator()
            except Exception:
                self.alloc = None
        self.M, self.N = M, N
        self.h = wp_lattice_build(M, N, two_J, parity, j_max, swave_only, n_x, n_phi, alpha, p_max, q_max,
                                  hbar2_over_m, p_edges, q_edges, self.alloc)
        if weights not in WEIGHTS:
            raise ValueError(f"weights must be one of {sorted(WEIGHTS)}")
        self.weights = weights
        if weights != "unit":
            _check(_lib.wp_lattice_weights(self.h, WEIGHTS[weights]))
        n = C.c_int()
        _check(_lib.wp_lattice_channels(self.h, C.byref(n), None))
        tab = (C.c_int * (6 * n.value))()
        _check(_lib.wp_lattice_channels(self.h, C.byref(n), tab))
        self.channels = [tuple(tab[6 * a: 6 * a + 6]) for a in range(n.value)]
        self.nch = n.value
        nm, npk = C.c_int(), C.c_int()
        _check(_lib.wp_lattice_info(self.h, C.byref(nm), C.byref(npk)))
        self.nmom, self.n_stored = nm.value, npk.value
        self.perm_stats = None

    def edges(self):
        pe, qe = np.zeros(self.M + 1), np.zeros(self.N + 1)
        _check(_lib.wp_lattice_edges(self.h, _dptr(pe), _dptr(qe)))
        return pe, qe

    def pseudostates(self, **kw):
        self.eps0, self.strength = twobody_pseudostates(self.h, **kw)
        return self.eps0, self.strength

    def pseudostate_data(self, channel):
        nb = C.c_int()
        eps = np.zeros(self.M)
        O = np.zeros(self.M * self.M)
        _check(_lib.wp_lattice_pseudostates(self.h, channel, C.byref(nb), _dptr(eps), _dptr(O), None))
        bins = np.zeros(self.M - nb.value + 1)
        _check(_lib.wp_lattice_pseudostates(self.h, channel, None, None, None, _dptr(bins)))
        return nb.value, eps, O.reshape(self.M, self.M), bins

    def resolvent(self, E_lab, channel):
        G = np.zeros(2 * self.M * self.N)
        _check(_lib.wp_lattice_resolvent(self.h, E_lab, channel, _dptr(G)))
        return (G[0::2] + 1j * G[1::2]).reshape(self.M, self.N)

    def resolvent_noalloc(self, E_lab, channel):
        """As resolvent(), through the entry point that allocates no device memory."""
        G = np.zeros(2 * self.M * self.N)
        _check(_lib.wp_lattice_resolvent_noalloc(self.h, E_lab, channel, _dptr(G)))
        return (G[0::2] + 1j * G[1::2]).reshape(self.M, self.N)

    def build_perm(self, precision="fp64", stream=None):
        p = {"fp64": WP_P_FP64, "fp32": WP_P_FP32}[precision]
        self.perm_stats = perm_matrix_build(self.h, p, stream if stream is not None else current_stream())
        return self.perm_stats

    def export_perm(self):
        st = self.perm_stats
        R = self.M * self.N
        rp = np.zeros(R + 1, dtype=np.int64)
        col = np.zeros(max(st["blocks"], 1), dtype=np.int32)
        val = np.zeros(max(st["blocks"], 1) * self.nch * self.nch)
        _check(_lib.perm_matrix_export(self.h, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                       col.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(val)))
        nb = st["blocks"]
        return rp, col[:nb], val[:nb * self.nch * self.nch].reshape(nb, self.nch, self.nch)

    def solve(self, E_lab, mode="fp64", tol=1e-12, accept=1e-7, max_iter=200, refine_every=0, stream=None,
              allow_noconv=False, graph=False, step_tile="auto", spmm_cols=0, breakup=False):
        m = SOLVE_MODES[mode]
        E = np.atleast_1d(E_lab)
        h, ok = faddeev_solve(self.h, E, m, tol, accept, max_iter, refine_every,
                              stream if stream is not None else current_stream(), allow_noconv,
                              int(bool(graph)), STEP_TILES[step_tile], int(spmm_cols), int(bool(breakup)))
        return Solution(h, len(E), ok)

    def __del__(self, _lib=_lib):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.wp_lattice_free(self.h)
            self.h = None
