"""Thin ctypes binding of ``libmfwf.so`` (include/mfwf.h).

Argument marshalling only: every step of the solver runs in the HIP library.  PyTorch
provides device memory and the stream.  PyTorch is imported before the library is loaded,
so the library binds to the HIP runtime PyTorch already has in the process.
If the library is missing or cannot be loaded this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch  # noqa: F401  (must precede loading libmfwf.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfwf.so")


class MFWFError(RuntimeError):
    pass


class SolveOpts(ctypes.Structure):
    _fields_ = [("n_stages", ctypes.c_int), ("lam", ctypes.POINTER(ctypes.c_double)),
                ("iters", ctypes.POINTER(ctypes.c_int)), ("n_check", ctypes.c_int),
                ("dchi2_tol", ctypes.c_double), ("source_is_rho", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_rows", ctypes.c_int), ("order", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int), ("lam", ctypes.c_double), ("chi2", ctypes.c_double),
                ("chi2_harm", ctypes.c_double), ("dnorm", ctypes.c_double),
                ("snorm", ctypes.c_double), ("tau", ctypes.c_double), ("n_dof", ctypes.c_long),
                ("n_checks", ctypes.c_int), ("dchi2", ctypes.c_double),
                ("rel_change", ctypes.c_double)]


class CoolOpts(ctypes.Structure):
    _fields_ = [("l_iter0", ctypes.c_int), ("l_step_max", ctypes.c_int), ("l_margin", ctypes.c_int),
                ("n_check", ctypes.c_int), ("plateau_tol", ctypes.c_double),
                ("final_tol", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("stages", ctypes.POINTER(ctypes.c_double)), ("stage_rows", ctypes.c_int),
                ("n_stages", ctypes.c_int), ("converged", ctypes.c_int)]


class BoundOpts(ctypes.Structure):
    _fields_ = [("m_sigma", ctypes.c_double), ("lam_tol", ctypes.c_double),
                ("stall_frac", ctypes.c_double), ("stall_iters", ctypes.c_int),
                ("max_iters", ctypes.c_int), ("trace", ctypes.POINTER(ctypes.c_double)),
                ("trace_rows", ctypes.c_int), ("n_iters", ctypes.c_int),
                ("n_b_updates", ctypes.c_int), ("reached_one", ctypes.c_int)]


EXPORTED = ["mfwf_plan_create", "mfwf_plan_destroy", "mfwf_set_covariances", "mfwf_sht_inv",
            "mfwf_sht_fwd", "mfwf_fluctuation_rhs", "mfwf_solve", "mfwf_time_kernels",
            "mfwf_plan_work", "mfwf_last_error", "mfwf_server_create", "mfwf_server_submit",
            "mfwf_server_poll", "mfwf_server_wait", "mfwf_server_stats", "mfwf_server_destroy",
            "mfwf_server_pool_bytes", "mfwf_solve_cooled", "mfwf_set_covariances_beam",
            "mfwf_remove_templates", "mfwf_solve_bounded", "mfwf_remove_templates_noalloc", "mfwf_plan_tuning"]


class Request(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("lmax", ctypes.c_int), ("dtype", ctypes.c_int),
                ("iters", ctypes.c_int), ("lam", ctypes.c_double),
                ("cl", ctypes.POINTER(ctypes.c_double)), ("ninv", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("s_alm_out", ctypes.c_void_p), ("s_map_out", ctypes.c_void_p)]

_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MFWFError("%s is not built; run paper_1210_4931_amd/build.py" % path)
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.mfwf_plan_create.argtypes = [ip, ip, ip, ip, ip, vp, ctypes.POINTER(vp)]
    L.mfwf_plan_destroy.argtypes = [vp]
    L.mfwf_set_covariances.argtypes = [vp, dp, ip, vp, vp]
    L.mfwf_set_covariances_beam.argtypes = [vp, dp, ip, dp, vp, vp]
    L.mfwf_remove_templates.argtypes = [vp, vp, vp, ip]
    L.mfwf_remove_templates_noalloc.argtypes = [vp, vp, vp, ip]
    L.mfwf_sht_inv.argtypes = [vp, vp, vp, ip]
    L.mfwf_sht_fwd.argtypes = [vp, vp, vp, ip]
    L.mfwf_fluctuation_rhs.argtypes = [vp, vp, vp, ip, vp]
    L.mfwf_solve.argtypes = [vp, vp, ip, vp, vp, ctypes.POINTER(SolveOpts),
                             ctypes.POINTER(SolveInfo)]
    L.mfwf_solve_cooled.argtypes = [vp, vp, ip, vp, vp, ctypes.POINTER(CoolOpts),
                                    ctypes.POINTER(SolveInfo)]
    L.mfwf_solve_bounded.argtypes = [vp, vp, ip, vp, vp, ctypes.POINTER(BoundOpts),
                                     ctypes.POINTER(SolveInfo)]
    L.mfwf_time_kernels.argtypes = [vp, ip, ip, dp]
    L.mfwf_plan_work.argtypes = [vp, dp]
    L.mfwf_plan_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.mfwf_server_create.argtypes = [ip, ctypes.c_double, ctypes.POINTER(vp)]
    L.mfwf_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.mfwf_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.mfwf_server_wait.argtypes = [vp, ctypes.c_uint64, dp]
    L.mfwf_server_stats.argtypes = [vp, dp]
    L.mfwf_server_destroy.argtypes = [vp]
    L.mfwf_server_pool_bytes.argtypes = [ip, ip, ip, ip, dp]
    L.mfwf_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name).restype = ctypes.c_char_p if name == "mfwf_last_error" else ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise MFWFError("mfwf status %d: %s" % (rc, _lib.mfwf_last_error().decode()))


def _dev_f64(x: torch.Tensor, shape) -> torch.Tensor:
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("expected a CUDA (HIP) tensor")
    if x.dtype == torch.complex128:
        x = torch.view_as_real(x)
    if x.dtype != torch.float64:
        raise TypeError("expected float64/complex128, got %s" % x.dtype)
    x = x.contiguous()
    if x.numel() != int(np.prod(shape)):
        raise ValueError("expected %s doubles, got %d" % (shape, x.numel()))
    return x


@dataclasses.dataclass
class Info:
    iters_done: int
    lam: float
    chi2: float
    chi2_harm: float
    dnorm: float
    snorm: float
    tau: float
    n_dof: int
    n_checks: int = 0
    dchi2: float = 0.0
    rel_change: float = 0.0


def _info(i: SolveInfo) -> Info:
    return Info(i.iters_done, i.lam, i.chi2, i.chi2_harm, i.dnorm, i.snorm, i.tau, i.n_dof,
                i.n_checks, i.dchi2, i.rel_change)


class Plan:
    """One (nside, lmax) problem shape on one GPU, with its own HIP stream.

    spin 0: maps [n][npix], alm [n][nalm].  spin 2 (T, Q, U): maps [n][3][npix], alm
    [n][3][nalm] (T, E, B), spectra [4][lmax+1] (TT, EE, BB, TE), inverse noise [npix][6]
    packed 3x3 blocks (TT, TQ, TU, QQ, QU, UU)."""

    def __init__(self, nside: int, lmax: int, max_batch: int = 1, spin: int = 0,
                 dtype: str = "f64", device: int = 0):
        L = load()
        self.nside, self.lmax, self.max_batch = nside, lmax, max_batch
        self.spin, self.ncomp = spin, (3 if spin == 2 else 1)
        self.npix = 12 * nside * nside
        self.nalm = (lmax + 1) * (lmax + 2) // 2
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        dt = {"f64": 0, "f32": 1}[dtype]
        with torch.cuda.device(self.device):
            _check(L.mfwf_plan_create(nside, lmax, spin, dt, max_batch,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.mfwf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers -------------------------------------------------------------------------
    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _shape(self, n, size):
        return (n, size) if self.ncomp == 1 else (n, self.ncomp, size)

    def _count(self, x):
        """maps or alm in this plan's per-map shape, with or without the leading n"""
        return x.shape[0] if x.dim() == (2 if self.ncomp == 1 else 3) else 1

    def zeros_map(self, n):
        return torch.zeros(self._shape(n, self.npix), dtype=torch.float64, device=self.device)

    def zeros_alm(self, n):
        return torch.zeros(self._shape(n, self.nalm), dtype=torch.complex128, device=self.device)

    # ---- entry points --------------------------------------------------------------------
    def set_covariances(self, cl, ninv: torch.Tensor, mask: torch.Tensor | None = None,
                        beam=None):
        """Signal spectra C_l (spin 2: rows TT, EE, BB, TE), inverse noise, mask, and an
        optional transfer function b_l (S_l = b_l^2 C_l)."""
        cl = np.ascontiguousarray(np.asarray(cl, dtype=np.float64).reshape(-1))
        ncl = 4 if self.spin == 2 else 1
        if cl.size != ncl * (self.lmax + 1):
            raise ValueError("cl must have %d x (lmax + 1) entries" % ncl)
        ninv = _dev_f64(ninv, (self.npix * (6 if self.spin == 2 else 1),))
        if mask is not None:
            if mask.dtype != torch.uint8 or not mask.is_cuda or mask.numel() != self.npix:
                raise TypeError("mask must be a CUDA uint8 tensor of npix entries")
            mask = mask.contiguous()
        bl = None
        if beam is not None:
            bl = np.ascontiguousarray(np.asarray(beam, dtype=np.float64).reshape(-1))
            if bl.size != self.lmax + 1:
                raise ValueError("beam must have lmax + 1 entries")
        self._enter()
        rc = _lib.mfwf_set_covariances_beam(
            self._h, cl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ncl,
            None if bl is None else bl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ninv.data_ptr(), None if mask is None else mask.data_ptr())
        _check(rc)
        self._keep = (ninv, mask)

    def remove_templates(self, d: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Monopole and dipole removal of Eq. (12) on the observed pixels (T for spin 2)."""
        n = self._count(d)
        x = _dev_f64(d, (n, self.ncomp, self.npix))
        out = self.zeros_map(n) if out is None else out
        self._enter()
        _check(_lib.mfwf_remove_templates(self._h, x.data_ptr(), out.data_ptr(), n))
        self._leave()
        return out

    def remove_templates_noalloc(self, d: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """remove_templates into a caller-provided output, with no device allocation in the
        library (at most 64 maps per call)."""
        n = self._count(d)
        x = _dev_f64(d, (n, self.ncomp, self.npix))
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and out.numel() == x.numel()):
            raise TypeError("out must be a contiguous CUDA float64 tensor shaped like d")
        self._enter()
        _check(_lib.mfwf_remove_templates_noalloc(self._h, x.data_ptr(), out.data_ptr(), n))
        self._leave()
        return out

    def sht_inv(self, alm: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = self._count(alm)
        a = _dev_f64(alm, (n, self.ncomp, 2 * self.nalm))
        out = self.zeros_map(n) if out is None else out
        self._enter()
        _check(_lib.mfwf_sht_inv(self._h, a.data_ptr(), out.data_ptr(), n))
        self._leave()
        return out

    def sht_fwd(self, maps: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = self._count(maps)
        m = _dev_f64(maps, (n, self.ncomp, self.npix))
        out = self.zeros_alm(n) if out is None else out
        self._enter()
        _check(_lib.mfwf_sht_fwd(self._h, m.data_ptr(), torch.view_as_real(out).data_ptr(), n))
        self._leave()
        return out

    def fluctuation_rhs(self, g1: torch.Tensor, h: torch.Tensor, out=None) -> torch.Tensor:
        n = self._count(g1)
        g = _dev_f64(g1, (n, self.ncomp, self.npix))
        hh = _dev_f64(h, (n, self.ncomp, 2 * self.nalm))
        out = self.zeros_map(n) if out is None else out
        self._enter()
        _check(_lib.mfwf_fluctuation_rhs(self._h, g.data_ptr(), hh.data_ptr(), n, out.data_ptr()))
        self._leave()
        return out

    def solve(self, inp: torch.Tensor, lam=None, iters=None, source_is_rho=False,
              use_graph=True, out_alm=None, out_map=None, want_map=True, n_check=0,
              dchi2_tol=0.0, chained=True):
        """Messenger iteration.  lam/iters: per-stage schedule (default lambda 1, 300 its).
        chained=False runs the FP32 form's iterations from the pixel map (same values).
        Returns (s_alm [n, nalm] complex128, s_map [n, npix] or None, [Info] * n); with
        n_check > 0 a fourth item, the diagnostics history as a numpy array
        [checks][n][5] of (iteration, lambda, chi^2, |s_k - s_{k-1}|, |s_k|).  dchi2_tol > 0
        ends the solve early once chi^2 changes by less than dchi2_tol sigma_chi2 per
        iteration between two checks of one stage (Info.iters_done says where)."""
        import numpy as np
        n = self._count(inp)
        x = _dev_f64(inp, (n, self.ncomp, self.npix))
        if lam is None:
            lam, iters = [1.0], [300 if iters is None else int(iters)]
        lam_a = (ctypes.c_double * len(lam))(*[float(v) for v in lam])
        it_a = (ctypes.c_int * len(iters))(*[int(v) for v in iters])
        total = sum(int(v) for v in iters)
        rows = (total // n_check + 1) if n_check > 0 else 0
        hist = np.zeros((rows, n, 5)) if rows else None
        hptr = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if rows else None
        opts = SolveOpts(len(lam), lam_a, it_a, int(n_check), float(dchi2_tol),
                         int(bool(source_is_rho)),
                         int(bool(use_graph)), hptr, rows, 0 if chained else 1)
        s_alm = self.zeros_alm(n) if out_alm is None else out_alm
        s_map = (self.zeros_map(n) if out_map is None else out_map) if want_map else None
        infos = (SolveInfo * n)()
        self._enter()
        _check(_lib.mfwf_solve(self._h, x.data_ptr(), n, torch.view_as_real(s_alm).data_ptr(),
                               None if s_map is None else s_map.data_ptr(), ctypes.byref(opts),
                               infos))
        self._leave()
        info = [_info(i) for i in infos]
        if n_check > 0:
            return s_alm, s_map, info, hist[:max(i.n_checks for i in infos)] if n else hist
        return s_alm, s_map, info

    def solve_cooled(self, data: torch.Tensor, l_iter0=0, l_step_max=0, l_margin=0, n_check=0,
                     plateau_tol=0.0, final_tol=0.0, max_iters=0, want_map=True):
        """Converged Wiener filter with the cooling schedule of Sect. 3 (0 = the default of
        each option).  Returns (s_alm, s_map or None, [Info] * n, stages, converged), stages a
        numpy array [n_stages][5] of (l_iter, lambda, lmax_SHT, iterations, chi^2/n_dof)."""
        import numpy as np
        n = self._count(data)
        x = _dev_f64(data, (n, self.ncomp, self.npix))
        rows = 64
        st = np.zeros((rows, 5))
        opts = CoolOpts(int(l_iter0), int(l_step_max), int(l_margin), int(n_check),
                        float(plateau_tol), float(final_tol), int(max_iters),
                        st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows, 0, 0)
        s_alm = self.zeros_alm(n)
        s_map = self.zeros_map(n) if want_map else None
        infos = (SolveInfo * n)()
        self._enter()
        _check(_lib.mfwf_solve_cooled(self._h, x.data_ptr(), n, torch.view_as_real(s_alm).data_ptr(),
                                      None if s_map is None else s_map.data_ptr(),
                                      ctypes.byref(opts), infos))
        self._leave()
        info = [_info(i) for i in infos]
        return s_alm, s_map, info, st[:min(opts.n_stages, rows)], bool(opts.converged)

    def solve_bounded(self, data: torch.Tensor, m_sigma=0.0, lam_tol=0.0, stall_frac=0.0,
                      stall_iters=0, max_iters=0, want_map=True):
        """Wiener filter under the error bound of Sect. 2.2 (0 = the default of each option).
        Returns (s_alm, s_map or None, [Info] * n, trace, n_b_updates, reached_one), trace a
        numpy array [iterations][3] of (lambda, chi^2(lambda, x) after the iteration, b)."""
        import numpy as np
        n = self._count(data)
        x = _dev_f64(data, (n, self.ncomp, self.npix))
        rows = max_iters if max_iters > 0 else 5000
        tr = np.zeros((rows, 3))
        opts = BoundOpts(float(m_sigma), float(lam_tol), float(stall_frac), int(stall_iters),
                         int(max_iters), tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows,
                         0, 0, 0)
        s_alm = self.zeros_alm(n)
        s_map = self.zeros_map(n) if want_map else None
        infos = (SolveInfo * n)()
        self._enter()
        _check(_lib.mfwf_solve_bounded(self._h, x.data_ptr(), n, torch.view_as_real(s_alm).data_ptr(),
                                       None if s_map is None else s_map.data_ptr(),
                                       ctypes.byref(opts), infos))
        self._leave()
        info = [_info(i) for i in infos]
        return (s_alm, s_map, info, tr[:min(opts.n_iters, rows)], opts.n_b_updates,
                bool(opts.reached_one))

    def work(self):
        """(Legendre triples evaluated, full triangle pairs*nalm, ring pairs, max FFT length)."""
        out = (ctypes.c_double * 4)()
        _check(_lib.mfwf_plan_work(self._h, out))
        return tuple(out)

    def tuning(self) -> dict:
        """Kernel shapes in use (autotuned, default or forced by MFWF_TUNE_FORCE)."""
        out = (ctypes.c_int * 8)()
        _check(_lib.mfwf_plan_tuning(self._h, out))
        keys = ["synth", "ana", "g0", "g1", "cta", "cts", "lamgen", "source"]
        return dict(zip(keys, list(out)))

    def time_kernels(self, nmaps=1, reps=10):
        """Mean ms per launch of [pixel, fft_fwd, leg_analysis, harmonic, leg_synth, fft_inv]."""
        out = (ctypes.c_double * 6)()
        self._enter()
        _check(_lib.mfwf_time_kernels(self._h, nmaps, reps, out))
        return list(out)


class Server:
    """Continuous-batching server for independent temperature Wiener-filter requests (each
    with its own data, noise variance map and mask).  submit() returns an id and the output
    tensors (filled when the request completes); wait(id) blocks and returns the latency in
    seconds from submission to results ready."""

    def __init__(self, slots: int = 64, hbm_gb: float = 200.0, device: int = 0):
        L = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.mfwf_server_create(slots, float(hbm_gb), ctypes.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, nside, lmax, cl, ninv, data, mask=None, dtype="f64", iters=300, lam=1.0,
               want_map=True):
        npix, nalm = 12 * nside * nside, (lmax + 1) * (lmax + 2) // 2
        cl = np.ascontiguousarray(np.asarray(cl, dtype=np.float64).reshape(-1))
        if cl.size != lmax + 1:
            raise ValueError("cl must have lmax + 1 entries")
        ninv = _dev_f64(ninv, (npix,))
        data = _dev_f64(data, (npix,))
        if mask is not None:
            if mask.dtype != torch.uint8 or not mask.is_cuda or mask.numel() != npix:
                raise TypeError("mask must be a CUDA uint8 tensor of npix entries")
            mask = mask.contiguous()
        s_alm = torch.zeros(nalm, dtype=torch.complex128, device=self.device)
        s_map = torch.zeros(npix, dtype=torch.float64, device=self.device) if want_map else None
        torch.cuda.current_stream(self.device).synchronize()  # inputs complete before submission
        req = Request(nside, lmax, {"f64": 0, "f32": 1}[dtype], int(iters), float(lam),
                      cl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ninv.data_ptr(),
                      None if mask is None else mask.data_ptr(), data.data_ptr(),
                      torch.view_as_real(s_alm).data_ptr(),
                      None if s_map is None else s_map.data_ptr())
        rid = ctypes.c_uint64()
        _check(_lib.mfwf_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._live[rid.value] = (ninv, mask, data, s_alm, s_map)
        return rid.value, s_alm, s_map

    @staticmethod
    def pool_bytes(nside, lmax, dtype="f64", slots=64) -> float:
        """Bytes a pool of this shape is charged against the server's HBM budget."""
        out = ctypes.c_double()
        _check(load().mfwf_server_pool_bytes(nside, lmax, {"f64": 0, "f32": 1}[dtype], slots,
                                             ctypes.byref(out)))
        return out.value

    def done(self, rid) -> bool:
        d = ctypes.c_int()
        _check(_lib.mfwf_server_poll(self._h, rid, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid) -> float:
        lat = ctypes.c_double()
        try:
            _check(_lib.mfwf_server_wait(self._h, rid, ctypes.byref(lat)))
        finally:
            self._live.pop(rid, None)
        return lat.value

    def stats(self) -> dict:
        out = (ctypes.c_double * 8)()
        _check(_lib.mfwf_server_stats(self._h, out))
        keys = ["completed", "queued", "occupied_slots", "pools", "pool_bytes", "iterations",
                "pools_created", "pools_evicted"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.mfwf_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
