"""ctypes binding of liblrt (include/lrt.h): argument marshalling only.

Every step of the radiation path runs in the library's HIP kernels; this module
converts the seeded inputs (synth) to the C structures, passes torch device
buffers by pointer and raises LrtError on any non-OK status.  It refuses to
work without the built library: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrt.so")

LRT_FP64 = 0
LRT_FP32_COMP = 1
PRECISIONS = {"fp64": LRT_FP64, "fp32c": LRT_FP32_COMP}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_vp = C.c_void_p

EXPORTS = ["lrt_version", "lrt_status_string", "lrt_create", "lrt_destroy", "lrt_last_error",
           "lrt_set_species", "lrt_set_lines", "lrt_set_grid", "lrt_set_cells", "lrt_set_continuum", "lrt_set_lorentz",
           "lrt_set_rays_slab", "lrt_set_rays_axi", "lrt_set_rays_axi_fibonacci",
           "lrt_fibonacci_quadrature", "lrt_set_march", "lrt_set_far_temperature", "lrt_trace_axi_ray", "lrt_get_sizes", "lrt_get_ray",
           "lrt_coeffs", "lrt_march", "lrt_solve", "lrt_solve_ranges", "lrt_count_terms",
           "lrt_count_terms_ranges", "lrt_profile",
           "lrt_profile_read", "lrt_server_start", "lrt_submit", "lrt_poll", "lrt_wait",
           "lrt_cancel", "lrt_server_info", "lrt_server_stop", "lrt_set_cr", "lrt_set_line_levels",
           "lrt_cr_populations", "lrt_probe", "lrt_gen_rovib_lines", "lrt_march_noalloc"]

KERNELS = {"thermo": 0, "scale": 1, "ranges": 2, "accum": 3, "march": 4, "cr": 5}


class LrtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("lrt status %d: %s" % (status, msg))
        self.status = status


class _Species(C.Structure):
    _fields_ = [("kind", C.c_int), ("mass", C.c_double), ("n_levels", C.c_int),
                ("level_E", _dp), ("level_g", _dp), ("n_el", C.c_int), ("el_T", _dp),
                ("el_g", _dp), ("el_nv", _ip), ("el_Jmax", _ip), ("vib_G", _dp),
                ("vib_B", _dp), ("vib_D", _dp)]


class _Lines(C.Structure):
    _fields_ = [("n", C.c_int64), ("nu0", _dp), ("A", _dp), ("Eu_ev", _dp), ("Eu_rot", _dp),
                ("El_ev", _dp), ("El_rot", _dp), ("gu", _dp), ("gl", _dp), ("species", _i32p),
                ("on_device", C.c_int)]


class _BandSystem(C.Structure):
    _fields_ = [("species", C.c_int32), ("hund", C.c_int32), ("Lambda_u", C.c_int32), ("Lambda_l", C.c_int32),
                *[(k, C.c_double) for k in ("Te_u", "Te_l", "g_u", "g_l",
                                            "we_u", "wexe_u", "weye_u", "Be_u", "ae_u", "De_u", "be_u", "gamma_u",
                                            "we_l", "wexe_l", "weye_l", "Be_l", "ae_l", "De_l", "be_l", "gamma_l")],
                ("nv_u", C.c_int32), ("nv_l", C.c_int32), ("J_max", C.c_int32), ("Re2", _dp)]


class _LineBuffers(C.Structure):
    _fields_ = [(k, _dp) for k in ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")] + \
        [("species", _i32p)]


LINE_FIELDS = ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")


class _Continuum(C.Structure):
    _fields_ = [("species", C.c_int32), ("ion", C.c_int32), ("E_ion", C.c_double),
                ("Q_ion", C.c_double), ("sigma0", _dp), ("peach", C.c_double * 8), ("z", C.c_double)]


class _CRSpecies(C.Structure):
    _fields_ = [("species", C.c_int32), ("ion", C.c_int32), ("partner", C.c_int32),
                ("partner_ion", C.c_int32), ("n_model", C.c_int32), ("diss_x", C.c_int32),
                ("diss_y", C.c_int32), ("E_ion", C.c_double), ("Q_ion", C.c_double),
                ("partner_E_ion", C.c_double), ("partner_Q_ion", C.c_double), ("Q_x", C.c_double),
                ("Q_y", C.c_double), ("E_diss", C.c_double), ("nu_cut", C.c_double),
                ("texp", C.c_double * 12), ("hpie", _dp), ("eie", _dp), ("A", _dp), ("eii", _dp),
                ("ce", _dp), ("hpid", _dp), ("eid", _dp)]


class _Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_species", C.c_int), ("T_tr", _dp), ("T_v", _dp),
                ("N", _dp), ("n_e", _dp), ("on_device", C.c_int)]


class _LosRequest(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_species", C.c_int), ("T_tr", _dp), ("T_v", _dp),
                ("N", _dp), ("n_e", _dp), ("ds", _dp), ("k_first", C.c_int64),
                ("n_window", C.c_int64), ("species_mask", C.c_uint64), ("keep_spectrum", C.c_int),
                ("T_far", C.c_double), ("scheme", C.c_int)]


class _LosResult(C.Structure):
    _fields_ = [("status", C.c_int), ("I_int", C.c_double), ("n_window", C.c_int64),
                ("queue_ms", C.c_double), ("latency_ms", C.c_double)]


_lib = None


def lib():
    """Load liblrt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblrt.so not built: run __graft_entry__.build() "
                              "(python -m paper_2604_11856_amd.build)")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        sig = {
            "lrt_version": (C.c_char_p, []),
            "lrt_status_string": (C.c_char_p, [st]),
            "lrt_create": (st, [C.c_int, C.POINTER(_vp)]),
            "lrt_destroy": (None, [_vp]),
            "lrt_last_error": (C.c_char_p, [_vp]),
            "lrt_set_species": (st, [_vp, C.c_int, C.POINTER(_Species)]),
            "lrt_set_lines": (st, [_vp, C.POINTER(_Lines)]),
            "lrt_set_grid": (st, [_vp, C.c_double, C.c_double, C.c_int64, C.c_int64]),
            "lrt_set_cells": (st, [_vp, C.POINTER(_Cells)]),
            "lrt_set_continuum": (st, [_vp, C.c_int, C.POINTER(_Continuum)]),
            "lrt_set_lorentz": (st, [_vp, _dp]),
            "lrt_set_rays_slab": (st, [_vp, C.c_int64, _dp, C.c_int]),
            "lrt_set_rays_axi": (st, [_vp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                      _dp, C.c_int, C.c_int]),
            "lrt_set_rays_axi_fibonacci": (st, [_vp, C.c_int, C.c_int, C.c_double, C.c_double,
                                                C.c_int, _dp, C.c_int, C.c_int, C.c_int]),
            "lrt_fibonacci_quadrature": (st, [C.c_int, C.c_int, C.c_int, C.c_int64, _dp, _dp, _i64p]),
            "lrt_set_march": (st, [_vp, C.c_int]),
            "lrt_set_far_temperature": (st, [_vp, _dp, C.c_int64]),
            "lrt_trace_axi_ray": (st, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_int64, _i32p, _dp, _i64p]),
            "lrt_get_sizes": (st, [_vp, _i64p, _i64p, _i64p, _i64p, _i64p, _i64p]),
            "lrt_get_ray": (st, [_vp, C.c_int64, C.c_int64, _i32p, _dp, _i64p, _dp, _i64p]),
            "lrt_coeffs": (st, [_vp, C.c_int64, C.c_int, _vp, _vp, _vp, _vp]),
            "lrt_march": (st, [_vp, C.c_int64, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]),
            "lrt_solve": (st, [_vp, C.c_int, C.c_int64, _dp, _dp, _dp, _vp]),
            "lrt_count_terms": (st, [_vp, C.c_int64, _i64p, _i64p, _vp]),
            "lrt_solve_ranges": (st, [_vp, C.c_int, C.c_int64, _i64p, _i64p, _dp, _dp, _dp, _vp]),
            "lrt_probe": (st, [C.c_int, C.c_int, _dp, _dp]),
            "lrt_march_noalloc": (st, [_vp, C.c_int64, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]),
            "lrt_gen_rovib_lines": (st, [_vp, C.c_int, C.POINTER(_BandSystem), C.c_double, C.c_double,
                                         C.c_int64, C.POINTER(_LineBuffers), _i64p, _vp]),
            "lrt_count_terms_ranges": (st, [_vp, C.c_int64, _i64p, _i64p, _i64p, _i64p, _vp]),
            "lrt_profile": (st, [_vp, C.c_int]),
            "lrt_profile_read": (st, [_vp, C.c_int, _dp, _i64p]),
            "lrt_server_start": (st, [_vp, C.c_size_t, C.c_int, C.POINTER(_vp)]),
            "lrt_submit": (st, [_vp, C.POINTER(_LosRequest), C.POINTER(C.c_uint64)]),
            "lrt_poll": (st, [_vp, C.c_uint64, C.POINTER(_LosResult), _dp]),
            "lrt_wait": (st, [_vp, C.c_uint64, C.c_double, C.POINTER(_LosResult), _dp]),
            "lrt_cancel": (st, [_vp, C.c_uint64]),
            "lrt_server_info": (st, [_vp, _i64p, _i64p, _i64p, _i64p, C.POINTER(C.c_size_t)]),
            "lrt_server_stop": (st, [_vp]),
            "lrt_set_cr": (st, [_vp, C.c_int, C.POINTER(_CRSpecies), _dp]),
            "lrt_set_line_levels": (st, [_vp, _i32p, _i32p, C.c_int64]),
            "lrt_cr_populations": (st, [_vp, C.c_int, _dp, _vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    return int(getattr(stream, "cuda_stream", stream)) or None


class Context:
    """One liblrt context on one HIP device."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = _vp()
        s = self._L.lrt_create(device, C.byref(h))
        if s != 0:
            raise LrtError(s, self._L.lrt_last_error(None).decode())
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self._L.lrt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s):
        if s != 0:
            raise LrtError(s, self._L.lrt_last_error(self.h).decode())

    # -- state ---------------------------------------------------------------
    def set_species(self, species):
        arr = (_Species * len(species))()
        keep = []
        for i, sp in enumerate(species):
            f = lambda x, t=np.float64: np.ascontiguousarray(x, t)
            lE, lg = f(sp.level_E), f(sp.level_g)
            eT, eg = f(sp.el_T), f(sp.el_g)
            env, eJ = f(sp.el_nv, np.int32), f(sp.el_Jmax, np.int32)
            vG, vB, vD = f(sp.vib_G), f(sp.vib_B), f(sp.vib_D)
            keep += [lE, lg, eT, eg, env, eJ, vG, vB, vD]
            arr[i] = _Species(sp.kind, sp.mass, lE.size, _p(lE), _p(lg), eT.size, _p(eT), _p(eg),
                              _p(env, _ip), _p(eJ, _ip), _p(vG), _p(vB), _p(vD))
        self._chk(self._L.lrt_set_species(self.h, len(species), arr))

    def set_lines(self, lines):
        a = {k: np.ascontiguousarray(getattr(lines, k), np.float64)
             for k in ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")}
        sp = np.ascontiguousarray(lines.species, np.int32)
        s = _Lines(lines.n, _p(a["nu0"]), _p(a["A"]), _p(a["Eu_ev"]), _p(a["Eu_rot"]),
                   _p(a["El_ev"]), _p(a["El_rot"]), _p(a["gu"]), _p(a["gl"]), _p(sp, _i32p), 0)
        self._chk(self._L.lrt_set_lines(self.h, C.byref(s)))

    def set_lines_device(self, t):
        """Line list from contiguous device tensors: t maps LINE_FIELDS to
        float64 and "species" to int32 tensors of one length."""
        n = int(t["nu0"].shape[0])
        dp = lambda x: C.cast(C.c_void_p(x.data_ptr()), _dp)
        for k in LINE_FIELDS + ("species",):
            if not (t[k].is_cuda and t[k].is_contiguous() and int(t[k].shape[0]) == n):
                raise ValueError("device lines: %s must be a contiguous device tensor of length %d" % (k, n))
        s = _Lines(n, *[dp(t[k]) for k in LINE_FIELDS], C.cast(C.c_void_p(t["species"].data_ptr()), _i32p), 1)
        self._chk(self._L.lrt_set_lines(self.h, C.byref(s)))

    def gen_rovib_lines(self, systems, nu_min: float, nu_max: float, device="cuda:0", stream=None):
        """Rovibronic lines of synth.BandSystem records generated on the device
        (lrt_gen_rovib_lines): dict of device tensors (LINE_FIELDS float64,
        "species" int32), in the generator's order."""
        import torch
        arr = (_BandSystem * len(systems))()
        keep = []
        for i, b in enumerate(systems):
            re2 = np.ascontiguousarray(b.Re2, np.float64)
            keep.append(re2)
            arr[i] = _BandSystem(b.species, b.hund, b.Lambda_u, b.Lambda_l,
                                 *[float(getattr(b, k)) for k in (
                                     "Te_u", "Te_l", "g_u", "g_l", "we_u", "wexe_u", "weye_u", "Be_u", "ae_u",
                                     "De_u", "be_u", "gamma_u", "we_l", "wexe_l", "weye_l", "Be_l", "ae_l",
                                     "De_l", "be_l", "gamma_l")],
                                 b.nv_u, b.nv_l, b.J_max, _p(re2))
        n = C.c_int64()
        self._chk(self._L.lrt_gen_rovib_lines(self.h, len(systems), arr, float(nu_min), float(nu_max), 0, None,
                                              C.byref(n), _stream(stream)))
        out = {k: torch.empty(max(1, n.value), dtype=torch.float64, device=device) for k in LINE_FIELDS}
        out["species"] = torch.empty(max(1, n.value), dtype=torch.int32, device=device)
        bufs = _LineBuffers(*[C.cast(C.c_void_p(out[k].data_ptr()), _dp) for k in LINE_FIELDS],
                            C.cast(C.c_void_p(out["species"].data_ptr()), _i32p))
        if n.value:
            self._chk(self._L.lrt_gen_rovib_lines(self.h, len(systems), arr, float(nu_min), float(nu_max), n.value,
                                                  C.byref(bufs), C.byref(n), _stream(stream)))
        return {k: v[:n.value] for k, v in out.items()}

    def set_grid(self, grid):
        self._chk(self._L.lrt_set_grid(self.h, float(grid.nu_min), float(grid.nu_max),
                                       int(grid.n_points), int(grid.band_points)))

    def set_cells(self, cells):
        T_tr = np.ascontiguousarray(cells.T_tr, np.float64)
        T_v = np.ascontiguousarray(cells.T_v, np.float64)
        N = np.ascontiguousarray(cells.N, np.float64)
        ne = np.ascontiguousarray(cells.n_e, np.float64)
        s = _Cells(T_tr.shape[0], N.shape[1], _p(T_tr), _p(T_v), _p(N), _p(ne), 0)
        self._chk(self._L.lrt_set_cells(self.h, C.byref(s)))

    def set_cells_device(self, T_tr, T_v, N, n_e):
        """Cell states from contiguous float64 device tensors ([n], [n], [n, S], [n])
        on the context's device; copied and validated on the device."""
        for t in (T_tr, T_v, N, n_e):
            if not (t.is_cuda and t.dtype.itemsize == 8 and t.is_contiguous()):
                raise ValueError("device cells must be contiguous float64 device tensors")
        dp = lambda t: C.cast(C.c_void_p(t.data_ptr()), _dp)
        s = _Cells(int(T_tr.shape[0]), int(N.shape[1]), dp(T_tr), dp(T_v), dp(N), dp(n_e), 1)
        self._chk(self._L.lrt_set_cells(self.h, C.byref(s)))

    def set_rays(self, geom):
        if isinstance(geom, synth.SlabGeometry):
            dx = np.ascontiguousarray(geom.dx, np.float64)
            self._chk(self._L.lrt_set_rays_slab(self.h, dx.size, _p(dx), int(geom.n_mu)))
        elif isinstance(geom, synth.AxiGeometry) and geom.fib_los > 0:
            wr = np.ascontiguousarray(geom.wall_r, np.float64)
            self._chk(self._L.lrt_set_rays_axi_fibonacci(
                self.h, geom.nx, geom.nr, float(geom.Lx), float(geom.R), wr.size, _p(wr),
                int(geom.fib_los), int(geom.fib_polar), int(geom.fib_azim)))
        elif isinstance(geom, synth.AxiGeometry):
            wr = np.ascontiguousarray(geom.wall_r, np.float64)
            self._chk(self._L.lrt_set_rays_axi(self.h, geom.nx, geom.nr, float(geom.Lx),
                                               float(geom.R), wr.size, _p(wr), int(geom.n_mu),
                                               int(geom.n_phi)))
        else:
            raise TypeError("unknown geometry %r" % type(geom))

    def set_continuum(self, records):
        """Atomic continuum records (synth.Continuum), or None / [] for none."""
        records = records or []
        keep = [np.ascontiguousarray(r.sigma0, np.float64) for r in records]
        arr = (_Continuum * max(1, len(records)))()
        for j, (r, s0) in enumerate(zip(records, keep)):
            arr[j] = _Continuum(int(r.species), int(r.ion), float(r.E_ion), float(r.Q_ion), _p(s0),
                                (C.c_double * 8)(*[float(v) for v in r.peach]), float(r.z))
        self._chk(self._L.lrt_set_continuum(self.h, len(records), arr))

    def set_lorentz(self, E_ion):
        """Per-species ionization energies (cm^-1) for the full Lorentz width of
        atomic lines, or None for the uniform Stark law."""
        if E_ion is None:
            self._chk(self._L.lrt_set_lorentz(self.h, None))
            return
        e = np.ascontiguousarray(E_ion, np.float64)
        self._chk(self._L.lrt_set_lorentz(self.h, _p(e)))

    def set_cr(self, cr):
        """QSS collisional-radiative atoms and molecules (synth.CRModel), or
        None for none."""
        if cr is None or not cr.species:
            self._chk(self._L.lrt_set_cr(self.h, 0, None, None))
            return
        keep, arr = [], (_CRSpecies * len(cr.species))()
        for j, r in enumerate(cr.species):
            L = int(r.n_model)
            z = np.zeros((L, 3))
            t = [np.ascontiguousarray(a, np.float64) for a in
                 (r.hpie, r.eie, r.A, r.eii, r.ce,
                  z if r.hpid is None else r.hpid, z if r.eid is None else r.eid)]
            keep.append(t)
            texp = np.zeros(12)
            texp[:len(r.texp)] = r.texp
            arr[j] = _CRSpecies(int(r.species), int(r.ion), int(r.partner), int(r.partner_ion),
                                L, int(r.diss_x), int(r.diss_y), float(r.E_ion), float(r.Q_ion),
                                float(r.partner_E_ion), float(r.partner_Q_ion), float(r.Q_x),
                                float(r.Q_y), float(r.E_diss), float(r.nu_cut),
                                (C.c_double * 12)(*[float(v) for v in texp]), *[_p(a) for a in t])
        w = np.ascontiguousarray(cr.collider_w, np.float64)
        self._chk(self._L.lrt_set_cr(self.h, len(cr.species), arr, _p(w)))

    def set_line_levels(self, levels):
        """[n_lines, 2] (upper, lower) level per line (-1: none), or None."""
        if levels is None:
            self._chk(self._L.lrt_set_line_levels(self.h, None, None, 0))
            return
        lev = np.asarray(levels, np.int32)
        u, l = np.ascontiguousarray(lev[:, 0]), np.ascontiguousarray(lev[:, 1])
        self._chk(self._L.lrt_set_line_levels(self.h, _p(u, _i32p), _p(l, _i32p), lev.shape[0]))

    def cr_populations(self, rec: int, n_levels: int, stream=None):
        """State populations [n_cells, n_levels] of QSS-CR record `rec`."""
        nc = max(self.sizes()["n_cells"], 0)
        out = np.zeros((nc, n_levels))
        self._chk(self._L.lrt_cr_populations(self.h, int(rec), _p(out), _stream(stream)))
        return out

    def set_march(self, scheme: int):
        self._chk(self._L.lrt_set_march(self.h, int(scheme)))

    def set_far_temperature(self, T_far):
        """Scalar (every ray), per-ray array, or None (all free)."""
        if T_far is None:
            self._chk(self._L.lrt_set_far_temperature(self.h, None, 0))
            return
        t = np.ascontiguousarray(np.atleast_1d(np.asarray(T_far, np.float64)))
        self._chk(self._L.lrt_set_far_temperature(self.h, _p(t), t.size))

    def load(self, wl):
        """Species, lines, grid, cells and rays of a synth.Workload."""
        self.set_species(wl.species)
        if getattr(wl, "lorentz_E_ion", None) is not None:
            self.set_lorentz(wl.lorentz_E_ion)
        self.set_lines(wl.lines)
        self.set_grid(wl.grid)
        self.set_cells(wl.cells)
        self.set_rays(wl.geometry)
        if getattr(wl, "continuum", None):
            self.set_continuum(wl.continuum)
        if getattr(wl, "cr", None) is not None:
            self.set_cr(wl.cr)
            if getattr(wl, "line_levels", None) is not None:
                self.set_line_levels(wl.line_levels)
        return self

    def sizes(self):
        v = [C.c_int64() for _ in range(6)]
        self._chk(self._L.lrt_get_sizes(self.h, *[C.byref(x) for x in v]))
        keys = ("n_cells", "n_rays", "n_wall", "n_points", "n_bands", "band_points")
        return {k: x.value for k, x in zip(keys, v)}

    def band_len(self, band: int) -> int:
        s = self.sizes()
        return min(s["band_points"], s["n_points"] - band * s["band_points"])

    def segment_count(self) -> int:
        """Segments of all rays (lrt_get_ray's count query per ray)."""
        n, w, wall = C.c_int64(), C.c_double(), C.c_int64()
        tot = 0
        for r in range(self.sizes()["n_rays"]):
            self._chk(self._L.lrt_get_ray(self.h, r, 0, None, None, C.byref(n), C.byref(w), C.byref(wall)))
            tot += n.value
        return tot

    def ray(self, r: int):
        n, w, wall = C.c_int64(), C.c_double(), C.c_int64()
        self._chk(self._L.lrt_get_ray(self.h, r, 0, None, None, C.byref(n), C.byref(w), C.byref(wall)))
        cell = np.zeros(n.value, np.int32)
        ds = np.zeros(n.value)
        self._chk(self._L.lrt_get_ray(self.h, r, n.value, _p(cell, _i32p), _p(ds), C.byref(n),
                                      C.byref(w), C.byref(wall)))
        return cell, ds, w.value, wall.value

    # -- compute ---------------------------------------------------------------
    def coeffs(self, band: int, precision: int, eta, kappa, escale=None, stream=None):
        self._chk(self._L.lrt_coeffs(self.h, band, precision, _ptr(eta), _ptr(kappa),
                                     _ptr(escale), _stream(stream)))

    def march(self, band: int, precision: int, eta, kappa, escale, I_out, I_int_out, stream=None):
        self._chk(self._L.lrt_march(self.h, band, precision, _ptr(eta), _ptr(kappa),
                                    _ptr(escale), _ptr(I_out), _ptr(I_int_out), _stream(stream)))

    def march_noalloc(self, band: int, precision: int, eta, kappa, escale, I_out, I_int_out, stream=None):
        """lrt_march_noalloc: lrt_march with the library's static scratch
        instead of an allocated workspace."""
        self._chk(self._L.lrt_march_noalloc(self.h, band, precision, _ptr(eta), _ptr(kappa),
                                            _ptr(escale), _ptr(I_out), _ptr(I_int_out), _stream(stream)))

    def solve(self, precision: int, first_band: int = 0, stream=None):
        s = self.sizes()
        q = np.zeros(s["n_wall"])
        I_int = np.zeros(s["n_rays"])
        qb = np.zeros((s["n_wall"], s["n_bands"]))
        self._chk(self._L.lrt_solve(self.h, precision, first_band, _p(q), _p(I_int), _p(qb),
                                    _stream(stream)))
        return q, I_int, qb

    def solve_ranges(self, precision: int, k_first, n_points, stream=None):
        """The whole path over grid-point ranges [k_first[i], k_first[i] + n_points[i]):
        (q [n_wall], I_int [n_rays], q_range [n_wall, n_ranges])."""
        kf = np.ascontiguousarray(k_first, np.int64)
        npt = np.ascontiguousarray(n_points, np.int64)
        s = self.sizes()
        q = np.zeros(s["n_wall"])
        I_int = np.zeros(s["n_rays"])
        qr = np.zeros((s["n_wall"], kf.size))
        self._chk(self._L.lrt_solve_ranges(self.h, precision, kf.size, _p(kf, _i64p), _p(npt, _i64p),
                                           _p(q), _p(I_int), _p(qr), _stream(stream)))
        return q, I_int, qr

    def count_terms_ranges(self, k_first, n_points, stream=None, core: bool = False):
        kf = np.ascontiguousarray(k_first, np.int64)
        npt = np.ascontiguousarray(n_points, np.int64)
        n, nc = C.c_int64(), C.c_int64()
        self._chk(self._L.lrt_count_terms_ranges(self.h, kf.size, _p(kf, _i64p), _p(npt, _i64p),
                                                 C.byref(n), C.byref(nc), _stream(stream)))
        return (n.value, nc.value) if core else n.value

    def count_terms(self, band: int, stream=None, core: bool = False):
        """In-window terms of a band; with core=True also those within 25
        Voigt HWHM of their line centre: (total, core)."""
        n, nc = C.c_int64(), C.c_int64()
        self._chk(self._L.lrt_count_terms(self.h, band, C.byref(n), C.byref(nc), _stream(stream)))
        return (n.value, nc.value) if core else n.value

    def profile(self, enable: bool = True):
        self._chk(self._L.lrt_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel: str):
        """(total ms, launches) of one kernel family since profile(True)."""
        ms, n = C.c_double(), C.c_int64()
        self._chk(self._L.lrt_profile_read(self.h, KERNELS[kernel], C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # -- conveniences over torch buffers --------------------------------------
    def coeffs_torch(self, band: int, precision: int, device="cuda:0"):
        """Allocate eta/kappa(/escale) on the device and run lrt_coeffs."""
        import torch
        nc = self.sizes()["n_cells"]
        nb = self.band_len(band)
        dt = torch.float64 if precision == LRT_FP64 else torch.float32
        eta = torch.empty((nc, nb), dtype=dt, device=device)
        kap = torch.empty((nc, nb), dtype=dt, device=device)
        esc = torch.zeros((nc, 2), dtype=torch.int32, device=device)
        self.coeffs(band, precision, eta, kap, esc if precision == LRT_FP32_COMP else None)
        return eta, kap, esc


LRT_E_NOT_READY = 5


class Server:
    """Serving loop on a context whose species, lines and grid are set."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 64):
        self._L = lib()
        self.ctx = ctx
        h = _vp()
        s = self._L.lrt_server_start(ctx.h, int(budget_bytes), int(max_slots), C.byref(h))
        if s != 0:
            raise LrtError(s, self._L.lrt_last_error(ctx.h).decode())
        self.h = h
        self._windows = {}

    def _err(self, s):
        raise LrtError(s, self._L.lrt_last_error(None).decode())

    def submit(self, req, keep_spectrum: bool = False, T_far: float = 0.0,
               scheme: int = 0) -> int:
        """req: synth.LosRequest; T_far > 0: a solid far boundary at that
        temperature; scheme: LRT_MARCH_CELL or LRT_MARCH_LINEAR_J.  Returns the
        ticket."""
        c = req.cells
        a = [np.ascontiguousarray(x, np.float64) for x in (c.T_tr, c.T_v, c.N, c.n_e, req.ds)]
        q = _LosRequest(a[0].shape[0], a[2].shape[1], _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]),
                        _p(a[4]), int(req.k_first), int(req.n_window), int(req.species_mask),
                        1 if keep_spectrum else 0, float(T_far), int(scheme))
        t = C.c_uint64()
        s = self._L.lrt_submit(self.h, C.byref(q), C.byref(t))
        if s != 0:
            self._err(s)
        self._windows[t.value] = int(req.n_window) if keep_spectrum else 0
        return t.value

    def _result(self, fn, ticket, *extra):
        n = self._windows.get(ticket, 0)
        spec = np.zeros(n) if n else None
        r = _LosResult()
        s = fn(self.h, C.c_uint64(ticket), *extra, C.byref(r), _p(spec) if spec is not None else None)
        if s == LRT_E_NOT_READY:
            return None
        if s != 0:
            self._err(s)
        self._windows.pop(ticket, None)
        return {"status": r.status, "I_int": r.I_int, "n_window": r.n_window,
                "queue_ms": r.queue_ms, "latency_ms": r.latency_ms, "spectrum": spec}

    def poll(self, ticket: int):
        """None while running, else the result dict."""
        return self._result(self._L.lrt_poll, ticket)

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        return self._result(self._L.lrt_wait, ticket, C.c_double(timeout_ms))

    def cancel(self, ticket: int):
        s = self._L.lrt_cancel(self.h, C.c_uint64(ticket))
        if s != 0:
            self._err(s)

    def info(self):
        v = [C.c_int64() for _ in range(4)]
        b = C.c_size_t()
        s = self._L.lrt_server_info(self.h, *[C.byref(x) for x in v], C.byref(b))
        if s != 0:
            self._err(s)
        return {"pending": v[0].value, "admitted": v[1].value, "completed": v[2].value,
                "epochs": v[3].value, "bytes_in_use": b.value}

    def stop(self):
        if getattr(self, "h", None):
            s = self._L.lrt_server_stop(self.h)
            self.h = None
            if s != 0:
                self._err(s)

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


LRT_MARCH_CELL, LRT_MARCH_LINEAR_J = 0, 1


def fibonacci_quadrature(n_los: int, n_polar: int, n_azim: int):
    """Directions [m, 3] and flux weights [m] of the Fibonacci-LOS angular
    rule (host only)."""
    L = lib()
    dirs = np.zeros((n_los, 3))
    w = np.zeros(n_los)
    n = C.c_int64()
    s = L.lrt_fibonacci_quadrature(n_los, n_polar, n_azim, n_los, _p(dirs), _p(w), C.byref(n))
    if s != 0:
        raise LrtError(s, L.lrt_last_error(None).decode())
    return dirs[:n.value].copy(), w[:n.value].copy()


def trace_axi_ray(nx, nr, Lx, R, rw, mu, phi):
    """Segments (cell, ds), far -> wall, of one axisymmetric ray (host only)."""
    L = lib()
    cap = 4 * (nx + 2 * nr) + 16
    cell = np.zeros(cap, np.int32)
    ds = np.zeros(cap)
    n = C.c_int64()
    s = L.lrt_trace_axi_ray(nx, nr, Lx, R, rw, mu, phi, cap, _p(cell, _i32p), _p(ds), C.byref(n))
    if s != 0:
        raise LrtError(s, L.lrt_last_error(None).decode())
    return cell[:n.value].copy(), ds[:n.value].copy()


def scaled_to_f64(eta, kappa, escale):
    """Host FP64 values of a single-precision result: stored * 2^escale."""
    e = eta.double().cpu().numpy()
    k = kappa.double().cpu().numpy()
    s = escale.cpu().numpy().astype(np.int64)
    return np.ldexp(e, s[:, :1]), np.ldexp(k, s[:, 1:2])


PROBES = {"fma_f32": 0, "fma_f64": 1, "exp_f32": 2, "log_f32": 3, "rcp_f32": 4, "mix_f32": 5,
          "copy": 6}


def probe(kind: str, device: int = 0):
    """(rate, ms) of one throughput probe (lrt_probe): lane-ops/s for the
    arithmetic kinds, bytes read + written per second for the copy."""
    rate, ms = C.c_double(), C.c_double()
    s = lib().lrt_probe(device, PROBES[kind], C.byref(rate), C.byref(ms))
    if s != 0:
        raise LrtError(s, "lrt_probe(%s) failed" % kind)
    return rate.value, ms.value
