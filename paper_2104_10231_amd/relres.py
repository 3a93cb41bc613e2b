"""Thin Python binding of the RelRes C ABI (include/relres.h).

Argument marshalling only: every step of the hot path runs in the HIP library
``librelres_hip.so`` built in-tree for gfx950.  PyTorch provides device memory
and the current stream.  There is no CPU fallback: without the built library,
or without a GPU, constructing :class:`RelRes` raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librelres_hip.so")

RELRES_OK = 0
RELRES_ERR_LIST_RETRY = -10
RELRES_ERR_STALE_LISTS = -11
RELRES_ERR_EW_TIMEOUT = -12
RELRES_WARN_DANGEROUS_BUILD = 1
FTM2V_REAL = 4.184e-4          # (kcal/mol/A) / amu -> A/fs^2
KB_REAL = 0.0019872067         # kcal/mol/K
MIX_GEOMETRIC = 0
MIX_ARITHMETIC = 1
MIX_SIXTHPOWER = 2
LIST_ATOM = 0
LIST_SITE = 1

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [("rs_in", ctypes.c_double), ("rs_out", ctypes.c_double),
                ("rc_in", ctypes.c_double), ("rc_out", ctypes.c_double),
                ("skin", ctypes.c_double), ("ntypes", ctypes.c_int),
                ("eps_fg", _c_double_p), ("sig_fg", _c_double_p),
                ("eps_cg", _c_double_p), ("sig_cg", _c_double_p),
                ("mix", ctypes.c_int), ("precision", ctypes.c_int),
                ("pair_math", ctypes.c_int), ("no_shift", ctypes.c_int),
                ("cut_type", _c_double_p), ("cut_pair", _c_double_p)]


class Stats(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_longlong), ("n_sites", ctypes.c_longlong),
                ("atom_entries", ctypes.c_longlong), ("site_entries", ctypes.c_longlong),
                ("atom_max_row", ctypes.c_int), ("site_max_row", ctypes.c_int),
                ("atom_capacity", ctypes.c_int), ("site_capacity", ctypes.c_int),
                ("atom_cells", ctypes.c_int * 3), ("site_cells", ctypes.c_int * 3),
                ("builds", ctypes.c_longlong), ("regrows", ctypes.c_longlong),
                ("box", ctypes.c_double * 3), ("generation", ctypes.c_longlong),
                ("dangerous_builds", ctypes.c_longlong),
                ("moved_at_last_build", ctypes.c_longlong),
                ("place_launches", ctypes.c_int)]


class Tune(ctypes.Structure):
    _fields_ = [("rows_atom", ctypes.c_int), ("rows_site", ctypes.c_int),
                ("cand_per_lane", ctypes.c_int), ("lanes_atom", ctypes.c_int),
                ("lanes_site", ctypes.c_int), ("trials", ctypes.c_int),
                ("build_us", ctypes.c_double), ("build_us_auto", ctypes.c_double),
                ("force_us", ctypes.c_double), ("force_us_auto", ctypes.c_double),
                ("cell_div_atom", ctypes.c_int), ("cell_div_site", ctypes.c_int)]


# exported symbol -> (restype, argtypes); mirrors include/relres.h
SIGNATURES = {
    "relres_abi_version": (ctypes.c_int, []),
    "relres_mix_distance": (ctypes.c_double, [ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "relres_cg_site_params": (ctypes.c_int, [ctypes.c_int, _c_double_p, _c_double_p, _c_double_p,
                                             _c_double_p]),
    "relres_cg_pair_params": (ctypes.c_int, [ctypes.c_int, _c_double_p, _c_double_p, _c_double_p,
                                             _c_double_p]),
    "relres_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "relres_last_error": (ctypes.c_char_p, []),
    "relres_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_void_p)]),
    "relres_set_topology": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "relres_build_lists": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_double_p,
                                          ctypes.c_void_p]),
    "relres_build_lists_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_double_p,
                                                ctypes.c_void_p]),
    "relres_check_lists": (ctypes.c_int, [ctypes.c_void_p]),
    "relres_sync": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "relres_moved_atoms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int)]),
    "relres_forces": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "relres_forces_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "relres_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "relres_set_list_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int]),
    "relres_set_cells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "relres_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_double_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Tune)]),
    "relres_set_systems": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "relres_set_skins": (ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    "relres_set_pair_params": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p,
                                              _c_double_p, _c_double_p]),
    "relres_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "relres_set_type_params": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p,
                                              _c_double_p, _c_double_p]),
    "relres_backward_types": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "relres_list_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "relres_generation": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]),
    "relres_get_pairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]),
    "relres_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "relres_get_timing": (ctypes.c_int, [ctypes.c_void_p, _c_double_p,
                                         ctypes.POINTER(ctypes.c_longlong), _c_double_p,
                                         ctypes.POINTER(ctypes.c_longlong)]),
    "relres_set_bonded": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, _c_double_p,
                                         _c_double_p, ctypes.c_int, ctypes.c_void_p, _c_double_p,
                                         _c_double_p, ctypes.c_int, ctypes.c_void_p, _c_double_p,
                                         ctypes.c_void_p, _c_double_p, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_double]),
    "relres_bonded_forces": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "relres_md_setup": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    "relres_md_state": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p, ctypes.c_int]),
    "relres_md_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "relres_destroy": (None, [ctypes.c_void_p]),
}

_LIB = None


class RelResError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load the built HIP library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"RelRes HIP library not built: {path} missing "
                          "(run __graft_entry__.build() or paper_2104_10231_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(rc: int, where: str):
    if rc != RELRES_OK:
        lib = load_library()
        raise RelResError(rc, where, lib.relres_last_error().decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a) -> Optional[int]:
    return None if a is None else a.ctypes.data


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_c_double_p)


def cg_site_params(eps_fg, sig_fg):
    """Eq. 15: (eps_CG, sigma_CG) of one CG site from the FG parameters of the
    sites it groups (geometric FG mixing).  Host computation in the library."""
    e, sg = _f64(eps_fg).ravel(), _f64(sig_fg).ravel()
    if e.shape != sg.shape:
        raise ValueError("eps_fg and sig_fg differ in length")
    eo, so = ctypes.c_double(), ctypes.c_double()
    _check(load_library().relres_cg_site_params(int(e.shape[0]), _dp(e), _dp(sg),
                                                ctypes.byref(eo), ctypes.byref(so)),
           "relres_cg_site_params")
    return eo.value, so.value


def cg_pair_params(eps_mn, sig_mn):
    """Eq. 13: (eps_CG, sigma_CG) of a pair of CG sites from the FG pair
    parameters of every mu-nu pair between them (any mixing)."""
    e, sg = _f64(eps_mn).ravel(), _f64(sig_mn).ravel()
    if e.shape != sg.shape:
        raise ValueError("eps_mn and sig_mn differ in length")
    eo, so = ctypes.c_double(), ctypes.c_double()
    _check(load_library().relres_cg_pair_params(int(e.shape[0]), _dp(e), _dp(sg),
                                                ctypes.byref(eo), ctypes.byref(so)),
           "relres_cg_pair_params")
    return eo.value, so.value


def mix_distance(mix: int, a: float, b: float) -> float:
    """Distance of an unlike type pair mixed from two per-type values."""
    return float(load_library().relres_mix_distance(int(mix), float(a), float(b)))


class RelRes:
    """One RelRes LJ evaluator bound to the current GPU.

    Parameters follow Sec. 2.5 of the paper (pair_style lj/relres r_s- r_s+
    r_c- r_c+ with per-type FG/CG epsilon and sigma); ``eps_cg == 0`` marks an
    ordinary type.  ``precision`` is the force type (32 or 64), ``pair_math``
    the type of the per-pair terms (0 = same as precision).  ``shift`` is
    pair_modify shift yes/no; ``cut_type`` (ntypes x 4) or ``cut_pair``
    (ntypes x ntypes x 4) give r_s-, r_s+, r_c-, r_c+ per type (mixed for
    unlike types with the sigma rule) or per type pair.
    """

    def __init__(self, *, rs_in: float, rs_out: float, rc_in: float, rc_out: float,
                 skin: float, eps_fg: Sequence[float], sig_fg: Sequence[float],
                 eps_cg: Sequence[float], sig_cg: Sequence[float], mix: int = MIX_GEOMETRIC,
                 precision: int = 32, pair_math: int = 0, shift: bool = True,
                 cut_type=None, cut_pair=None):
        if not torch.cuda.is_available():
            raise RuntimeError("RelRes needs a ROCm GPU; none is visible")
        self._lib = load_library()
        self._arrays = [_f64(eps_fg), _f64(sig_fg), _f64(eps_cg), _f64(sig_cg)]
        nt = len(self._arrays[0])
        ct = None if cut_type is None else _f64(cut_type).reshape(nt, 4)
        cp = None if cut_pair is None else _f64(cut_pair).reshape(nt, nt, 4)
        self._cuts = [ct, cp]
        p = Params(rs_in, rs_out, rc_in, rc_out, skin, nt,
                   *[a.ctypes.data_as(_c_double_p) for a in self._arrays],
                   int(mix), int(precision), int(pair_math), 0 if shift else 1,
                   None if ct is None else _dp(ct), None if cp is None else _dp(cp))
        ctx = ctypes.c_void_p()
        torch.cuda.init()
        _check(self._lib.relres_create(ctypes.byref(p), ctypes.byref(ctx)), "relres_create")
        self._ctx = ctx
        self.precision = int(precision)
        self.ntypes = nt
        self.mix = int(mix)
        self.hybrid = [float(x) > 0.0 for x in self._arrays[2]]
        self.n = 0
        self.last_check_dangerous = False   # set by check_lists()
        self.device = torch.device("cuda", torch.cuda.current_device())

    # -- topology ----------------------------------------------------------
    def set_topology(self, types, mol=None, exclude_same_mol: bool = True,
                     excl_offsets=None, excl_idx=None):
        t = _i32(types)
        m = _i32(mol)
        eo = _i32(excl_offsets) if excl_idx is not None and len(excl_idx) else None
        ei = _i32(excl_idx) if eo is not None else None
        _check(self._lib.relres_set_topology(self._ctx, int(t.shape[0]), _ptr(t), _ptr(m),
                                             int(bool(exclude_same_mol)), _ptr(eo), _ptr(ei)),
               "relres_set_topology")
        self.n = int(t.shape[0])
        self.nsys = 1

    def set_systems(self, atom_offsets):
        """Atoms [off[s], off[s+1]) form system s; one box per system."""
        off = _i32(atom_offsets)
        _check(self._lib.relres_set_systems(self._ctx, int(off.shape[0] - 1), _ptr(off)),
               "relres_set_systems")
        self.nsys = int(off.shape[0] - 1)

    def set_skins(self, skins):
        """Skin of every system (nsys values), in place of the context's skin;
        build the lists again afterwards."""
        sk = _f64(skins).reshape(-1)
        if sk.shape[0] != self.nsys:
            raise ValueError(f"need {self.nsys} skins, got {sk.shape[0]}")
        _check(self._lib.relres_set_skins(self._ctx, sk.ctypes.data_as(_c_double_p)),
               "relres_set_skins")

    # -- hot path ------------------------------------------------------------
    def _pos(self, pos: torch.Tensor) -> torch.Tensor:
        if pos.dtype != torch.float64 or pos.device.type != "cuda" or not pos.is_contiguous():
            raise TypeError("pos must be a contiguous float64 CUDA tensor of shape (N, 3)")
        if tuple(pos.shape) != (self.n, 3):
            raise ValueError(f"pos has shape {tuple(pos.shape)}, expected ({self.n}, 3)")
        return pos

    def build_lists(self, pos: torch.Tensor, box, stream=None, wait: bool = True) -> bool:
        """Build both lists.  With wait=False the build is only enqueued; call
        check_lists() before trusting results computed from these lists.

        Returns True when the (waited-for) build found atoms more than half
        the skin from their positions at the previous build
        (RELRES_WARN_DANGEROUS_BUILD: lists used before it were kept too long)."""
        pos = self._pos(pos)
        bx = np.asarray(box, dtype=np.float64).reshape(-1)
        if bx.shape[0] != 3 * self.nsys:
            raise ValueError(f"box needs {3 * self.nsys} values ({self.nsys} systems x 3)")
        b = (ctypes.c_double * bx.shape[0])(*bx.tolist())
        fn = self._lib.relres_build_lists if wait else self._lib.relres_build_lists_async
        rc = fn(self._ctx, pos.data_ptr() if self.n else None, b, _stream(stream))
        if rc == RELRES_WARN_DANGEROUS_BUILD:
            return True
        _check(rc, "relres_build_lists" if wait else "relres_build_lists_async")
        return False

    def check_lists(self) -> bool:
        """True when the last build's lists are complete; False when a row
        overflowed (capacity grown: build again and redo what used them)."""
        rc = self._lib.relres_check_lists(self._ctx)
        if rc == RELRES_ERR_LIST_RETRY:
            return False
        self.last_check_dangerous = rc == RELRES_WARN_DANGEROUS_BUILD
        if not self.last_check_dangerous:
            _check(rc, "relres_check_lists")
        return True

    def sync(self, stream=None):
        """Wait for the stream; raises if a force call's energy/virial wait
        gave up since the last report (relres_sync)."""
        _check(self._lib.relres_sync(self._ctx, _stream(stream)), "relres_sync")

    def moved_atoms(self, pos: torch.Tensor, stream=None) -> int:
        """Atoms of pos more than half the skin from their positions at the
        last build (0: the lists are still exact).  Waits for the result."""
        pos = self._pos(pos)
        n = ctypes.c_int()
        _check(self._lib.relres_moved_atoms(self._ctx, pos.data_ptr() if self.n else None,
                                            _stream(stream), ctypes.byref(n)),
               "relres_moved_atoms")
        return n.value

    def forces(self, pos: torch.Tensor, out: Optional[torch.Tensor] = None,
               energy: Optional[torch.Tensor] = None, virial: Optional[torch.Tensor] = None,
               want_energy: bool = True, want_virial: bool = True, stream=None):
        """Return (forces, energy[3], virial[6]); outputs may be given to reuse."""
        pos = self._pos(pos)
        dt = torch.float64 if self.precision == 64 else torch.float32
        if out is None:
            out = torch.empty((self.n, 3), dtype=dt, device=pos.device)
        elif out.dtype != dt or tuple(out.shape) != (self.n, 3) or not out.is_contiguous():
            raise TypeError("out must be a contiguous (N, 3) tensor of the force dtype")
        eshape = (3,) if self.nsys == 1 else (self.nsys, 3)
        wshape = (6,) if self.nsys == 1 else (self.nsys, 6)
        if want_energy and energy is None:
            energy = torch.empty(eshape, dtype=torch.float64, device=pos.device)
        if want_virial and virial is None:
            virial = torch.empty(wshape, dtype=torch.float64, device=pos.device)
        for t, n in ((energy, 3), (virial, 6)):
            if t is not None and (t.numel() != n * self.nsys or not t.is_contiguous()):
                raise ValueError(f"energy/virial buffers need {n} x nsys contiguous doubles")
        _check(self._lib.relres_forces(self._ctx, pos.data_ptr() if self.n else None,
                                       out.data_ptr() if self.n else None,
                                       energy.data_ptr() if energy is not None else None,
                                       virial.data_ptr() if virial is not None else None,
                                       _stream(stream)), "relres_forces")
        return out, energy, virial

    def forces_noalloc(self, pos: torch.Tensor, out: torch.Tensor,
                       energy: Optional[torch.Tensor] = None,
                       virial: Optional[torch.Tensor] = None, stream=None):
        """relres_forces_noalloc: the caller passes every output (nothing is
        allocated here or in the library); energy/virial may be None."""
        pos = self._pos(pos)
        dt = torch.float64 if self.precision == 64 else torch.float32
        if out.dtype != dt or tuple(out.shape) != (self.n, 3) or not out.is_contiguous():
            raise TypeError("out must be a contiguous (N, 3) tensor of the force dtype")
        for t, n in ((energy, 3), (virial, 6)):
            if t is not None and (t.numel() != n * self.nsys or not t.is_contiguous()
                                  or t.dtype != torch.float64):
                raise ValueError(f"energy/virial buffers need {n} x nsys contiguous doubles")
        _check(self._lib.relres_forces_noalloc(
            self._ctx, pos.data_ptr() if self.n else None, out.data_ptr() if self.n else None,
            energy.data_ptr() if energy is not None else None,
            virial.data_ptr() if virial is not None else None, _stream(stream)),
            "relres_forces_noalloc")
        return out, energy, virial

    # -- parameters and gradients -------------------------------------------------
    def set_pair_params(self, eps_fg, sig_fg, eps_cg, sig_cg):
        """Pair tables (ntypes x ntypes each, host arrays or CPU tensors)."""
        arrs = []
        for t in (eps_fg, sig_fg, eps_cg, sig_cg):
            if isinstance(t, torch.Tensor):
                t = t.detach().cpu().numpy()
            a = _f64(t)
            if a.shape != (self.ntypes, self.ntypes):
                raise ValueError(f"pair table shape {a.shape}, expected {(self.ntypes,) * 2}")
            arrs.append(a)
        _check(self._lib.relres_set_pair_params(self._ctx,
                                                *[a.ctypes.data_as(_c_double_p) for a in arrs]),
               "relres_set_pair_params")
        self._installed_params = None       # the tables no longer come from per-type values

    def set_type_params(self, eps_fg, sig_fg, eps_cg, sig_cg):
        """Per-type parameters (ntypes each, host arrays or CPU tensors),
        mixed again by the library."""
        arrs = []
        for t in (eps_fg, sig_fg, eps_cg, sig_cg):
            if isinstance(t, torch.Tensor):
                t = t.detach().cpu().numpy()
            a = _f64(t)
            if a.shape != (self.ntypes,):
                raise ValueError(f"per-type array shape {a.shape}, expected ({self.ntypes},)")
            arrs.append(a)
        _check(self._lib.relres_set_type_params(self._ctx,
                                                *[a.ctypes.data_as(_c_double_p) for a in arrs]),
               "relres_set_type_params")
        self._installed_params = None

    def _grad_args(self, pos, grad_forces, grad_energy):
        gf = None
        if grad_forces is not None:
            gf = grad_forces.to(dtype=torch.float64).contiguous()
            if tuple(gf.shape) != (self.n, 3) or gf.device != pos.device:
                raise ValueError("grad_forces must be an (N, 3) tensor on the positions' device")
        ge = None
        if grad_energy is not None:
            ge = grad_energy.to(device=pos.device, dtype=torch.float64).reshape(-1).contiguous()
            if ge.numel() != self.nsys:
                raise ValueError(f"grad_energy needs {self.nsys} values (one per system)")
        gpos = torch.empty((self.n, 3), dtype=torch.float64, device=pos.device)
        return (pos.data_ptr() if self.n else None,
                gf.data_ptr() if gf is not None and self.n else None,
                ge.data_ptr() if ge is not None else None,
                gpos.data_ptr() if self.n else None), gpos, (gf, ge)

    def backward_types(self, pos: torch.Tensor, grad_forces: Optional[torch.Tensor] = None,
                       grad_energy: Optional[torch.Tensor] = None, stream=None):
        """dJ/dx (N, 3) and dJ/d(per-type parameter) (4, ntypes) for
        J = e_bar E + sum g.F (relres_backward_types)."""
        pos = self._pos(pos)
        ptrs, gpos, keep = self._grad_args(pos, grad_forces, grad_energy)
        gtype = torch.empty((4, self.ntypes), dtype=torch.float64, device=pos.device)
        _check(self._lib.relres_backward_types(self._ctx, *ptrs, gtype.data_ptr(),
                                               _stream(stream)), "relres_backward_types")
        return gpos, gtype

    def backward(self, pos: torch.Tensor, grad_forces: Optional[torch.Tensor] = None,
                 grad_energy: Optional[torch.Tensor] = None, stream=None):
        """dJ/dx (N, 3) and dJ/dP (4, ntypes, ntypes) for J = e_bar E + sum g.F."""
        pos = self._pos(pos)
        ptrs, gpos, keep = self._grad_args(pos, grad_forces, grad_energy)
        gpair = torch.empty((4, self.ntypes, self.ntypes), dtype=torch.float64, device=pos.device)
        _check(self._lib.relres_backward(self._ctx, *ptrs, gpair.data_ptr(), _stream(stream)),
               "relres_backward")
        return gpos, gpair

    # -- inspection ------------------------------------------------------------
    def set_launch(self, lanes_atom: int = 0, lanes_site: int = 0):
        _check(self._lib.relres_set_launch(self._ctx, int(lanes_atom), int(lanes_site)),
               "relres_set_launch")

    def set_cells(self, div_atom: int = 0, div_site: int = 0):
        """Cells per list radius of the atom and site grids (1 or 2; 0 =
        automatic) for the next builds."""
        _check(self._lib.relres_set_cells(self._ctx, int(div_atom), int(div_site)),
               "relres_set_cells")

    def set_list_launch(self, rows_atom: int = 0, rows_site: int = 0, cand_per_lane: int = 0):
        """List-kernel shape for the next builds (0 = automatic)."""
        _check(self._lib.relres_set_list_launch(self._ctx, int(rows_atom), int(rows_site),
                                                int(cand_per_lane)), "relres_set_list_launch")

    def autotune(self, pos: torch.Tensor, box, reps: int = 3, stream=None) -> dict:
        """Time every list-kernel and force-kernel shape on these positions and
        box(es), keep the fastest (lists rebuilt from pos); returns the choice
        and the mean device times (us) of the chosen and automatic shapes."""
        pos = self._pos(pos)
        bx = np.asarray(box, dtype=np.float64).reshape(-1)
        if bx.shape[0] != 3 * self.nsys:
            raise ValueError(f"box needs {3 * self.nsys} values ({self.nsys} systems x 3)")
        b = (ctypes.c_double * bx.shape[0])(*bx.tolist())
        t = Tune()
        _check(self._lib.relres_autotune(self._ctx, pos.data_ptr() if self.n else None, b,
                                         _stream(stream), int(reps), ctypes.byref(t)),
               "relres_autotune")
        return {k: getattr(t, k) for k, _ in Tune._fields_}

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.relres_list_stats(self._ctx, ctypes.byref(s)), "relres_list_stats")
        d = {k: getattr(s, k) for k, _ in Stats._fields_}
        for k in ("atom_cells", "site_cells", "box"):
            d[k] = list(d[k])
        return d

    def generation(self) -> int:
        """Buffer generation: a captured graph stays valid while it is unchanged."""
        g = ctypes.c_longlong()
        _check(self._lib.relres_generation(self._ctx, ctypes.byref(g)), "relres_generation")
        return g.value

    def pairs(self, which: int) -> np.ndarray:
        n = ctypes.c_longlong()
        _check(self._lib.relres_get_pairs(self._ctx, int(which), None, 0, ctypes.byref(n)),
               "relres_get_pairs")
        out = np.zeros((max(1, n.value), 2), np.int32)
        _check(self._lib.relres_get_pairs(self._ctx, int(which), out.ctypes.data, n.value,
                                          ctypes.byref(n)), "relres_get_pairs")
        return out[: n.value]

    def set_timing(self, enable: bool = True):
        _check(self._lib.relres_set_timing(self._ctx, int(bool(enable))), "relres_set_timing")

    def timing(self) -> dict:
        fm, bm = ctypes.c_double(), ctypes.c_double()
        fc, bc = ctypes.c_longlong(), ctypes.c_longlong()
        _check(self._lib.relres_get_timing(self._ctx, ctypes.byref(fm), ctypes.byref(fc),
                                           ctypes.byref(bm), ctypes.byref(bc)), "relres_get_timing")
        return dict(force_ms=fm.value, force_calls=fc.value, build_ms=bm.value,
                    build_calls=bc.value)

    # -- molecular model and dynamics -----------------------------------------
    def set_bonded(self, bonded: dict):
        """Bonds, angles, dihedrals and scaled 1-4 pairs (keys as in
        ``workloads.hexane_liquid``)."""
        b = bonded
        arr = dict(bonds=_i32(b["bonds"]), bond_k=_f64(b["bond_k"]), bond_r0=_f64(b["bond_r0"]),
                   angles=_i32(b["angles"]), angle_k=_f64(b["angle_k"]), angle_t0=_f64(b["angle_t0"]),
                   dihedrals=_i32(b["dihedrals"]), dih_k=_f64(b["dih_k"]), dih_n=_i32(b["dih_n"]),
                   dih_d=_f64(b["dih_d"]), pairs14=_i32(b["pairs14"]))
        self._bonded = arr
        _check(self._lib.relres_set_bonded(
            self._ctx, len(arr["bond_k"]), _ptr(arr["bonds"]), _dp(arr["bond_k"]), _dp(arr["bond_r0"]),
            len(arr["angle_k"]), _ptr(arr["angles"]), _dp(arr["angle_k"]), _dp(arr["angle_t0"]),
            len(arr["dih_k"]), _ptr(arr["dihedrals"]), _dp(arr["dih_k"]), _ptr(arr["dih_n"]),
            _dp(arr["dih_d"]), len(arr["pairs14"]), _ptr(arr["pairs14"]), float(b["scale14"])),
            "relres_set_bonded")

    def bonded_forces(self, pos: torch.Tensor, forces: torch.Tensor, want_energy: bool = True,
                      stream=None):
        """Add the bonded and 1-4 forces to ``forces``; returns (energy[4],
        virial[6]) device tensors (None when not wanted)."""
        pos = self._pos(pos)
        E = torch.empty(4, dtype=torch.float64, device=pos.device) if want_energy else None
        W = torch.empty(6, dtype=torch.float64, device=pos.device) if want_energy else None
        _check(self._lib.relres_bonded_forces(self._ctx, pos.data_ptr() if self.n else None,
                                              forces.data_ptr() if self.n else None,
                                              E.data_ptr() if E is not None else None,
                                              W.data_ptr() if W is not None else None,
                                              _stream(stream)), "relres_bonded_forces")
        return E, W

    def md_setup(self, masses, dt: float, temperature: float, tau: float,
                 rebuild_every: int = 10, kB: float = KB_REAL, ftm2v: float = FTM2V_REAL):
        """Nose-Hoover velocity Verlet (defaults: kcal/mol, A, amu, fs, K)."""
        m = _f64(masses)
        self._masses = m
        _check(self._lib.relres_md_setup(self._ctx, _dp(m), float(dt), float(kB * temperature),
                                         float(tau), float(ftm2v), int(rebuild_every)),
               "relres_md_setup")

    def md_state(self, xi: Optional[float] = None, eta: Optional[float] = None):
        """Return (xi, eta); set them when both are given."""
        a, b = ctypes.c_double(xi or 0.0), ctypes.c_double(eta or 0.0)
        setting = xi is not None and eta is not None
        _check(self._lib.relres_md_state(self._ctx, ctypes.byref(a), ctypes.byref(b), int(setting)),
               "relres_md_state")
        return a.value, b.value

    def md_run(self, pos: torch.Tensor, vel: torch.Tensor, nsteps: int, thermo_every: int = 0,
               stream=None):
        """Advance ``pos`` and ``vel`` (float64 (N, 3) CUDA tensors) in
        place; returns the thermo rows (nsteps // thermo_every, 8) or None."""
        pos = self._pos(pos)
        vel = self._pos(vel)
        rows = nsteps // thermo_every if thermo_every > 0 else 0
        th = torch.empty((max(rows, 1), 8), dtype=torch.float64, device=pos.device)
        _check(self._lib.relres_md_run(self._ctx, pos.data_ptr(), vel.data_ptr(), int(nsteps),
                                       int(thermo_every), th.data_ptr() if rows else None,
                                       _stream(stream)), "relres_md_run")
        return th[:rows] if rows else None

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.relres_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
