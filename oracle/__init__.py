"""FP64 CPU oracle for the RelRes Lennard-Jones hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg; never by the product path.  It shares no code
with the HIP library.  The arithmetic lives in ``relres_oracle.c`` (plain C,
FP64, no FMA contraction); this module only marshals numpy arrays.

Every function follows a passage of arXiv:2104.10231:
  setup_table   -- mixing (Sec. 2.3, Sec. 2.5 mix keyword), per-type-pair
                   distances (Sec. 2.5, Sec. 3.4), Eq. 14, Eqs. 7/8 solved
                   numerically, Eq. 9 with the Sec. 2.5 shift keyword
  pair          -- Eq. 20, case by case
  compute       -- Eq. 3 energy, forces, pair virial (brute force, all pairs)
  pairs         -- the two neighbour pair sets (Sec. 2.6 lists)
  grad          -- gradient of e_bar E + sum_i g_i . F_i with respect to the
                   per-type parameters and the positions (Eqs. 7-9 and 20
                   differentiated; the systems of Eqs. 7/8 are linear)
  bonded        -- bonds, angles and Fourier dihedrals of the paper's
                   simulations (Sec. 3.2), in md_oracle.c
  pairs14       -- the 1-4 pairs: Eq. 20 scaled (Sec. 3.2)
  nvt_run       -- velocity Verlet with a Nose-Hoover thermostat (the
                   canonical ensemble of Sec. 3.2), all forces from the above
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
REC = 27   # doubles per type-pair record
# record field offsets
EPS_FG, SIG_FG, EPS_CG, SIG_CG, FG_SM, CG_SP, CG_CM, G_CM, G_SP, G_SM = 0, 1, 2, 3, 4, 9, 14, 19, 20, 21
CUT, G_OUT = 22, 26   # the pair's r_s-, r_s+, r_c-, r_c+; constant of Eq. 20 cases 3-4

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_record_size.restype = ctypes.c_int
        L.oracle_lj.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _d]
        L.oracle_solve_poly.argtypes = [ctypes.c_int, ctypes.c_double, _d, _d]
        L.oracle_solve_poly.restype = ctypes.c_int
        L.oracle_setup.argtypes = [ctypes.c_int, _d, _d, _d, _d, ctypes.c_int, _d,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _d]
        L.oracle_setup.restype = ctypes.c_int
        L.oracle_pair_vec.argtypes = [_d, ctypes.c_int, _d, _d, _d,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_wrap.argtypes = [ctypes.c_int, _d, _d, _d]
        L.oracle_compute.argtypes = [ctypes.c_int, _d, _d, _i, _i, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _d,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     _d, _d, _d]
        L.oracle_compute.restype = ctypes.c_int
        L.oracle_pairs.argtypes = [ctypes.c_int, _d, _d, _i, _i, _i, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]
        L.oracle_pairs.restype = ctypes.c_long
        L.oracle_grad.argtypes = [ctypes.c_int, _d, _d, _i, _i, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _d, _d, _d, _d,
                                  ctypes.c_int, _d, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                  _d, ctypes.c_double, _d, _d]
        L.oracle_grad.restype = ctypes.c_int
        L.oracle_bonded.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, _i, _d, _d,
                                    ctypes.c_int, _i, _d, _d, ctypes.c_int, _i, _d, _i, _d,
                                    _d, _d, _d]
        L.oracle_dihedral_angle.argtypes = [_d, _d, _d, _d, _d]
        L.oracle_dihedral_angle.restype = ctypes.c_double
        L.oracle_pairs14.argtypes = [_d, _d, _i, ctypes.c_int, _d, ctypes.c_int, _i,
                                     ctypes.c_double, _d, _d, _d]
        assert L.oracle_record_size() == REC
        _LIB = L
    return _LIB


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def cutoffs(sys) -> np.ndarray:
    """The global distances r_s-, r_s+, r_c-, r_c+."""
    return np.array([sys.rs_in, sys.rs_out, sys.rc_in, sys.rc_out], np.float64)


def _cut_args(sys):
    ct = getattr(sys, "cut_type", None)
    cp = getattr(sys, "cut_pair", None)
    ct = None if ct is None else _f64(ct).reshape(sys.ntypes, 4)
    cp = None if cp is None else _f64(cp).reshape(sys.ntypes, sys.ntypes, 4)
    return ct, cp, int(bool(getattr(sys, "shift", True)))


def lj(eps, sig, r):
    """u, u', u'' of Eq. 11/12 at distance r."""
    out = np.zeros(3)
    lib().oracle_lj(float(eps), float(sig), float(r), out)
    return out


def solve_poly(kind: int, dr: float, u3) -> np.ndarray:
    """Smoothing-polynomial coefficients from Eq. 7 (kind 0) or Eq. 8 (kind 1)."""
    g = np.zeros(5)
    rc = lib().oracle_solve_poly(int(kind), float(dr), _f64(u3), g)
    if rc:
        raise ValueError("singular boundary-condition system")
    return g


def setup_table(sys) -> np.ndarray:
    """(ntypes, ntypes, REC) table of mixed parameters, distances, gammas and
    Gammas."""
    nt = sys.ntypes
    tab = np.zeros(nt * nt * REC)
    ct, cp, shift = _cut_args(sys)
    rc = lib().oracle_setup(nt, _f64(sys.eps_fg), _f64(sys.sig_fg), _f64(sys.eps_cg),
                            _f64(sys.sig_cg), int(sys.mix), cutoffs(sys), _ptr(ct), _ptr(cp),
                            shift, tab)
    if rc == -1:
        raise ValueError("cutoffs must satisfy r_s- <= r_s+ <= r_c- <= r_c+")
    if rc:
        raise ValueError("singular boundary-condition system")
    return tab.reshape(nt, nt, REC)


def pair(rec, r):
    """Eq. 20 for distances r with one record (its own distances): returns
    (u, du/dr, case index 1..5, e_fg, e_cg)."""
    r = _f64(np.atleast_1d(r))
    m = r.shape[0]
    u, du, efg, ecg = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)
    which = np.zeros(m, np.int32)
    lib().oracle_pair_vec(_f64(rec), m, r, u, du, _ptr(which), _ptr(efg), _ptr(ecg))
    return u, du, which, efg, ecg


def wrap(pos, box):
    pos = _f64(pos)
    out = np.zeros_like(pos)
    lib().oracle_wrap(pos.shape[0], pos, _f64(box), out)
    return out


def _excl(sys):
    if sys.excl_idx is None or len(sys.excl_idx) == 0:
        return None, None
    return _i32(sys.excl_offsets), _i32(sys.excl_idx)


def compute(sys, pos=None, nthreads: int = 0, sel=None, table=None):
    """Forces (N,3), energy {total, FG, CG} and virial {xx,yy,zz,xy,xz,yz}.

    With ``sel`` (atom indices) only those atoms' forces are computed and
    returned (len(sel), 3); E and W are then None.
    """
    pos = _f64(sys.pos if pos is None else pos)
    tab = setup_table(sys) if table is None else table
    eo, ei = _excl(sys)
    n = pos.shape[0]
    if sel is not None:
        sel = _i32(sel)
        F = np.zeros((len(sel), 3))
    else:
        F = np.zeros((n, 3))
    E, W = np.zeros(3), np.zeros(6)
    rc = lib().oracle_compute(n, pos, _f64(sys.box), _i32(sys.types), _i32(sys.mol),
                              int(bool(sys.exclude_same_mol)), _ptr(eo), _ptr(ei),
                              sys.ntypes, _f64(tab.reshape(-1)),
                              int(nthreads), 0 if sel is None else len(sel), _ptr(sel),
                              F, E, W)
    if rc:
        raise MemoryError("oracle_compute failed")
    if sel is not None:
        return F, None, None
    return F, E, W


def grad(sys, g, e_bar: float = 0.0, pos=None):
    """Gradient of J = e_bar * E + sum_i g_i . F_i.

    Returns (dtheta, dpos): dtheta is (4, ntypes) for per-type eps_FG, sigma_FG,
    eps_CG, sigma_CG (CG rows zero for ordinary types), dpos is (N, 3).
    """
    pos = _f64(sys.pos if pos is None else pos)
    n = pos.shape[0]
    eo, ei = _excl(sys)
    dtheta = np.zeros(4 * sys.ntypes)
    dpos = np.zeros((n, 3))
    ct, cp, shift = _cut_args(sys)
    rc = lib().oracle_grad(n, pos, _f64(sys.box), _i32(sys.types), _i32(sys.mol),
                           int(bool(sys.exclude_same_mol)), _ptr(eo), _ptr(ei), sys.ntypes,
                           _f64(sys.eps_fg), _f64(sys.sig_fg), _f64(sys.eps_cg), _f64(sys.sig_cg),
                           int(sys.mix), cutoffs(sys), _ptr(ct), _ptr(cp), shift,
                           _f64(np.asarray(g).reshape(n, 3)), float(e_bar), dtheta, dpos)
    if rc:
        raise ValueError(f"oracle_grad failed ({rc})")
    return dtheta.reshape(4, sys.ntypes), dpos


def hybrid_flags(sys) -> np.ndarray:
    return (np.asarray(sys.eps_cg) > 0.0).astype(np.int32)


def list_radii(sys, table=None):
    """Outer distances the two lists are built for: the largest r_s+ over all
    type pairs, and the largest r_c+ over hybrid-hybrid pairs (over all pairs
    when there is none)."""
    tab = setup_table(sys) if table is None else table
    h = hybrid_flags(sys).astype(bool)
    hh = h[:, None] & h[None, :]
    rso = float(tab[:, :, CUT + 1].max())
    rco = float(tab[:, :, CUT + 3][hh].max()) if hh.any() else float(tab[:, :, CUT + 3].max())
    return rso, rco


def pairs(sys, which: int, pos=None, rows=None):
    """Neighbour pair set: which=0 atom list (r < largest r_s+ + skin),
    which=1 site list (hybrid pairs, r < largest hybrid r_c+ + skin).  Returns
    an (M,2) int32 array of (i, j), i < j, sorted; with ``rows`` the full
    ordered rows (i, j != i) of the selected atoms."""
    pos = _f64(sys.pos if pos is None else pos)
    eo, ei = _excl(sys)
    r_out = list_radii(sys)[which]
    n = pos.shape[0]
    rsel = None if rows is None else _i32(rows)
    args = (n, pos, _f64(sys.box), _i32(sys.types), hybrid_flags(sys), _i32(sys.mol),
            int(bool(sys.exclude_same_mol)), _ptr(eo), _ptr(ei), float(r_out),
            float(sys.skin), int(which), 0 if rsel is None else len(rsel), _ptr(rsel))
    cnt = lib().oracle_pairs(*args, None, 0)
    out = np.zeros((max(cnt, 1), 2), np.int32)
    cnt2 = lib().oracle_pairs(*args, _ptr(out), cnt)
    assert cnt2 == cnt
    return out[:cnt]


def cg_params_eq13(eps_mn, sig_mn):
    """Eq. 13: CG (sigma_ij, eps_ij) of a pair of groups from all FG pair
    parameters eps_{mu nu}, sigma_{mu nu} (any shape, summed over all pairs)."""
    e = np.asarray(eps_mn, float).ravel()
    s = np.asarray(sig_mn, float).ravel()
    a12 = np.sum(e * s ** 12)
    a6 = np.sum(e * s ** 6)
    return a12 ** (1.0 / 6.0) / a6 ** (1.0 / 6.0), a6 ** 2 / a12


def cg_params_eq15(eps_sites, sig_sites):
    """Eq. 15: per-group CG (sigma_l, eps_l) from the FG parameters of the
    group's sites, valid under geometric mixing."""
    e = np.asarray(eps_sites, float)
    s = np.asarray(sig_sites, float)
    b12 = np.sum(np.sqrt(e * s ** 12))
    b6 = np.sum(np.sqrt(e * s ** 6))
    return b12 ** (1.0 / 3.0) / b6 ** (1.0 / 3.0), b6 ** 4 / b12 ** 2


# ----------------------------------------------------------------------------
# molecular dynamics (Sec. 3.2)
# ----------------------------------------------------------------------------

FTM2V = 4.184e-4          # (kcal/mol/A) / amu -> A/fs^2
KB = 0.0019872067         # kcal/mol/K


def bonded(sys, pos=None):
    """Bonds, angles and dihedrals of ``sys.bonded``: forces (N,3), energies
    {bonds, angles, dihedrals} and virial {xx,yy,zz,xy,xz,yz}."""
    b = sys.bonded
    pos = _f64(sys.pos if pos is None else pos)
    n = pos.shape[0]
    F, E, W = np.zeros((n, 3)), np.zeros(3), np.zeros(6)
    lib().oracle_bonded(n, pos, _f64(sys.box),
                        len(b["bonds"]), _i32(b["bonds"]), _f64(b["bond_k"]), _f64(b["bond_r0"]),
                        len(b["angles"]), _i32(b["angles"]), _f64(b["angle_k"]), _f64(b["angle_t0"]),
                        len(b["dihedrals"]), _i32(b["dihedrals"]), _f64(b["dih_k"]),
                        _i32(b["dih_n"]), _f64(b["dih_d"]), F, E, W)
    return F, E, W


def dihedral_angle(xi, xj, xk, xl, box):
    return lib().oracle_dihedral_angle(_f64(xi), _f64(xj), _f64(xk), _f64(xl), _f64(box))


def pairs14(sys, pos=None, table=None):
    """The 1-4 pairs of ``sys.bonded``: Eq. 20 times ``scale14``.  Forces
    (N,3), energy {total, FG part, CG part}, virial."""
    b = sys.bonded
    pos = _f64(sys.pos if pos is None else pos)
    tab = setup_table(sys) if table is None else table
    F, E, W = np.zeros((pos.shape[0], 3)), np.zeros(3), np.zeros(6)
    p = _i32(b["pairs14"])
    lib().oracle_pairs14(pos, _f64(sys.box), _i32(sys.types), sys.ntypes, _f64(tab.reshape(-1)),
                         len(p), p, float(b["scale14"]), F, E, W)
    return F, E, W


def md_forces(sys, pos, table=None, nthreads: int = 0):
    """All forces of the molecular model: Eq. 20 over non-excluded pairs,
    scaled 1-4 pairs and bonded terms.  Returns (F, energies) with energies
    = {non-bonded (Eq. 3), 1-4 pairs, bonds, angles, dihedrals} and the
    total virial."""
    tab = setup_table(sys) if table is None else table
    F, E, W = compute(sys, pos=pos, table=tab, nthreads=nthreads)
    F14, E14, W14 = pairs14(sys, pos=pos, table=tab)
    Fb, Eb, Wb = bonded(sys, pos=pos)
    return F + F14 + Fb, np.array([E[0], E14[0], Eb[0], Eb[1], Eb[2]]), W + W14 + Wb


def nvt_run(sys, pos, vel, n_steps: int, dt: float, temperature: float, tau: float,
            xi: float = 0.0, eta: float = 0.0, nthreads: int = 0):
    """Velocity Verlet with one Nose-Hoover thermostat (Sec. 3.2's canonical
    ensemble), the thermostat propagated in symmetric half steps:

      thermostat(dt/2):  xi += dt/4 G;  v *= exp(-xi dt/2);  eta += dt/2 xi;
                         xi += dt/4 G     with G = (2K - g kT)/Q
      v += dt/2 F/m;  x += dt v;  F = F(x);  v += dt/2 F/m;  thermostat(dt/2)

    with K the kinetic energy, g = 3N - 3, Q = g kT tau^2, units kcal/mol,
    A, fs, amu.  Returns (pos, vel, xi, eta, trace) where trace holds per
    step the potential energies, K and the conserved extended energy
    K + U + Q xi^2 / 2 + g kT eta."""
    b = sys.bonded
    m = np.asarray(b["masses"], np.float64)[:, None]
    tab = setup_table(sys)
    x = np.array(pos, np.float64, copy=True)
    v = np.array(vel, np.float64, copy=True)
    n = x.shape[0]
    g = 3 * n - 3
    kT = KB * temperature
    Q = g * kT * tau * tau

    def kinetic(v):
        return 0.5 * float(np.sum(m * v * v)) / FTM2V

    def thermostat(v, xi, eta):
        K = kinetic(v)
        xi += 0.25 * dt * (2.0 * K - g * kT) / Q
        s = np.exp(-xi * 0.5 * dt)
        v = v * s
        eta += 0.5 * dt * xi
        K = kinetic(v)
        xi += 0.25 * dt * (2.0 * K - g * kT) / Q
        return v, xi, eta

    F, U, _ = md_forces(sys, x, table=tab, nthreads=nthreads)
    trace = []
    for _ in range(n_steps):
        v, xi, eta = thermostat(v, xi, eta)
        v = v + 0.5 * dt * FTM2V * F / m
        x = x + dt * v
        F, U, _ = md_forces(sys, x, table=tab, nthreads=nthreads)
        v = v + 0.5 * dt * FTM2V * F / m
        v, xi, eta = thermostat(v, xi, eta)
        K = kinetic(v)
        trace.append(np.concatenate([U, [K, K + U.sum() + 0.5 * Q * xi * xi + g * kT * eta]]))
    return x, v, xi, eta, np.array(trace)
