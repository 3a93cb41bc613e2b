"""Seeded synthetic inputs for the RelRes Lennard-Jones hot path.

This module builds geometry, topology and literal parameter tables only.  It
holds none of the method's arithmetic: no mixing rules, no smoothing
polynomials, no shifting constants, no pair terms.  Both the CPU oracle and the
HIP path receive exactly the arrays produced here.

Units are kcal/mol and Angstrom.  The paper tabulates energies in zJ and
lengths in nm (Table 1); ``ZJ`` converts zJ to kcal/mol (N_A * 1e-21 J / 4184 J).

Workloads (stand-ins for the paper's equilibrated liquids, which are not
available; see the Verification section, setup of molecular simulations):

* ``propane_liquid``    500 C3H8 molecules (3 united atoms, hybrid = middle
  atom), cubic lattice, random orientations, 0.1 A jitter, 0.0095 atoms/A^3.
* ``neopentane_liquid`` 4096 C5H12 molecules (central C hybrid + 4 CH3),
  16^3 lattice, random orientations, 0.1 A jitter, 0.0085 atoms/A^3,
  FG/CG parameters from Table 1 (C5H12 rows).
* ``copolymer_melt``    2048 A24-B24 chains of 48 beads grown as seeded
  self-avoiding random walks (bond 1.54 A, angle 112 deg, uniform torsion,
  trial beads rejected closer than 3 A to any bead more than three bonds
  away), one CG site per four-bead segment (bead 4k+1), 1-2/1-3/1-4 pairs
  excluded, Lorentz-Berthelot mixing, 0.0090 atoms/A^3.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# zJ -> kcal/mol (unit conversion only)
ZJ = 6.02214076e23 * 1e-21 / 4184.0

MIX_GEOMETRIC = 0
MIX_ARITHMETIC = 1   # Lorentz-Berthelot: geometric eps, arithmetic sigma
MIX_SIXTHPOWER = 2

# Cutoffs used by every workload (Angstrom): r_s- r_s+ r_c- r_c+ and the skin.
RELRES_CUTOFFS = dict(rs_in=5.5, rs_out=6.0, rc_in=12.0, rc_out=14.0, skin=2.0)


@dataclass
class System:
    """One periodic orthorhombic system, in caller (user) atom order."""
    name: str
    pos: np.ndarray            # (N,3) float64, wrapped into [0, L) per axis
    box: np.ndarray            # (3,) float64 edge lengths
    types: np.ndarray          # (N,) int32 atom types
    mol: np.ndarray            # (N,) int32 molecule ids
    excl_offsets: np.ndarray   # (N+1,) int32 CSR offsets of extra exclusions
    excl_idx: np.ndarray       # int32 excluded partners (user indices)
    exclude_same_mol: bool     # exclude every intramolecular pair
    eps_fg: np.ndarray         # (ntypes,) float64
    sig_fg: np.ndarray
    eps_cg: np.ndarray         # 0 for ordinary types
    sig_cg: np.ndarray
    mix: int = MIX_GEOMETRIC
    rs_in: float = 5.5
    rs_out: float = 6.0
    rc_in: float = 12.0
    rc_out: float = 14.0
    skin: float = 2.0
    precision: int = 32
    shift: bool = True         # pair_modify shift yes / no
    cut_type: np.ndarray | None = None   # (ntypes, 4) per-type r_s-, r_s+, r_c-, r_c+
    cut_pair: np.ndarray | None = None   # (ntypes, ntypes, 4) per-type-pair distances
    bonded: dict | None = None # bonded topology and parameters (see hexane_liquid)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def ntypes(self) -> int:
        return int(self.eps_fg.shape[0])

    def replace(self, **kw) -> "System":
        return dataclasses.replace(self, **kw)

    def conventional(self) -> "System":
        """The reference (all-FG) system: r_s -> r_c and no CG sites.

        The FG potential is kept up to r_c- and switched off over [r_c-, r_c+)
        by the same kind of polynomial; the outer smoothing zone is empty.
        """
        return self.replace(
            name=self.name + "/conventional",
            rs_in=self.rc_in, rs_out=self.rc_out,
            rc_in=self.rc_out, rc_out=self.rc_out,
            eps_cg=np.zeros_like(self.eps_cg),
            meta=dict(self.meta, conventional=True))


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def wrap(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Wrap positions into [0, L) per axis."""
    w = np.mod(pos, box)
    w = np.where(w >= box, 0.0, w)
    return np.ascontiguousarray(w, dtype=np.float64)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly distributed rotation matrices (normalised Gaussian quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def propane_template(bond=1.54, angle_deg=112.0) -> np.ndarray:
    """CH3 - CH2 - CH3 with the middle (hybrid) atom at the origin."""
    h = np.deg2rad(angle_deg) / 2.0
    return np.array([[bond * np.sin(h), bond * np.cos(h), 0.0],
                     [0.0, 0.0, 0.0],
                     [-bond * np.sin(h), bond * np.cos(h), 0.0]])


def neopentane_template(bond=1.54) -> np.ndarray:
    """Central C at the origin plus four CH3 on tetrahedral directions."""
    d = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    d /= np.sqrt(3.0)
    return np.vstack([np.zeros((1, 3)), bond * d])


def _csr_empty(n: int):
    return np.zeros(n + 1, np.int32), np.zeros(0, np.int32)


def _lattice_molecules(rng, template, n_mol, n_side, box_len, jitter):
    """Place n_mol rigid molecules on the first n_mol sites of an n_side^3
    lattice (x-major order), each with a uniform random rotation, plus
    N(0, jitter^2) noise on every coordinate."""
    a = box_len / n_side
    m = np.arange(n_mol)
    site = np.stack([m // (n_side * n_side), (m // n_side) % n_side, m % n_side], 1)
    centres = (site + 0.5) * a
    rot = random_rotations(rng, n_mol)
    atoms = centres[:, None, :] + np.einsum("mij,aj->mai", rot, template)
    atoms = atoms.reshape(-1, 3)
    if jitter > 0:
        atoms = atoms + rng.normal(scale=jitter, size=atoms.shape)
    return atoms


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def propane_liquid(seed: int = 0, n_mol: int = 500, density: float = 0.0095,
                   precision: int = 64, jitter: float = 0.1) -> System:
    """Propane-like liquid: 3 united atoms per molecule, middle atom hybrid.

    Types: 0 = ordinary CH3 (eps 0.195, sigma 3.75), 1 = hybrid middle atom
    (same FG parameters; CG eps 1.0 kcal/mol, sigma 4.6 A).  Geometric mixing.
    """
    rng = np.random.default_rng(seed)
    n = 3 * n_mol
    box_len = (n / density) ** (1.0 / 3.0)
    n_side = int(np.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    pos = _lattice_molecules(rng, propane_template(), n_mol, n_side, box_len, jitter)
    box = np.full(3, box_len)
    types = np.tile(np.array([0, 1, 0], np.int32), n_mol)
    mol = np.repeat(np.arange(n_mol, dtype=np.int32), 3)
    eo, ei = _csr_empty(n)
    return System(
        name="propane_liquid", pos=wrap(pos, box), box=box, types=types, mol=mol,
        excl_offsets=eo, excl_idx=ei, exclude_same_mol=True,
        eps_fg=np.array([0.195, 0.195]), sig_fg=np.array([3.75, 3.75]),
        eps_cg=np.array([0.0, 1.0]), sig_cg=np.array([4.6, 4.6]),
        mix=MIX_GEOMETRIC, precision=precision,
        meta=dict(seed=seed, n_mol=n_mol, density=density, mapping_ratio=3),
        **RELRES_CUTOFFS)


def neopentane_liquid(seed: int = 0, n_side: int = 16, density: float = 0.0085,
                      precision: int = 32, jitter: float = 0.1) -> System:
    """Neopentane-like liquid: central C (hybrid) + 4 CH3 (ordinary).

    Parameters are Table 1's C5H12 rows converted to kcal/mol and Angstrom:
    CH3 eps 1.0074 zJ, sigma 0.3960 nm; C eps 0.3474 zJ, sigma 0.3800 nm;
    hybrid C CG eps 21.133 zJ, sigma 0.3942 nm.  Geometric mixing.
    """
    rng = np.random.default_rng(seed)
    n_mol = n_side ** 3
    n = 5 * n_mol
    box_len = (n / density) ** (1.0 / 3.0)
    pos = _lattice_molecules(rng, neopentane_template(), n_mol, n_side, box_len, jitter)
    box = np.full(3, box_len)
    types = np.tile(np.array([1, 0, 0, 0, 0], np.int32), n_mol)
    mol = np.repeat(np.arange(n_mol, dtype=np.int32), 5)
    eo, ei = _csr_empty(n)
    return System(
        name="neopentane_liquid", pos=wrap(pos, box), box=box, types=types, mol=mol,
        excl_offsets=eo, excl_idx=ei, exclude_same_mol=True,
        eps_fg=np.array([1.0074 * ZJ, 0.3474 * ZJ]),
        sig_fg=np.array([3.960, 3.800]),
        eps_cg=np.array([0.0, 21.133 * ZJ]),
        sig_cg=np.array([3.942, 3.942]),
        mix=MIX_GEOMETRIC, precision=precision,
        meta=dict(seed=seed, n_mol=n_mol, density=density, mapping_ratio=5),
        **RELRES_CUTOFFS)


def _grow_chains(rng, n_chains, n_beads, box_len, bond=1.54, angle_deg=112.0,
                 min_dist=3.0, excl_bonds=3, lockstep_tries=20):
    """Grow all chains in lockstep as self-avoiding random walks.

    A trial bead is rejected when it lies closer than ``min_dist`` to any
    placed bead that is not within ``excl_bonds`` bonds along its own chain
    (and to trial beads accepted earlier in the same step).
    Returns unwrapped positions (n_chains, n_beads, 3).
    """
    L = box_len
    ncell = max(3, int(L // min_dist))
    cs = L / ncell
    cap = 16
    grid = -np.ones((ncell, ncell, ncell, cap), np.int64)
    fill = np.zeros((ncell, ncell, ncell), np.int32)
    pos = np.zeros((n_chains, n_beads, 3))
    offs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    flat_pos = np.zeros((n_chains * n_beads, 3))   # wrapped positions of placed beads
    theta = np.deg2rad(180.0 - angle_deg)           # angle between successive bonds

    def cell_of(p):
        c = np.floor(np.mod(p, L) / cs).astype(np.int64)
        return np.minimum(c, ncell - 1)

    def check(trials, chains, b):
        """Return mask of trials with no clash against placed beads."""
        c = cell_of(trials)
        nb = (c[:, None, :] + offs[None, :, :]) % ncell
        ids = grid[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(len(trials), -1)
        valid = ids >= 0
        same_chain = (ids // n_beads) == chains[:, None]
        near = same_chain & ((b - ids % n_beads) <= excl_bonds)
        valid &= ~near
        d = flat_pos[np.where(valid, ids, 0)] - np.mod(trials, L)[:, None, :]
        d -= L * np.round(d / L)
        r2 = np.einsum("kij,kij->ki", d, d)
        r2 = np.where(valid, r2, np.inf)
        ok = r2.min(axis=1) >= min_dist * min_dist if r2.shape[1] else np.ones(len(trials), bool)
        # clashes among this step's accepted trials (keep lower chain index)
        idx = np.nonzero(ok)[0]
        if len(idx) > 1:
            t = np.mod(trials[idx], L)
            dd = t[:, None, :] - t[None, :, :]
            dd -= L * np.round(dd / L)
            rr = np.einsum("ijk,ijk->ij", dd, dd)
            clash = np.triu(rr < min_dist * min_dist, 1)
            bad = clash.any(axis=0)          # clashes with a lower-index trial
            ok[idx[bad]] = False
        return ok

    def insert(p, chains, b):
        c = cell_of(p)
        gid = chains * n_beads + b
        flat_pos[gid] = np.mod(p, L)
        # accepted trials of one step never share a cell twice only by chance,
        # so insert cell by cell in index order
        lin = (c[:, 0] * ncell + c[:, 1]) * ncell + c[:, 2]
        order = np.argsort(lin, kind="stable")
        lin_s = lin[order]
        first = np.searchsorted(lin_s, lin_s, side="left")
        rank = np.arange(len(lin_s)) - first
        cs_ = c[order]
        f = fill[cs_[:, 0], cs_[:, 1], cs_[:, 2]] + rank
        if len(f) and f.max() >= cap:
            raise RuntimeError("chain growth: cell capacity exceeded")
        grid[cs_[:, 0], cs_[:, 1], cs_[:, 2], f] = gid[order]
        np.add.at(fill, (cs_[:, 0], cs_[:, 1], cs_[:, 2]), 1)

    def remove_chain(ch, upto):
        for bb in range(upto):
            gid = ch * n_beads + bb
            x, y, z = cell_of(pos[ch, bb][None, :])[0]
            f = fill[x, y, z]
            slots = np.nonzero(grid[x, y, z, :f] == gid)[0]
            if len(slots) == 0:
                continue
            s = slots[0]
            grid[x, y, z, s] = grid[x, y, z, f - 1]
            grid[x, y, z, f - 1] = -1
            fill[x, y, z] = f - 1

    def propose(chs, b):
        if b == 0:
            return rng.uniform(0.0, L, size=(len(chs), 3))
        prev = pos[chs, b - 1]
        if b == 1:
            v = rng.normal(size=(len(chs), 3))
            v /= np.linalg.norm(v, axis=1, keepdims=True)
        else:
            u = pos[chs, b - 1] - pos[chs, b - 2]
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            a = np.where(np.abs(u[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
            e1 = np.cross(u, a)
            e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
            e2 = np.cross(u, e1)
            phi = rng.uniform(0.0, 2 * np.pi, size=(len(chs), 1))
            v = np.cos(theta) * u + np.sin(theta) * (np.cos(phi) * e1 + np.sin(phi) * e2)
        return prev + bond * v

    def regrow_alone(ch, target):
        """Restart one trapped chain and grow it alone up to bead ``target``."""
        in_grid = target                      # beads [0, in_grid) are in the grid
        for _ in range(200):
            remove_chain(ch, in_grid)
            in_grid = 0
            chs = np.array([ch])
            for bb in range(target + 1):
                for _t in range(50):
                    t = propose(chs, bb)
                    if check(t, chs, bb)[0]:
                        pos[ch, bb] = t[0]
                        insert(t, chs, bb)
                        in_grid = bb + 1
                        break
                else:
                    break
            if in_grid == target + 1:
                return
        raise RuntimeError("chain growth: could not place a trapped chain")

    for b in range(n_beads):
        todo = np.arange(n_chains)
        for _ in range(lockstep_tries):
            if len(todo) == 0:
                break
            trial = propose(todo, b)
            ok = check(trial, todo, b)
            acc = todo[ok]
            pos[acc, b] = trial[ok]
            insert(trial[ok], acc, b)
            todo = todo[~ok]
        for ch in todo:
            regrow_alone(int(ch), b)
    return pos


_CHAIN_CACHE: dict = {}


def copolymer_melt(seed: int = 0, n_chains: int = 2048, n_beads: int = 48,
                   block: int = 24, density: float = 0.0090,
                   precision: int = 32) -> System:
    """A_block-B_block copolymer melt with one CG site per four-bead segment.

    Types: 0 A-ordinary, 1 A-hybrid, 2 B-ordinary, 3 B-hybrid.  FG: A eps 0.195
    sigma 3.75, B eps 0.091 sigma 3.95.  The hybrid is bead 4k+1 of its
    segment.  CG parameters of a segment of four identical beads follow from
    the multipole parametrisation (Eq. 13 with 16 identical pair terms): eps_CG
    = 16 eps, sigma_CG = sigma, i.e. A 3.12 / 3.75 and B 1.456 / 3.95.
    Lorentz-Berthelot mixing.  Pairs up to three bonds apart are excluded.
    """
    rng = np.random.default_rng(seed)
    n = n_chains * n_beads
    box_len = (n / density) ** (1.0 / 3.0)
    key = (seed, n_chains, n_beads, density)
    if key not in _CHAIN_CACHE:
        _CHAIN_CACHE[key] = _grow_chains(rng, n_chains, n_beads, box_len)
    chains = _CHAIN_CACHE[key]
    box = np.full(3, box_len)
    b = np.arange(n_beads)
    is_b = b >= block
    hyb = (b % 4) == 1
    t_chain = (2 * is_b + hyb).astype(np.int32)
    types = np.tile(t_chain, n_chains)
    mol = np.repeat(np.arange(n_chains, dtype=np.int32), n_beads)
    # 1-2, 1-3, 1-4 exclusions along each chain (user indices)
    offs = np.zeros(n + 1, np.int32)
    lists = []
    for bb in range(n_beads):
        lists.append([bb + d for d in (-3, -2, -1, 1, 2, 3) if 0 <= bb + d < n_beads])
    per_chain_counts = np.array([len(l) for l in lists], np.int32)
    counts = np.tile(per_chain_counts, n_chains)
    offs[1:] = np.cumsum(counts)
    base = np.repeat(np.arange(n_chains) * n_beads, per_chain_counts.sum())
    rel = np.tile(np.concatenate([np.array(l, np.int64) for l in lists]), n_chains)
    idx = (base + rel).astype(np.int32)
    return System(
        name="copolymer_melt", pos=wrap(chains.reshape(-1, 3), box), box=box,
        types=types, mol=mol, excl_offsets=offs, excl_idx=idx,
        exclude_same_mol=False,
        eps_fg=np.array([0.195, 0.195, 0.091, 0.091]),
        sig_fg=np.array([3.75, 3.75, 3.95, 3.95]),
        eps_cg=np.array([0.0, 3.12, 0.0, 1.456]),
        sig_cg=np.array([3.75, 3.75, 3.95, 3.95]),
        mix=MIX_ARITHMETIC, precision=precision,
        meta=dict(seed=seed, n_chains=n_chains, n_beads=n_beads, density=density,
                  mapping_ratio=4),
        **RELRES_CUTOFFS)


def random_molecules(seed: int, n_mol: int, box_len: float, kind: str = "propane",
                     min_dist: float = 2.6, precision: int = 64,
                     hybrid_fraction: float = 1.0) -> System:
    """Small randomly placed molecules for property and edge-case tests.

    Molecule centres are uniform in the box; a molecule is re-drawn when any of
    its atoms comes closer than ``min_dist`` to an atom of another molecule.
    ``hybrid_fraction`` < 1 turns the hybrid atom of some molecules ordinary.
    """
    rng = np.random.default_rng(seed)
    tpl = propane_template() if kind == "propane" else neopentane_template()
    hyb_slot = 1 if kind == "propane" else 0
    m = tpl.shape[0]
    box = np.full(3, float(box_len))
    placed = np.zeros((0, 3))
    mols = []
    tries = 0
    while len(mols) < n_mol:
        tries += 1
        if tries > 200000:
            raise RuntimeError("random_molecules: box too crowded")
        c = rng.uniform(0, box_len, size=3)
        atoms = c + tpl @ random_rotations(rng, 1)[0].T
        if len(placed):
            d = atoms[:, None, :] - placed[None, :, :]
            d -= box * np.round(d / box)
            if (np.einsum("ijk,ijk->ij", d, d) < min_dist ** 2).any():
                continue
        mols.append(atoms)
        placed = np.vstack([placed, atoms])
    pos = np.vstack(mols) if mols else np.zeros((0, 3))
    n = pos.shape[0]
    types = np.zeros(n, np.int32)
    is_h = rng.uniform(size=n_mol) < hybrid_fraction
    for k in range(n_mol):
        if is_h[k]:
            types[k * m + hyb_slot] = 1
    mol = np.repeat(np.arange(n_mol, dtype=np.int32), m)
    eo, ei = _csr_empty(n)
    if kind == "propane":
        pars = dict(eps_fg=np.array([0.195, 0.195]), sig_fg=np.array([3.75, 3.75]),
                    eps_cg=np.array([0.0, 1.0]), sig_cg=np.array([4.6, 4.6]))
    else:
        pars = dict(eps_fg=np.array([1.0074 * ZJ, 0.3474 * ZJ]),
                    sig_fg=np.array([3.960, 3.800]),
                    eps_cg=np.array([0.0, 21.133 * ZJ]),
                    sig_cg=np.array([3.942, 3.942]))
    return System(name=f"random_{kind}", pos=wrap(pos, box), box=box, types=types,
                  mol=mol, excl_offsets=eo, excl_idx=ei, exclude_same_mol=True,
                  mix=MIX_GEOMETRIC, precision=precision,
                  meta=dict(seed=seed, n_mol=n_mol), **pars, **RELRES_CUTOFFS)


def two_atoms(r: float, hybrid=(True, True), box_len: float = 40.0,
              precision: int = 64, direction=(1.0, 0.0, 0.0)) -> System:
    """Two atoms at distance r along ``direction`` (different molecules)."""
    u = np.asarray(direction, float)
    u = u / np.linalg.norm(u)
    box = np.full(3, float(box_len))
    c = box / 2.0
    pos = np.vstack([c - 0.5 * r * u, c + 0.5 * r * u])
    types = np.array([1 if hybrid[0] else 0, 1 if hybrid[1] else 0], np.int32)
    eo, ei = _csr_empty(2)
    return System(name="two_atoms", pos=wrap(pos, box), box=box, types=types,
                  mol=np.array([0, 1], np.int32), excl_offsets=eo, excl_idx=ei,
                  exclude_same_mol=True,
                  eps_fg=np.array([0.195, 0.195]), sig_fg=np.array([3.75, 3.75]),
                  eps_cg=np.array([0.0, 1.0]), sig_cg=np.array([4.6, 4.6]),
                  mix=MIX_GEOMETRIC, precision=precision, meta=dict(r=r),
                  **RELRES_CUTOFFS)


def perturbed_frames(base: System, n_frames: int = 64, sigma: float = 0.05,
                     seed: int = 0) -> list:
    """Frames of ``base`` with N(0, sigma^2) noise on every coordinate."""
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n_frames):
        p = base.pos + rng.normal(scale=sigma, size=base.pos.shape)
        out.append(base.replace(pos=wrap(p, base.box), meta=dict(base.meta, frame=f)))
    return out


# Types of the mixed propane/neopentane liquids: 0 propane CH3, 1 propane
# middle atom (hybrid), 2 neopentane CH3, 3 neopentane central C (hybrid).
MIXED_EPS_FG = np.array([0.195, 0.195, 1.0074 * ZJ, 0.3474 * ZJ])
MIXED_SIG_FG = np.array([3.75, 3.75, 3.960, 3.800])
MIXED_EPS_CG = np.array([0.0, 1.0, 0.0, 21.133 * ZJ])
MIXED_SIG_CG = np.array([4.6, 4.6, 3.942, 3.942])


def mixed_liquid(seed: int, n_atoms: int, density: float, p_neopentane: float = 0.5,
                 skin: float = 1.5, precision: int = 32, jitter: float = 0.1,
                 name: str = "mixed_liquid") -> System:
    """A liquid of propane- and neopentane-like molecules in random order
    (each molecule neopentane with probability p_neopentane) on a cubic
    lattice, random orientations, N(0, jitter^2) noise, at least n_atoms
    atoms at the given density.  Geometric mixing; intramolecular pairs
    excluded."""
    rng = np.random.default_rng(seed)
    kinds = []
    atoms = 0
    while atoms < n_atoms:
        k = bool(rng.random() < p_neopentane)
        kinds.append(k)
        atoms += 5 if k else 3
    kinds = np.array(kinds)
    n_mol = len(kinds)
    box_len = (atoms / density) ** (1.0 / 3.0)
    n_side = int(np.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    a = box_len / n_side
    m = np.arange(n_mol)
    site = np.stack([m // (n_side * n_side), (m // n_side) % n_side, m % n_side], 1)
    centres = (site + 0.5) * a
    rot = random_rotations(rng, n_mol)
    tp, tn = propane_template(), neopentane_template()
    pos, types, mol = [], [], []
    for k in range(n_mol):
        tpl = tn if kinds[k] else tp
        pos.append(centres[k] + tpl @ rot[k].T)
        types.append([3, 2, 2, 2, 2] if kinds[k] else [0, 1, 0])
        mol.append(np.full(tpl.shape[0], k))
    pos = np.concatenate(pos)
    if jitter > 0:
        pos = pos + rng.normal(scale=jitter, size=pos.shape)
    box = np.full(3, box_len)
    n = pos.shape[0]
    eo, ei = _csr_empty(n)
    cut = dict(RELRES_CUTOFFS, skin=skin)
    return System(
        name=name, pos=wrap(pos, box), box=box, types=np.concatenate(types).astype(np.int32),
        mol=np.concatenate(mol).astype(np.int32), excl_offsets=eo, excl_idx=ei,
        exclude_same_mol=True, eps_fg=MIXED_EPS_FG.copy(), sig_fg=MIXED_SIG_FG.copy(),
        eps_cg=MIXED_EPS_CG.copy(), sig_cg=MIXED_SIG_CG.copy(), mix=MIX_GEOMETRIC,
        precision=precision, meta=dict(seed=seed, n_mol=n_mol, density=density), **cut)


@dataclass
class Batch:
    """Replica systems that share one parameter set, concatenated in order.

    ``systems[s]`` is replica s alone; ``whole`` holds the concatenated atoms
    (molecule ids made unique across replicas, box of replica 0) for the
    topology call; ``offsets`` (nsys + 1) and ``boxes`` (nsys, 3) describe
    the replicas; ``skins`` (nsys) is each replica's own skin."""
    systems: list
    offsets: np.ndarray
    boxes: np.ndarray
    whole: System
    skins: np.ndarray = None

    @property
    def nsys(self) -> int:
        return len(self.systems)


def batch_of(systems: list) -> Batch:
    sizes = [s.n for s in systems]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    mol_base = np.concatenate([[0], np.cumsum([int(s.mol.max()) + 1 if s.n else 0
                                               for s in systems])])
    s0 = systems[0]
    n = int(offsets[-1])
    eo, ei = _csr_empty(n)
    whole = s0.replace(
        name="batch", pos=np.concatenate([s.pos for s in systems]),
        types=np.concatenate([s.types for s in systems]).astype(np.int32),
        mol=np.concatenate([s.mol + mol_base[k] for k, s in enumerate(systems)]).astype(np.int32),
        excl_offsets=eo, excl_idx=ei, meta=dict(nsys=len(systems)))
    return Batch(systems=systems, offsets=offsets,
                 boxes=np.stack([s.box for s in systems]), whole=whole,
                 skins=np.array([s.skin for s in systems], dtype=np.float64))


def replica_batch(seed: int = 0, n_systems: int = 256, min_atoms: int = 300,
                  max_atoms: int = 30000, total_atoms: int = 1_200_000,
                  dmin: float = 0.0080, dmax: float = 0.0100, skin: float = 1.5,
                  precision: int = 32, skin_max: float = None) -> Batch:
    """Replicas of uneven size: sizes log-uniform in [min_atoms, max_atoms]
    rescaled (and clipped) towards total_atoms, densities uniform in
    [dmin, dmax], each a mixed propane/neopentane liquid with its own
    neopentane fraction.  The 1.5 A skin keeps the smallest box (300 atoms at
    0.0100 / A^3, L = 31.07 A) above twice the site-list radius.  With
    skin_max, a replica whose box allows it (every edge above
    2 (r_c+ + skin_max)) gets skin_max instead: per-replica skins."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(min_atoms), np.log(max_atoms), n_systems))
    for _ in range(20):
        sizes = np.clip(sizes * total_atoms / sizes.sum(), min_atoms, max_atoms)
    dens = rng.uniform(dmin, dmax, n_systems)
    pneo = rng.uniform(0.0, 1.0, n_systems)
    seeds = rng.integers(0, 2 ** 31, n_systems)
    systems = [mixed_liquid(int(seeds[k]), int(sizes[k]), float(dens[k]), float(pneo[k]),
                            skin=skin, precision=precision, name=f"replica{k}")
               for k in range(n_systems)]
    if skin_max is not None:
        systems = [s.replace(skin=skin_max)
                   if float(np.min(s.box)) > 2.0 * (s.rc_out + skin_max) * (1.0 + 1e-9) else s
                   for s in systems]
    return batch_of(systems)


WORKLOADS = {
    "propane_1500": lambda seed=0: propane_liquid(seed),
    "neopentane_20480": lambda seed=0: neopentane_liquid(seed),
    "copolymer_98304": lambda seed=0: copolymer_melt(seed),
}


# ----------------------------------------------------------------------------
# molecular dynamics workload: hexane as a C3H7-C3H7 dimer
# ----------------------------------------------------------------------------

# united-atom masses (amu)
MASS_CH3 = 15.035
MASS_CH2 = 14.027
# AMBER_UA bonded parameters of the paper's simulations, in kcal/mol and A:
# E_bond = K (r - r0)^2, E_angle = K (theta - theta0)^2, E_dih = K (1 + cos(n phi - d))
BOND_K = 180640.0 * ZJ / 100.0       # 180,640 zJ/nm^2
BOND_R0 = 1.526
ANGLE_K = 437.7 * ZJ                 # 437.7 zJ/rad^2
ANGLE_T0 = 1.9618
DIH_K = 13.9 * ZJ                    # 13.9 zJ (1 + cos 3 phi)
DIH_N = 3
SCALE_14 = 0.5


def chain_positions(n: int, dihedrals, bond: float = BOND_R0, angle: float = ANGLE_T0) -> np.ndarray:
    """Positions of an n-atom chain from internal coordinates: bond length,
    bond angle and the n-3 dihedral angles (trans = pi), centred at the
    origin."""
    x = np.zeros((n, 3))
    x[1] = [bond, 0.0, 0.0]
    if n > 2:
        x[2] = x[1] + bond * np.array([-np.cos(angle), np.sin(angle), 0.0])
    for k in range(3, n):
        a, b, c = x[k - 3], x[k - 2], x[k - 1]
        bc = c - b
        bc /= np.linalg.norm(bc)
        nrm = np.cross(b - a, bc)
        nrm /= np.linalg.norm(nrm)
        m = np.cross(nrm, bc)
        phi = dihedrals[k - 3]
        d2 = np.array([-bond * np.cos(angle), bond * np.sin(angle) * np.cos(phi),
                       bond * np.sin(angle) * np.sin(phi)])
        x[k] = c + d2[0] * bc + d2[1] * m + d2[2] * nrm
    return x - x.mean(axis=0)


def hexane_liquid(seed: int = 0, n_mol: int = 1000, density: float = 0.0120,
                  min_dist: float = 3.0, precision: int = 64, p_trans: float = 0.7,
                  temperature: float = 290.0) -> System:
    """Hexane as the dimer C3H7-C3H7 of the paper's dimer study: six united
    atoms CH3-CH2-CH2-CH2-CH2-CH3 in two groups of three, the middle CH2 of
    each group hybrid (types 0 CH3, 1 CH2, 2 hybrid CH2; Table 1's C3H7 rows,
    r_s = 0.6 nm with a 0.05 nm zone, r_c 1.2/1.4 nm).  Chains are built from
    internal coordinates (AMBER_UA bond 1.526 A and angle 1.9618 rad; each
    dihedral trans with probability p_trans, else gauche +-60 deg; conformers
    that bring atoms four or more bonds apart closer than min_dist are
    redrawn), placed at uniform random centres and orientations and redrawn
    when any atom comes closer than min_dist to another chain.  Intramolecular 1-2, 1-3 and 1-4
    pairs are excluded from the pair lists; the 1-4 pairs interact through
    the pair potential scaled by 0.5.  ``bonded`` holds the bonds, angles,
    dihedrals, 1-4 pairs, their parameters, the masses and Maxwell-Boltzmann
    velocities at ``temperature`` (K) with zero total momentum."""
    rng = np.random.default_rng(seed)
    m = 6
    n = n_mol * m
    box_len = (n / density) ** (1.0 / 3.0)
    box = np.full(3, box_len)
    placed = np.zeros((0, 3))
    mols = []
    tries = 0
    while len(mols) < n_mol:
        tries += 1
        if tries > 400 * n_mol:
            raise RuntimeError("hexane_liquid: box too crowded")
        u = rng.uniform(size=m - 3)
        dih = np.where(u < p_trans, np.pi, np.where(u < 0.5 + 0.5 * p_trans, np.pi / 3, -np.pi / 3))
        tpl = chain_positions(m, dih)
        # atoms four or more bonds apart interact; a g+g- sequence would put
        # them on top of each other
        far = [(i, j) for i in range(m) for j in range(i + 4, m)]
        if any(np.linalg.norm(tpl[i] - tpl[j]) < min_dist for i, j in far):
            continue
        atoms = rng.uniform(0, box_len, size=3) + tpl @ random_rotations(rng, 1)[0].T
        if len(placed):
            d = atoms[:, None, :] - placed[None, :, :]
            d -= box * np.round(d / box)
            if (np.einsum("ijk,ijk->ij", d, d) < min_dist ** 2).any():
                continue
        mols.append(atoms)
        placed = np.vstack([placed, atoms])
    pos = np.vstack(mols)
    types = np.tile(np.array([0, 2, 1, 1, 2, 0], np.int32), n_mol)
    mol = np.repeat(np.arange(n_mol, dtype=np.int32), m)
    base = (np.arange(n_mol) * m)[:, None]
    bonds = (base[:, :, None] + np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5]])[None]).reshape(-1, 2)
    angles = (base[:, :, None] + np.array([[0, 1, 2], [1, 2, 3], [2, 3, 4], [3, 4, 5]])[None]).reshape(-1, 3)
    dihs = (base[:, :, None] + np.array([[0, 1, 2, 3], [1, 2, 3, 4], [2, 3, 4, 5]])[None]).reshape(-1, 4)
    p14 = dihs[:, [0, 3]].copy()
    # exclusions: 1-2, 1-3 and 1-4 partners of every atom (CSR, symmetric)
    partners = [[] for _ in range(n)]
    for a, b in np.vstack([bonds, angles[:, [0, 2]], p14]):
        partners[a].append(b)
        partners[b].append(a)
    offs = np.zeros(n + 1, np.int32)
    offs[1:] = np.cumsum([len(q) for q in partners])
    idx = np.array([j for q in partners for j in sorted(q)], np.int32)
    masses = np.where(types == 0, MASS_CH3, MASS_CH2).astype(np.float64)
    # Maxwell-Boltzmann velocities in A/fs, zero total momentum
    kT = 0.0019872067 * temperature                       # kcal/mol
    sd = np.sqrt(kT / masses * 4.184e-4)                  # A/fs
    vel = rng.normal(size=(n, 3)) * sd[:, None]
    vel -= (masses[:, None] * vel).sum(axis=0) / masses.sum()
    nb, na, nd = len(bonds), len(angles), len(dihs)
    bonded = dict(bonds=bonds.astype(np.int32), bond_k=np.full(nb, BOND_K), bond_r0=np.full(nb, BOND_R0),
                  angles=angles.astype(np.int32), angle_k=np.full(na, ANGLE_K),
                  angle_t0=np.full(na, ANGLE_T0),
                  dihedrals=dihs.astype(np.int32), dih_k=np.full(nd, DIH_K),
                  dih_n=np.full(nd, DIH_N, np.int32), dih_d=np.zeros(nd),
                  pairs14=p14.astype(np.int32), scale14=SCALE_14, masses=masses, velocities=vel)
    eps = np.array([1.2158, 0.8198, 0.8198]) * ZJ
    sig = np.array([3.905, 3.905, 3.905])
    return System(name="hexane_liquid", pos=wrap(pos, box), box=box, types=types, mol=mol,
                  excl_offsets=offs, excl_idx=idx, exclude_same_mol=False,
                  eps_fg=eps, sig_fg=sig, eps_cg=np.array([0.0, 0.0, 8.4887 * ZJ]),
                  sig_cg=np.array([0.0, 0.0, 3.905]), mix=MIX_GEOMETRIC, precision=precision,
                  rs_in=5.75, rs_out=6.25, rc_in=12.0, rc_out=14.0, skin=2.0,
                  bonded=bonded, meta=dict(seed=seed, n_mol=n_mol, density=density,
                                           temperature=temperature))
