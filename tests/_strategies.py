"""Hypothesis strategies: small random RelRes systems (2-64 atoms, 1-3 types
with random hybrid flags, random LJ parameters, mixing rule, distances with
empty or finite zones, skin, orthorhombic boxes just above twice the list
radius, molecules).  Input generation only; the scale helper below uses the
oracle's pair function to say how large the summed terms are."""
import numpy as np
from hypothesis import strategies as st

import oracle
import workloads as w


@st.composite
def tiny_systems(draw, precision=64, max_atoms=64, min_dist=2.6):
    n = draw(st.integers(2, max_atoms), label="atoms")
    nt = draw(st.integers(1, 3), label="types")
    hybrid = draw(st.lists(st.booleans(), min_size=nt, max_size=nt), label="hybrid")
    rs_in = draw(st.floats(3.5, 7.0), label="rs_in")
    rs_out = rs_in + draw(st.sampled_from([0.0, 0.3, 0.5, 1.0]), label="s zone")
    rc_in = rs_out + draw(st.floats(0.0, 5.0), label="rc_in - rs_out")
    rc_out = rc_in + draw(st.sampled_from([0.0, 0.5, 2.0]), label="c zone")
    skin = draw(st.sampled_from([0.0, 0.5, 2.0]), label="skin")
    lo = 2.0 * (rc_out + skin) + 0.05
    box = np.array([draw(st.floats(lo, lo + 10.0), label=f"L{k}") for k in range(3)])
    seed = draw(st.integers(0, 2 ** 31 - 1), label="seed")
    rng = np.random.default_rng(seed)
    pos = []
    for _ in range(50 * n):
        if len(pos) == n:
            break
        x = rng.uniform(0.0, box)
        if pos:
            d = np.asarray(pos) - x
            d -= box * np.rint(d / box)
            if np.min(np.sum(d * d, axis=1)) < min_dist * min_dist:
                continue
        pos.append(x)
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    types = rng.integers(0, nt, n).astype(np.int32)
    mol = rng.integers(0, max(1, n // 3), n).astype(np.int32)
    eps_fg = rng.uniform(0.05, 0.3, nt)
    sig_fg = rng.uniform(3.0, 4.2, nt)
    eps_cg = np.where(hybrid, rng.uniform(0.5, 3.0, nt), 0.0)
    sig_cg = rng.uniform(3.5, 4.8, nt)
    return w.System(
        name="tiny", pos=pos, box=box, types=types, mol=mol,
        excl_offsets=np.zeros(n + 1, np.int32), excl_idx=np.zeros(0, np.int32),
        exclude_same_mol=draw(st.booleans(), label="exclude_same_mol"),
        eps_fg=eps_fg, sig_fg=sig_fg, eps_cg=eps_cg, sig_cg=sig_cg,
        mix=draw(st.sampled_from([w.MIX_GEOMETRIC, w.MIX_ARITHMETIC, w.MIX_SIXTHPOWER]),
                 label="mix"),
        rs_in=rs_in, rs_out=rs_out, rc_in=rc_in, rc_out=rc_out, skin=skin,
        precision=precision, shift=draw(st.booleans(), label="shift"))


def term_scales(s):
    """Magnitudes of the summed pair terms: (sqrt(sum_i (sum_j |u'|)^2),
    sum |u|, sum |u'| r) over the non-excluded pairs, so that errors of sums
    that cancel are measured against the terms that make them."""
    tab = oracle.setup_table(s)
    n = s.n
    fi = np.zeros(n)
    es = ws = 0.0
    for i in range(n - 1):
        d = s.pos[i + 1:] - s.pos[i]
        d -= s.box * np.rint(d / s.box)
        r = np.sqrt(np.sum(d * d, axis=1))
        for k, j in enumerate(range(i + 1, n)):
            if s.exclude_same_mol and s.mol[i] == s.mol[j]:
                continue
            u, du, _, _, _ = oracle.pair(tab[s.types[i], s.types[j]], r[k])
            fi[i] += abs(du[0])
            fi[j] += abs(du[0])
            es += abs(u[0])
            ws += abs(du[0]) * r[k]
    return float(np.sqrt(np.sum(fi * fi))), es, ws
