"""Benchmark of the RelRes LJ hot path on one MI355X.

Workload (default): the neopentane-like liquid, 4096 molecules x 5 united
atoms = 20480 atoms, FP32 forces with FP64 energy/virial accumulation, cutoffs
r_s-/r_s+/r_c-/r_c+ = 5.5/6.0/12.0/14.0 A, skin 2 A.  One step = one force
call (forces, energy and virial) on the resident positions; the neighbour
lists are rebuilt every 10 steps inside the timed region.  The same protocol
is then run for the conventional all-FG system (r_s -> r_c, list at 16 A),
and the oracle is timed on the host for the CPU baseline.  Builds are enqueued
without waiting; the lists of a timed run are checked after its closing
synchronisation, and a run whose builds overflowed is discarded and run again
with the grown lists.

Prints ONE JSON line (rank 0).  value = RelRes atom-steps/s on this GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
FP64_VALU_PEAK_TFLOPS = 78.6    # MI355X vector FP64
FP32_VALU_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (packed; 78.6 without packed FP32)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make(sys_, precision, pair_math):
    from paper_2104_10231_amd.relres import RelRes
    rr = RelRes(rs_in=sys_.rs_in, rs_out=sys_.rs_out, rc_in=sys_.rc_in, rc_out=sys_.rc_out,
                skin=sys_.skin, eps_fg=sys_.eps_fg, sig_fg=sys_.sig_fg, eps_cg=sys_.eps_cg,
                sig_cg=sys_.sig_cg, mix=sys_.mix, precision=precision, pair_math=pair_math)
    csr = len(sys_.excl_idx) > 0
    rr.set_topology(sys_.types, sys_.mol, sys_.exclude_same_mol,
                    sys_.excl_offsets if csr else None, sys_.excl_idx if csr else None)
    return rr


def recorded_traffic(workload):
    """HBM bytes per force launch measured with rocprofv3 counters (FETCH_SIZE
    and WRITE_SIZE, scaled by a copy of known size) for this workload, if a
    summary under profiles/ records them for the kernel sources as they are
    now; None otherwise (the counters describe another kernel)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"k_forces_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    m_h = re.search(r"^kernel_sources_sha256: ([0-9a-f]{64})$", text, re.M)
    if not (m_t and m_h):
        return None
    h = hashlib.sha256()
    for f in ("relres_kernels.hip", "relres_internal.h", "relres_pair.h", "relres_lanes.h"):
        with open(os.path.join(ROOT, "paper_2104_10231_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_t.group(1)) if h.hexdigest() == m_h.group(1) else None


def algorithmic_bytes(st, force_bytes):
    """Bytes one force launch must move at minimum: FP64 positions read once
    (24 B/atom), forces written once, every list entry (4 B) and row count
    (4 B) read once.  Neighbour-position gathers are assumed cache hits."""
    n, ns = st["n_atoms"], st["n_sites"]
    return n * (24 + 3 * force_bytes) + 4 * (st["atom_entries"] + st["site_entries"]) + 4 * (n + ns)


class Stepper:
    """Runs the protocol: a list rebuild every `rebuild_every` steps, one force
    call (forces, energy, virial) per step.  With graphs, a cycle (the rebuild
    and the force calls behind it) is one captured HIP graph, re-captured
    whenever the library reallocates a buffer the calls use; the host enqueues
    the cycles of a run without waiting and checks the lists once after them
    (a captured build's status accumulates over replays on the device, so one
    check covers every cycle; a run whose builds overflowed is redone with the
    grown lists).  Without graphs every cycle is launched eagerly and checked
    after the force calls behind its build were enqueued.  `timed_run` is one
    timed run: with graphs its lists are checked after the closing
    synchronisation, outside the timed bracket, and an overflowed run is
    discarded and repeated."""

    def __init__(self, rr, pos, box, rebuild_every, use_graph):
        import torch
        self.rr, self.pos, self.box = rr, pos, box
        self.every = rebuild_every
        self.use_graph = use_graph
        dt = torch.float32 if rr.precision == 32 else torch.float64
        self.F = torch.empty((pos.shape[0], 3), dtype=dt, device=pos.device)
        self.E = torch.empty(3, dtype=torch.float64, device=pos.device)
        self.W = torch.empty(6, dtype=torch.float64, device=pos.device)
        self.graphs, self.graph_gen = {}, None
        self.redone = 0

    def force(self):
        self.rr.forces(self.pos, out=self.F, energy=self.E, virial=self.W)

    def _cycle_graph(self, n, with_build=True):
        """Graph of one cycle: the rebuild (unless with_build is False) and n
        force calls."""
        import torch
        gen = self.rr.generation()
        if gen != self.graph_gen:
            self.graphs = {}
        key = (n, with_build)
        if key not in self.graphs:
            # a waited build sizes every buffer outside capture
            self.rr.build_lists(self.pos, self.box)
            self.force()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                if with_build:
                    self.rr.build_lists(self.pos, self.box, wait=False)
                for _ in range(n):
                    self.force()
            self.graphs[key] = g
            self.graph_gen = self.rr.generation()
        return self.graphs[key]

    def enqueue(self, steps):
        """Enqueue `steps` steps (graph mode), no host wait."""
        k = 0
        while k < steps:
            n = min(self.every, steps - k)
            self._cycle_graph(n).replay()
            k += n

    def run(self, steps):
        """`steps` steps; returns when the GPU has finished them and the lists
        of every cycle are known to be complete."""
        import torch
        if self.use_graph:
            while True:
                self.enqueue(steps)
                torch.cuda.synchronize()
                if self.rr.check_lists():
                    return
                self.redone += 1          # rows grew: new buffers, new graphs
        k = 0
        while k < steps:
            n = min(self.every, steps - k)
            self.rr.build_lists(self.pos, self.box, wait=False)
            for _ in range(n):
                self.force()
            if not self.rr.check_lists():
                self.redone += 1
                self.rr.build_lists(self.pos, self.box)
                for _ in range(n):
                    self.force()
            k += n
        torch.cuda.synchronize()


    def timed_run(self, steps):
        """Seconds of one run of `steps` steps, bracketed by device
        synchronisation, whose lists are complete."""
        import torch
        while True:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if self.use_graph:
                self.enqueue(steps)
                torch.cuda.synchronize()
            else:
                self.run(steps)
            dt = time.perf_counter() - t0
            if not self.use_graph or self.rr.check_lists():
                return dt
            self.redone += 1              # rows grew: new buffers, new graphs


def run_protocol(rr, pos, box, steps, warmup, rebuild_every, repeats, use_graph=True):
    """`warmup` untimed steps, then `repeats` timed runs of exactly `steps`
    steps each (bracketed by device synchronisation); returns the seconds of
    every timed run and the stepper."""
    import torch
    st = Stepper(rr, pos, box, rebuild_every, use_graph)
    if use_graph:
        # capture every graph the runs use before anything is timed
        for n in {min(rebuild_every, steps - k) for k in range(0, steps, rebuild_every)} | \
                {min(rebuild_every, warmup - k) for k in range(0, warmup, rebuild_every)}:
            st._cycle_graph(n)
    if warmup > 0:
        st.run(warmup)
    times = [st.timed_run(steps) for _ in range(repeats)]
    return times, st


def time_kernels(rr, pos, box, force_calls, builds=20):
    """Average device time of one force launch (forces, energy, virial), of
    one list build and of one whole cycle (a build and 10 force calls), each
    with HIP events on the launch stream around replays of a captured graph
    (10 force launches, 10 builds, or one cycle), so host overhead never
    leaves the GPU idle inside the bracket."""
    import torch
    st = Stepper(rr, pos, box, 10, True)

    def per_replay(g, reps):
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    reps = max(1, force_calls // 10)
    force_us = per_replay(st._cycle_graph(10, with_build=False), reps) / 10
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb):
        for _ in range(10):
            rr.build_lists(pos, box, wait=False)
    build_us = per_replay(gb, max(1, builds // 10)) / 10
    cycle_us = per_replay(st._cycle_graph(10), reps)
    if not rr.check_lists():
        raise RuntimeError("list rows overflowed while timing kernels")
    return force_us, build_us, cycle_us


def batch_roofline(pair_math):
    """Roofline of the force launch at a size where it is not bound by the
    launch floor: the 256-replica batch (1.2 M atoms) in one context at the
    automatic kernel shapes, forces with energy and virial per replica, HIP
    events around replays of a graph of 10 launches (the per-system energy
    reduction kernel included)."""
    import torch
    import workloads as w
    b = w.replica_batch(0, skin_max=2.0)
    pos = torch.from_numpy(b.whole.pos).cuda()
    rr = make(b.whole, 32, pair_math)
    rr.set_systems(b.offsets)
    rr.set_skins(b.skins)
    rr.build_lists(pos, b.boxes)
    F = torch.empty((b.whole.n, 3), dtype=torch.float32, device="cuda")
    E = torch.empty((b.nsys, 3), dtype=torch.float64, device="cuda")
    W = torch.empty((b.nsys, 6), dtype=torch.float64, device="cuda")
    rr.forces(pos, out=F, energy=E, virial=W)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(10):
            rr.forces(pos, out=F, energy=E, virial=W)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 50
    st = rr.stats()
    rr.close()
    abytes = algorithmic_bytes(st, 4)
    achieved = abytes / (us * 1e-6) / 1e9
    return {"workload": f"replica_batch: {b.nsys} replicas, {b.whole.n} atoms",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": "k_forces + k_reduce_sys_ew",
            "kernel_us": us, "algorithmic_bytes_per_launch": abytes,
            "list_entries": st["atom_entries"] + st["site_entries"]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def boxes_by_atom(b):
    """The box of every atom of a batch (N x 3)."""
    import numpy as np
    return np.repeat(np.asarray(b.boxes, np.float64).reshape(-1, 3), np.diff(b.offsets), axis=0)


def pair_counts(rr, sys_, pos_np, box_of_atom=None):
    """Ordered pairs of the lists by regime of Eq. 20, for the FLOP count of
    the roofline: list entries, pairs inside r_s+ (atom list) or r_c+ (site
    list) and pairs inside a smoothing zone ([r_s-, r_s+) of the atom list,
    [r_s-, r_s+) or [r_c-, r_c+) of the site list).  Host bookkeeping from the
    library's own pair sets; nothing here feeds the computation."""
    import numpy as np
    from paper_2104_10231_amd.relres import LIST_ATOM, LIST_SITE
    box = np.asarray(sys_.box, np.float64)
    out = {}
    for name, which in (("atom", LIST_ATOM), ("site", LIST_SITE)):
        pr = rr.pairs(which)
        if len(pr) == 0:
            out[name] = (0, 0, 0)
            continue
        d = pos_np[pr[:, 0]] - pos_np[pr[:, 1]]
        bx = box if box_of_atom is None else box_of_atom[pr[:, 0]]
        d -= bx * np.rint(d / bx)
        r = np.sqrt((d * d).sum(1))
        if name == "atom":
            inside = r < sys_.rs_out
            smooth = (r >= sys_.rs_in) & inside
        else:
            inside = r < sys_.rc_out
            smooth = ((r >= sys_.rs_in) & (r < sys_.rs_out)) | ((r >= sys_.rc_in) & inside)
        out[name] = (2 * len(pr), 2 * int(inside.sum()), 2 * int(smooth.sum()))
    return out


def algorithmic_flops(counts):
    """FLOPs of one force launch: 8 per list entry (the distance), 30 per
    pair inside its cutoff (reciprocal, r^-6, scalar force, vector force and
    its accumulation, energy, virial), 17 more per smoothing-zone pair (square
    root and the two polynomials), per ordered pair of the full lists."""
    return sum(8 * e + 30 * p + 17 * z for e, p, z in counts.values())


def cpu_baseline(sys_, budget_s):
    import oracle
    threads = len(os.sched_getaffinity(0))
    oracle.compute(sys_.replace(pos=sys_.pos[:200], types=sys_.types[:200], mol=sys_.mol[:200],
                                excl_offsets=sys_.excl_offsets[:201]), nthreads=threads)
    calls, t0 = 0, time.perf_counter()
    while True:
        oracle.compute(sys_, nthreads=threads)
        calls += 1
        el = time.perf_counter() - t0
        if el >= budget_s or calls >= 1000:
            break
    return dict(value=sys_.n * calls / el, unit="atom-steps/s", cores=threads, kind="oracle",
                cpu=cpu_model(),
                sample=f"{calls} full FP64 O(N^2) force+energy+virial evaluations of the "
                       f"{sys_.n}-atom workload ({el:.1f} s)")


def grad_bench(args):
    """Differentiation workload: the 20480-atom liquid over perturbed frames
    (0.05 A Gaussian noise); per frame a list build, the forward call and the
    gradients of E and of the force-matching loss sum |F - F_ref|^2 with
    respect to positions and per-type eps/sigma (FG and CG), F_ref from the
    oracle at perturbed parameters.  Forward forces FP32, backward FP64."""
    import numpy as np
    import torch
    import oracle
    import workloads as w
    from paper_2104_10231_amd.autograd import energy_forces
    s = w.neopentane_liquid(args.seed)
    frames = w.perturbed_frames(s, n_frames=args.frames, sigma=0.05, seed=args.seed + 1)
    ref = dict(eps_fg=s.eps_fg * 1.03, sig_fg=s.sig_fg * 0.99, eps_cg=s.eps_cg * 1.05,
               sig_cg=s.sig_cg * 1.01)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    frefs = [torch.from_numpy(oracle.compute(f.replace(**ref), nthreads=threads)[0]).cuda()
             for f in frames]
    log(f"[bench] grad: {len(frames)} frames, F_ref from the oracle in {time.perf_counter() - t0:.1f} s")
    pos = [torch.from_numpy(f.pos).cuda() for f in frames]
    rr = make(s, 32, args.pair_math)
    theta = [torch.tensor(np.asarray(getattr(s, k), np.float64), requires_grad=True)
             for k in ("eps_fg", "sig_fg", "eps_cg", "sig_cg")]

    def frame(k):
        p = pos[k].clone().requires_grad_(True)
        rr.build_lists(p.detach(), s.box)
        F, E = energy_forces(rr, p, *theta)
        L = ((F.double() - frefs[k]) ** 2).sum()
        gL = torch.autograd.grad(L, theta + [p], retain_graph=True)
        gE = torch.autograd.grad(E, theta + [p])
        return gL, gE

    for k in range(min(2, len(frames))):
        frame(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(len(frames)):
        frame(k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # device time of one adjoint launch (kernel + bin reduction), back to back
    rr.build_lists(pos[0], s.box)
    g = torch.randn((s.n, 3), dtype=torch.float64, device="cuda")
    e1 = torch.ones(1, dtype=torch.float64, device="cuda")
    for _ in range(5):
        rr.backward(pos[0], g, e1)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 50
    ev0.record()
    for _ in range(reps):
        rr.backward(pos[0], g, e1)
    ev1.record()
    torch.cuda.synchronize()
    back_us = ev0.elapsed_time(ev1) * 1e3 / reps
    st = rr.stats()
    rr.close()
    entries = st["atom_entries"] + st["site_entries"]
    # algorithmic bytes of one adjoint launch: positions and dJ/dF read once,
    # dJ/dx written once, list entries and row counts read once
    abytes = s.n * (24 + 24 + 24) + 4 * entries + 4 * (s.n + st["n_sites"])
    achieved = abytes / (back_us * 1e-6) / 1e9
    out = {
        "metric": "RelRes forward+backward frames/s (gradients of E and of a force-matching loss "
                  "w.r.t. positions and per-type eps/sigma), 1 MI355X",
        "value": len(frames) / dt, "unit": "frames/s", "n_gpus": 1, "steps": len(frames),
        "warmup": 2, "ms_per_step": dt * 1e3 / len(frames), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 forward, f64 backward",
        "data": "synthetic",
        "config": {"workload": "neopentane_20480 perturbed frames (0.05 A)", "atoms": s.n,
                   "frames": len(frames), "parallelism": "single GPU",
                   "per_frame": "list build + forward + 2 adjoint launches (E, force matching)"},
        "atom_steps_per_s": s.n * len(frames) / dt,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_backward",
                     "kernel_us": back_us, "algorithmic_bytes_per_launch": abytes},
    }
    log(f"[bench] grad: {dt * 1e3 / len(frames):.3f} ms/frame, adjoint launch {back_us:.2f} us")
    print(json.dumps(out), flush=True)


def sequential_seconds(b, pos, args, cycles, every):
    """The batch as one context per replica, launched replica after replica:
    seconds for `cycles` cycles (a quarter of them timed, scaled)."""
    import torch
    ctxs = []
    for k, s in enumerate(b.systems):
        c = make(s, 32, args.pair_math)
        p = pos[int(b.offsets[k]):int(b.offsets[k + 1])]
        c.build_lists(p, s.box)
        ctxs.append((c, p, s.box, torch.empty((s.n, 3), dtype=torch.float32, device="cuda"),
                     torch.empty(3, dtype=torch.float64, device="cuda"),
                     torch.empty(6, dtype=torch.float64, device="cuda")))

    def seq_cycle():
        for c, p, box, Fk, Ek, Wk in ctxs:
            c.build_lists(p, box, wait=False)
            for _ in range(every):
                c.forces(p, out=Fk, energy=Ek, virial=Wk)
        for c, p, box, *_ in ctxs:
            if not c.check_lists():
                c.build_lists(p, box)
        torch.cuda.synchronize()

    seq_cycle()
    t0 = time.perf_counter()
    seq_cycles = max(1, cycles // 4)
    for _ in range(seq_cycles):
        seq_cycle()
    dt_s = (time.perf_counter() - t0) * cycles / seq_cycles
    for c, *_ in ctxs:
        c.close()

    return dt_s


def md_bench(args):
    """Dynamics workload: hexane as the C3H7-C3H7 dimer (1000 molecules, 6000
    united atoms, 0.016 atoms/A^3), NVT at 290 K with a Nose-Hoover
    thermostat (tau 100 fs), dt 1 fs, lists every 10 steps, FP32 forces with
    FP64 energies; RelRes (r_s = 0.6 nm) and the conventional 14 A model
    from the same start.  Timed: the production run; reported: atom-steps/s,
    ns/day, and the means of the non-bonded energy and of the virial per
    molecule with their RelRes/conventional ratios."""
    import numpy as np
    import torch
    import workloads as w
    s = w.hexane_liquid(args.seed, n_mol=1000, density=0.016, precision=32)
    n_mol = int(s.mol.max()) + 1
    dt_fs, T, tau, every = 1.0, 290.0, 100.0, 10
    thermo_every = 50
    legs = {}
    for name, sys_ in (("relres", s), ("conventional", s.conventional())):
        rr = make(sys_, 32, 32)
        rr.set_bonded(sys_.bonded)
        p = torch.from_numpy(sys_.pos).cuda()
        v = torch.from_numpy(np.ascontiguousarray(sys_.bonded["velocities"])).cuda()
        rr.build_lists(p, sys_.box)
        rr.md_setup(sys_.bonded["masses"], dt_fs, T, tau, rebuild_every=every)
        rr.md_run(p, v, args.md_equil, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = rr.md_run(p, v, args.md_steps, thermo_every)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        th = th.cpu().numpy()
        st = rr.stats()
        rr.close()
        g = 3 * s.n - 3
        legs[name] = {
            "value": s.n * args.md_steps / el, "ms_per_step": el * 1e3 / args.md_steps,
            "ns_per_day": args.md_steps * dt_fs * 1e-6 / el * 86400.0,
            "U_nonbonded_per_molecule": float(th[:, 0].mean() / n_mol),
            "W_per_molecule": float(th[:, 7].mean() / 3.0 / n_mol),
            "T_mean_K": float((2.0 * th[:, 5] / (g * 0.0019872067)).mean()),
            "extended_energy_drift_per_atom": float((th[-1, 6] - th[0, 6]) / s.n),
            "list_entries": st["atom_entries"] + st["site_entries"],
        }
        log(f"[bench] md {name}: {legs[name]['ms_per_step']:.4f} ms/step, "
            f"{legs[name]['ns_per_day']:.1f} ns/day, <U>/N {legs[name]['U_nonbonded_per_molecule']:.3f}")
    r, c = legs["relres"], legs["conventional"]
    out = {
        "metric": "RelRes NVT molecular dynamics atom-steps/s (hexane, 6000 united atoms, "
                  "bonded + 1-4 + RelRes pairs), 1 MI355X",
        "value": r["value"], "unit": "atom-steps/s", "n_gpus": 1, "steps": args.md_steps,
        "warmup": args.md_equil, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 forces, f64 integration",
        "data": "synthetic",
        "config": {"workload": "hexane_liquid: 1000 C3H7-C3H7 chains, 0.016 atoms/A^3",
                   "atoms": s.n, "dt_fs": dt_fs, "T_K": T, "tau_fs": tau,
                   "rebuild_every": every, "thermostat": "Nose-Hoover",
                   "parallelism": "single GPU"},
        "relres": r, "conventional": c,
        "speedup_vs_conventional": r["value"] / c["value"],
        "ratio_U": r["U_nonbonded_per_molecule"] / c["U_nonbonded_per_molecule"],
        "ratio_W": r["W_per_molecule"] / c["W_per_molecule"],
    }
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Batching workload: 256 replicas of 300-18000 atoms (1.2 M atoms),
    mixed propane/neopentane liquids at 0.0080-0.0100 atoms/A^3, each with
    its own box.  Batched: one context for all replicas; every cycle (a list
    rebuild and `rebuild_every` force calls with energy and virial per
    replica) is one HIP graph replay.  Sequential: one context per replica,
    the same cycle launched replica after replica.  Skins per replica: 2.0 A
    where the box allows it, 1.5 A in boxes below 2 (14 + 2.0) A."""
    import numpy as np
    import torch
    import workloads as w
    b = w.replica_batch(args.seed, skin_max=2.0)
    n = b.whole.n
    steps, every = args.steps, args.rebuild_every
    cycles = max(1, steps // every)
    pos = torch.from_numpy(b.whole.pos).cuda()
    log(f"[bench] batch: {b.nsys} replicas, {n} atoms, {cycles} cycles of 1 build + {every} force calls")

    rr = make(b.whole, 32, args.pair_math)
    rr.set_systems(b.offsets)
    rr.set_skins(b.skins)
    rr.build_lists(pos, b.boxes)
    tuned = None
    if args.lanes:
        rr.set_launch(*args.lanes)
    elif not args.no_tune:
        # setup, outside the timed region: every list and force kernel shape
        # timed on this batch, the fastest kept
        tuned = rr.autotune(pos, b.boxes, reps=2)
        log(f"[bench] autotune: {tuned}")
    F = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    E = torch.empty((b.nsys, 3), dtype=torch.float64, device="cuda")
    W = torch.empty((b.nsys, 6), dtype=torch.float64, device="cuda")
    rr.forces(pos, out=F, energy=E, virial=W)
    torch.cuda.synchronize()

    def capture():
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            rr.build_lists(pos, b.boxes, wait=False)
            for _ in range(every):
                rr.forces(pos, out=F, energy=E, virial=W)
        return g, rr.generation()

    g, gen = capture()
    redone = 0

    def cycle():
        nonlocal g, gen, redone
        g.replay()
        torch.cuda.synchronize()
        while not rr.check_lists():            # rows grew: new buffers, new graph
            redone += 1
            rr.build_lists(pos, b.boxes)
            g, gen = capture()
            g.replay()
            torch.cuda.synchronize()

    for _ in range(2):
        cycle()
    t0 = time.perf_counter()
    for _ in range(cycles):
        cycle()
    dt_b = time.perf_counter() - t0
    st = rr.stats()
    counts = pair_counts(rr, b.whole, b.whole.pos, boxes_by_atom(b))
    # force launch alone, graph of back-to-back launches
    fg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(fg):
        for _ in range(10):
            rr.forces(pos, out=F, energy=E, virial=W)
    fg.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        fg.replay()
    e1.record()
    torch.cuda.synchronize()
    force_us = e0.elapsed_time(e1) * 1e3 / 100
    rr.close()

    dt_s = None if args.no_sequential else sequential_seconds(b, pos, args, cycles, every)
    value = n * cycles * every / dt_b
    seq = None if dt_s is None else n * cycles * every / dt_s
    fb = 4
    abytes = algorithmic_bytes(st, fb)
    achieved = abytes / (force_us * 1e-6) / 1e9
    aflops = algorithmic_flops(counts)
    tflops = aflops / (force_us * 1e-6) / 1e12
    log(f"[bench] batch: {dt_b * 1e3 / (cycles * every):.4f} ms/step batched, "
        + ("" if dt_s is None else f"{dt_s * 1e3 / (cycles * every):.4f} ms/step sequential; ")
        + f"force launch {force_us:.1f} us")
    out = {
        "metric": "RelRes atom-steps/s, 256 batched replicas (1.2 M atoms) in one launch per step, "
                  "1 MI355X",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": cycles * every,
        "warmup": 2 * every, "ms_per_step": dt_b * 1e3 / (cycles * every),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # calls with energy/virial evaluate the pair terms in FP64 (forces FP32)
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "replica_batch: 256 mixed propane/neopentane liquids, "
                               "300-18000 atoms, 0.0080-0.0100 atoms/A^3", "atoms": n,
                   "replicas": b.nsys,
                   "skin_A": {f"{v:g}": int((b.skins == v).sum()) for v in np.unique(b.skins)},
                   "rebuild_every": every,
                   "forces": "fp32", "pair_math": 64, "energy_virial": "fp64 per replica",
                   "parallelism": "single GPU",
                   "launch": "one HIP graph per cycle (rebuild + force calls of all replicas)",
                   "tuned": None if tuned is None else {
                       k: tuned[k] for k in ("cell_div_atom", "cell_div_site", "rows_atom",
                                             "rows_site", "cand_per_lane", "lanes_atom",
                                             "lanes_site", "build_us", "build_us_auto",
                                             "force_us", "force_us_auto")}},
        "sequential": None if seq is None else {
            "value": seq, "ms_per_step": dt_s * 1e3 / (cycles * every),
            "what": "one context per replica, launched replica after replica"},
        "speedup_vs_sequential": None if seq is None else value / seq,
        "builds_redone": redone,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_forces",
                     "kernel_us": force_us, "algorithmic_bytes_per_launch": abytes},
        "roofline_other": {"bound": "alu", "achieved": tflops, "peak": FP64_VALU_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": tflops / FP64_VALU_PEAK_TFLOPS,
                           "valu": "fp64 vector (pair terms of calls with energy/virial)",
                           "algorithmic_flops_per_launch": aflops},
        "list_entries": st["atom_entries"] + st["site_entries"],
        "pairs_by_regime": {k: dict(zip(("entries", "inside_cutoff", "smoothing_zone"), v))
                            for k, v in counts.items()},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps steps each; the median is reported")
    ap.add_argument("--rebuild-every", type=int, default=10)
    ap.add_argument("--workload", default="neopentane_20480",
                    choices=["neopentane_20480", "propane_1500", "copolymer_98304"])
    ap.add_argument("--pair-math", type=int, default=0)
    ap.add_argument("--lanes", type=int, nargs=2, default=None)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-conventional", action="store_true")
    ap.add_argument("--no-batch-roofline", action="store_true",
                    help="skip the force-launch roofline of the 256-replica batch")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every force call eagerly instead of replaying a HIP graph")
    ap.add_argument("--grad", action="store_true",
                    help="run the differentiation workload instead (forward + backward over "
                         "perturbed frames) and print its line")
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--md", action="store_true",
                    help="dynamics workload (NVT hexane, RelRes vs conventional) instead")
    ap.add_argument("--md-equil", type=int, default=2000, help="--md: untimed equilibration steps")
    ap.add_argument("--md-steps", type=int, default=10000, help="--md: timed production steps")
    ap.add_argument("--no-tune", action="store_true",
                    help="--batch: keep the automatic kernel shapes (no autotuning)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch workload only: skip the one-context-per-replica comparison")
    ap.add_argument("--batch", action="store_true",
                    help="run the batching workload (256 replicas in one launch per step) "
                         "instead and print its line")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="finish with 5 device-to-device copies of this many MiB (a kernel "
                         "of known traffic for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the RelRes path "
              "here is single-GPU (it would shard by space, one brick and its halo per GPU).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as w
    from paper_2104_10231_amd.relres import LIB_PATH
    if not os.path.exists(LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    if args.grad:
        grad_bench(args)
        return
    if args.batch:
        batch_bench(args)
        return
    if args.md:
        md_bench(args)
        return
    s = w.WORKLOADS[args.workload](args.seed)
    precision = s.precision
    pos = torch.from_numpy(s.pos).cuda()
    log(f"[bench] workload {args.workload}: N={s.n}, box {s.box[0]:.3f} A, precision {precision}")
    use_graph = not args.no_graph

    def leg(sys_):
        """Kernel timing (the roofline figures; it also brings the device to
        its working clocks), then the protocol: warm-up steps and the timed
        repetitions."""
        rr = make(sys_, precision, args.pair_math)
        if args.lanes:
            rr.set_launch(*args.lanes)
        rr.build_lists(pos, sys_.box)
        force_us, build_us, cycle_us = time_kernels(rr, pos, sys_.box, max(args.steps, 200))
        times, stp = run_protocol(rr, pos, sys_.box, args.steps, args.warmup, args.rebuild_every,
                                  args.repeats, use_graph=use_graph)
        st = rr.stats()
        counts = pair_counts(rr, sys_, s.pos)
        rr.close()
        t_med = sorted(times)[len(times) // 2]
        return dict(times=times, t=t_med, force_us=force_us, build_us=build_us,
                    cycle_us=cycle_us, stats=st, counts=counts, redone=stp.redone)

    R = leg(s)
    st = R["stats"]
    dt = R["t"]
    value = s.n * args.steps / dt
    force_us, build_us = R["force_us"], R["build_us"]
    log(f"[bench] RelRes: {dt * 1e3 / args.steps:.4f} ms/step (median of "
        f"{[round(x * 1e3 / args.steps, 4) for x in R['times']]}), {value:.4e} atom-steps/s; "
        f"atom entries {st['atom_entries']}, site entries {st['site_entries']}, "
        f"builds redone {R['redone']}")
    fb = 4 if precision == 32 else 8
    abytes = algorithmic_bytes(st, fb)
    achieved = abytes / (force_us * 1e-6) / 1e9
    aflops = algorithmic_flops(R["counts"])
    tflops = aflops / (force_us * 1e-6) / 1e12
    # energy and virial are requested at every step: the pair terms then run
    # in the type the library reports for calls with energy/virial
    pm_ew = int(st.get("pair_math_ew", 64))
    alu_peak = FP64_VALU_PEAK_TFLOPS if pm_ew == 64 else FP32_VALU_PEAK_TFLOPS
    log(f"[bench] force launch {force_us:.2f} us, build {build_us:.1f} us, cycle "
        f"{R['cycle_us']:.1f} us (HIP events around graph replays); algorithmic "
        f"{abytes / 1e6:.3f} MB/launch -> {achieved:.1f} GB/s, {aflops / 1e6:.2f} MFLOP/launch "
        f"-> {tflops:.3f} TFLOP/s")

    conv = None
    if not args.no_conventional:
        sc = s.conventional()
        C = leg(sc)
        stc = C["stats"]
        conv = dict(value=s.n * args.steps / C["t"], ms_per_step=C["t"] * 1e3 / args.steps,
                    ms_per_step_runs=[x * 1e3 / args.steps for x in C["times"]],
                    force_us=C["force_us"], build_us=C["build_us"], cycle_us=C["cycle_us"],
                    atom_entries=stc["atom_entries"])
        log(f"[bench] conventional: {conv['ms_per_step']:.4f} ms/step, {conv['value']:.4e} "
            f"atom-steps/s, force launch {conv['force_us']:.2f} us, build "
            f"{conv['build_us']:.1f} us, entries {stc['atom_entries']}")

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 5 x {nbytes} B read + {nbytes} B written")

    big = None if args.no_batch_roofline else batch_roofline(args.pair_math)
    if big:
        log(f"[bench] batch force launch {big['kernel_us']:.1f} us, {big['achieved']:.0f} GB/s "
            f"algorithmic ({100 * big['frac']:.1f} % of HBM)")

    cpu = None if args.no_cpu_baseline else cpu_baseline(s, args.cpu_budget)
    if cpu:
        log(f"[bench] cpu oracle: {cpu['value']:.4e} atom-steps/s on {cpu['cores']} threads "
            f"({cpu['cpu']})")

    default_path = args.pair_math == 0 and args.lanes is None
    relres_entries = st["atom_entries"] + st["site_entries"]
    hbm_frac = achieved / HBM_PEAK_GBS
    alu_frac = tflops / alu_peak
    hbm_roof = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": hbm_frac,
        "traffic": recorded_traffic(args.workload) if default_path else None,
        "kernel": "k_forces", "kernel_us": force_us,
        "kernel_us_method": "HIP events on the launch stream around replays of a graph of "
                            "10 back-to-back force launches",
        "algorithmic_bytes_per_launch": abytes,
    }
    alu_roof = {
        "bound": "alu", "achieved": tflops, "peak": alu_peak, "unit": "TFLOP/s",
        "frac": alu_frac, "traffic": None, "kernel": "k_forces", "kernel_us": force_us,
        "valu": f"fp{pm_ew} vector (pair terms of calls with energy/virial)",
        "algorithmic_flops_per_launch": aflops,
    }
    # the binding roofline is the one the kernel comes closer to
    primary, secondary = (hbm_roof, alu_roof) if hbm_frac >= alu_frac else (alu_roof, hbm_roof)
    out = {
        "metric": "RelRes atom-steps/s vs conventional 14 Å LJ, 1 MI355X; % FP32/HBM roofline",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if (precision == 32 and pm_ew == 32) else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "atoms": s.n, "sites": int(st["n_sites"]),
            "box_A": float(s.box[0]), "cutoffs_A": [s.rs_in, s.rs_out, s.rc_in, s.rc_out],
            "skin_A": s.skin, "rebuild_every": args.rebuild_every, "seed": args.seed,
            "forces": "fp32" if precision == 32 else "fp64",
            "pair_math": pm_ew, "energy_virial": "fp64 accumulation, every step",
            "parallelism": "single GPU",
            "launch": ("one hip graph per cycle (rebuild + force calls), lists checked once "
                       "per timed run after its closing synchronisation (an overflowed run "
                       "is discarded and repeated)") if use_graph else "eager",
            "timing": f"median of {args.repeats} timed runs of {args.steps} steps after "
                      f"{args.warmup} warm-up steps; kernel timing (graph replays) before them",
        },
        "ms_per_step_runs": [x * 1e3 / args.steps for x in R["times"]],
        "roofline": primary,
        "roofline_other": secondary,
        "roofline_batch": big,
        "kernel_sum_us_per_step": force_us + build_us / args.rebuild_every,
        "cycle_us": R["cycle_us"],
        "cpu_baseline": cpu,
        "conventional": conv,
        "speedup_vs_conventional": (value / conv["value"]) if conv else None,
        "list_entries": {"relres": relres_entries,
                         "conventional": conv["atom_entries"] if conv else None,
                         "N_star": (relres_entries / conv["atom_entries"]) if conv else None},
        "pairs_by_regime": {k: dict(zip(("entries", "inside_cutoff", "smoothing_zone"), v))
                            for k, v in R["counts"].items()},
        "build_us": build_us,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
