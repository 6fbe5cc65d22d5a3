#!/usr/bin/env python3
"""Benchmark of the rod force-and-integrate loop on one MI355X.

Default workload: the rod array, 512 clamped rods of 512 particles
(262,144 particles) under a swept field, all-pairs dipoles, Hookean contact
through candidate lists, mixed path (FP32 pair/bond arithmetic, FP64 state and
sums), steps replayed from captured HIP graphs whose length divides the timed
steps. A step is one full pass of the loop (integrate, bonds, dipoles, contact,
gather and kick) over all particles. Keyed legs run the same array on the
FP64 path, the twisted rod, the cilia carpet (beside the plain per-rod loop)
and the ensemble.

Prints one JSON line: throughput in particle-steps/s (inputs resident in HBM),
dipole pair-evaluations/s, the roofline of the dominant (dipole) kernel timed
with HIP events on the library's stream, and the FP64 CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 67.0        # algorithmic FP32 flops per ordered dipole pair (FMA = 2)
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector peak (vendor figure)
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector peak (vendor figure)
# Algorithmic flops of one ordered real-space pair of the Ewald sum (FMA = 2; the
# square root, exp and erfc one each): 1/r, r, a r, (a r)^2, exp, erfc (6); 1/r^2,
# 1/r^3, 1/r^5, 1/r^7 (4); the shared sp r exp factor (2); the screened B, C, D
# factors (2 + 6 + 9); three dot products (15); the force (33) and field (16)
# terms with C and their accumulation.
EWALD_PAIR_FLOPS = 93.0
METRIC = "particle-steps/s and dipole pair-evals/s (% FP32 peak); adjoint/forward time"

WORKLOADS = {
    "twisted_rod": "twisted clamped-clamped rod, N=4096, contact + all-pairs dipoles",
    "cilia_carpet": "cilia carpet, 1024 rods on 32x32 grid, ~73.7k particles",
    "rod_array": "rod array, 512 rods x 512 particles = 262,144, field sweep",
    "ensemble": "ensemble, 64 members x 4096-particle rods",
    "cantilever": "cantilever, 20 particles, FP64",
    "adjoint_rod": "adjoint rod, N=256, FP64",
}


# Sources that make up the force kernels; a change to any of them voids the
# counter figures recorded for them.
FORCE_SOURCES = ("k_forces.hip", "dipole_body.h", "bond_body.h", "bond_core.h",
                  "contact_body.h", "k_dipole.hip", "rod_internal.h", "rod_math.h")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "force_kernel_counters.md")


def force_sources_digest():
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_27279_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def layout_key(tune_line):
    """'split/1024', 'spatial/32768' or 'small/256' from the autotuner's choice line."""
    m = re.search(r"(small-member|spatial split|split) layout target_wgs=\d+ work_items=(\d+)",
                  tune_line or "")
    if m is None:
        return None
    kind = {"small-member": "small", "spatial split": "spatial", "split": "split"}[m.group(1)]
    return kind + "/" + m.group(2)


def measured_traffic(kernel, workload, precision, layout):
    """HBM bytes per launch recorded from FETCH_SIZE / WRITE_SIZE counter runs
    (scaled by a plain copy of known size), or None when no record matches this
    kernel source, workload, precision and layout."""
    if layout is None or not os.path.exists(COUNTER_SUMMARY):
        return None
    want = {"kernel": kernel.replace(" ", ""), "workload": workload, "precision": precision,
            "layout": layout, "sources": force_sources_digest()}
    with open(COUNTER_SUMMARY) as fh:
        for line in fh:
            if not line.startswith("traffic "):
                continue
            rec = dict(kv.split("=", 1) for kv in line.split()[1:] if "=" in kv)
            if all(rec.get(k) == v for k, v in want.items()):
                try:
                    return float(rec["bytes_per_launch"])
                except (KeyError, ValueError):
                    return None
    return None


def ordered_pairs(w):
    off = np.asarray(w["rod_offset"])
    mem = np.asarray(w["rod_member"])
    sizes = np.zeros(int(w["n_members"]), dtype=np.int64)
    np.add.at(sizes, mem, np.diff(off))
    return int(np.sum(sizes * (sizes - 1)))


def cutoff_neighbours(w):
    """Mean list length of the rod array's dipole lists (cutoff plus the skin
    r_contact / 4), counted on the reference lattice, which the lists see."""
    return _lattice_neighbours(w, w["dipole_cutoff"] + 0.25 * w["r_contact"])


def contact_list_len(w):
    """Mean contact list length of the rod array: partners within r_contact plus
    the skin r_contact / 4 that are not bonded neighbours of the same rod
    (|i - j| <= exclude_depth along the rod)."""
    rad = 1.25 * w["r_contact"]
    same_rod = sum(1 for k in range(1, int(w["exclude_depth"]) + 1) if k < rad)
    return _lattice_neighbours(w, rad) - 2.0 * same_rod


def cutoff_pairs(w):
    """Mean number of partners within the cutoff itself (the pairs evaluated)."""
    return _lattice_neighbours(w, w["dipole_cutoff"])


def _lattice_neighbours(w, rad):
    # the rod array is a lateral grid of straight rods at spacing 1 along z:
    # count lattice points of one interior particle (i, j, k) within rad
    pitch = float(np.linalg.norm(w["x_ref"][w["rod_offset"][1]] - w["x_ref"][0]))
    r = int(np.ceil(rad / min(pitch, 1.0))) + 1
    g = np.arange(-r, r + 1)
    X, Y, Z = np.meshgrid(pitch * g, pitch * g, g, indexing="ij")
    d2 = X * X + Y * Y + Z * Z
    return float(np.count_nonzero((d2 < rad * rad) & (d2 > 0)))


ROW_SAMPLE_PAIRS = 2e9  # above this many dipole pairs per step the oracle is sampled by rows


def _oracle_rate(w, target_s):
    """Oracle throughput in particle-steps/s on the threads currently set. A
    workload whose step exceeds the budget is sampled by rows: the dipole and
    contact sums of evenly spaced particles (each over its whole member), the
    work that makes up all but a fraction of a step of such a size; otherwise
    whole steps from the initial state."""
    import oracle
    n = w["n"]
    pairs = ordered_pairs(w) if w["dipole_on"] else 0
    if pairs > ROW_SAMPLE_PAIRS:
        st = oracle.run(w, 0) if n <= 100_000 else {"x": w["x0"], "q": w["q0"]}
        rows = np.linspace(0, n - 1, num=min(n, 64)).astype(np.int32)
        t0 = time.perf_counter()
        oracle.rows(w, st["x"], st["q"], rows)
        per_row = (time.perf_counter() - t0) / len(rows)
        k = int(max(16, min(n, target_s / max(per_row, 1e-9))))
        rows = np.linspace(0, n - 1, num=k).astype(np.int32)
        t0 = time.perf_counter()
        oracle.rows(w, st["x"], st["q"], rows)
        dt = time.perf_counter() - t0
        return k / dt, (f"dipole and contact sums of {k} of the {n} particles (evenly spaced, "
                        f"each over its member of {n} particles) at the initial state, FP64, "
                        f"{dt:.2f} s; the bond and integration work of a step (under 0.1% of "
                        f"it at this size) is not timed")
    t0 = time.perf_counter()
    st = oracle.run(w, 0)                   # prepare (includes one force evaluation)
    t_prep = time.perf_counter() - t0
    k = int(max(1, min(w["steps"], target_s / max(t_prep, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(w, k, state=st)
    dt = time.perf_counter() - t0
    return n * k / dt, (f"{k} steps of the same workload (N={n}) from its initial state, "
                        f"FP64, {dt:.2f} s")


def cpu_baseline(w, target_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: on every thread
    its OpenMP runtime takes, then on one thread (a smaller sample)."""
    import ctypes
    import oracle
    lib = oracle._load()
    lib.orc_threads.restype = ctypes.c_int
    cores = int(lib.orc_threads())
    value, sample = _oracle_rate(w, target_s)
    lib.orc_set_threads(1)
    try:
        v1, s1 = _oracle_rate(w, max(2.0, target_s / 3))
    finally:
        lib.orc_set_threads(cores)
    model, ncpu = cpu_model()
    return {"value": float(value), "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": sample, "one_core": {"value": float(v1), "sample": s1},
            "cpu_model": model, "logical_cpus": ncpu}


def oracle_timings():
    """The FP64 oracle timed on the host cores, per workload, from its prepared
    initial state: whole runs of the cantilever (1000 steps), the adjoint rod
    (2000) and the twisted rod (20,000), and windows of the cilia carpet (10
    steps) and the rod array (2 steps); then on one thread, with shorter
    windows (the rod array left out). Steps run in chunks with a progress line
    each. Reports seconds, particle-steps/s and ordered dipole pair evaluations
    per second, with the thread count and the CPU model."""
    import ctypes
    import oracle
    import workloads
    lib = oracle._load()
    lib.orc_threads.restype = ctypes.c_int
    cores = int(lib.orc_threads())
    plan = (("cantilever", 1000, 1000), ("adjoint_rod", 2000, 2000), ("twisted_rod", 20000, 200),
            ("cilia_carpet", 10, 1), ("rod_array", 2, 0))
    rows = []
    try:
        for threads in (cores, 1):
            lib.orc_set_threads(threads)
            for name, n_all, n_one in plan:
                steps = n_all if threads == cores else n_one
                if steps == 0:
                    continue
                w = workloads.make(name)
                n = int(w["n"])
                pairs = ordered_pairs(w) if w["dipole_on"] else 0
                print(f"[oracle-timings] {name}: {threads} threads, preparing", file=sys.stderr,
                      flush=True)
                st = oracle.run(w, 0)
                done, secs = 0, 0.0
                chunk = 1
                while done < steps:
                    k = min(chunk, steps - done)
                    t0 = time.perf_counter()
                    st = oracle.run(w, k, state=st)
                    dt = time.perf_counter() - t0
                    done += k
                    secs += dt
                    # chunks of about 20 s between progress lines
                    chunk = max(1, int(k * 20.0 / max(dt, 1e-6)))
                    print(f"[oracle-timings] {name}: {done}/{steps} steps, {secs:.1f} s",
                          file=sys.stderr, flush=True)
                rows.append({"workload": name, "n_particles": n, "threads": threads,
                             "steps": steps, "seconds": secs,
                             "particle_steps_per_s": n * steps / secs,
                             "dipole_pair_evals_per_s": pairs * steps / secs if pairs else None})
    finally:
        lib.orc_set_threads(cores)
    model, ncpu = cpu_model()
    return {"cpu_model": model, "logical_cpus": ncpu, "threads": cores, "rows": rows}


def adjoint_leg():
    """Adjoint cost on the adjoint-rod workload (N = 256, T = 2000, checkpoints
    every 100): wall time of rod_grad against the taped forward run that
    precedes it and against the plain graph-replayed forward run."""
    import torch
    import workloads
    from paper_2603_27279_amd import RodSim
    w = workloads.make("adjoint_rod")
    T = w["steps"]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    plain = RodSim(w, precision="fp64", graph_steps=100)
    plain.step(100)
    plain.sync()
    t_plain = timed(lambda: (plain.step(T), plain.sync()))
    plain.free()
    sim = RodSim(w, precision="fp64", tape_every=w["tape_every"], tape_capacity=T)
    # one untimed pass to warm up every kernel of the reverse pass
    sim.tape_begin()
    sim.step(w["tape_every"])
    sim.grad(gx=torch.zeros((3, w["n"]), dtype=torch.float64, device="cuda"))
    sim.free()
    sim = RodSim(w, precision="fp64", tape_every=w["tape_every"], tape_capacity=T)
    sim.tape_begin()
    t_fwd = timed(lambda: (sim.step(T), sim.sync()))
    st = sim.state()
    gx = np.zeros((w["n"], 3))
    gx[-1] = 2.0 * (st["x"][-1] - w["target"])
    gxt = torch.as_tensor(np.ascontiguousarray(gx.T), device="cuda")
    t_grad = timed(lambda: sim.grad(gx=gxt))
    sim.free()
    return {"workload": f"adjoint rod N={w['n']}, T={T} steps, checkpoints every {w['tape_every']}",
            "forward_ms": 1e3 * t_plain, "forward_taped_ms": 1e3 * t_fwd,
            "grad_ms": 1e3 * t_grad, "adjoint_over_taped_forward": t_grad / t_fwd,
            "adjoint_over_forward": t_grad / t_plain,
            "total_over_forward": (t_fwd + t_grad) / t_plain}


HBM_PEAK_GBS = 8000.0       # MI355X HBM3E (vendor figure)

# Algorithmic bytes per unit of the memory-bound kernels (each datum counted
# once, however often a kernel re-reads it):
#   bond (per bond): x, q of one particle (56), reference vector and length (32),
#     rod id and flags (5), outputs F, tau_s, tau_b+tau_t (72)
#   bond with bond damping: the same, plus the velocity of one particle (24) and
#     the five measures of the previous level read and of this level written (80)
#   Hertz-Mindlin contact (per particle): own x, v, w (72), force and torque out
#     (48), contact counts of the previous and this level (8); per contact, its
#     previous and new partner and tangential displacement (56)
#   dipoles within a cutoff, list walk (per particle): own x and m (48), list
#     count (4), force and field out (48), and 4 per list entry; the partners'
#     x and m are other particles' own data
#   contact list walk (per particle): own position (24), list length (4), force
#     out (24), and 4 per list entry (the member range and rod id are read only
#     by a cell search)
#   pre (per particle): state x v q w F T and m_body, inverse mass and inertia,
#     ids (221 in); x v q w, m in FP64 and FP32 (140 out). With contact lists
#     (these systems) the cell-list entry (key, slot, count: 40 more) is written
#     only at list rebuilds, by the contact launch
#   kick (per particle): bond outputs of its bond (72), dipole slots (24 each on
#     the mixed path, 48 in FP64), contact force, state and constants (318 + slots
#     in); F T x v w q, m twice (188 out; the cell-list entry as for pre)
BYTES = {"bond": 165.0, "bond_damped": 269.0, "contact": 52.0, "contact_hm": 128.0,
         "contact_hm_per_contact": 56.0, "dipole_cutoff": 100.0, "pre": 361.0}


def kick_bytes(slots, slot_bytes=24.0):
    return 318.0 + slot_bytes * slots + 188.0


def hbm_microbench(sizes, steps=10):
    """Bond, contact and integration kernels of a dipole-free rod array at
    millions of particles: kernel time from per-launch HIP events, algorithmic
    bytes per unit as above, achieved GB/s against HBM peak. Contact lists are
    built at the first step of a call and reused after it, so the contact time
    of a one-step call (build) is taken apart from that of the later steps."""
    import workloads
    from paper_2603_27279_amd import RodSim
    out = []

    def entry(us, units, b):
        gbs = units * b / (us * 1e-6) / 1e9
        return {"us": us, "bytes_per_unit": b, "GB_s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}

    copy = copy_bandwidth()
    for side in sizes:
        w = workloads.rod_array(grid=(side, side), n_per_rod=1024, dipole_on=False)
        n, R = w["n"], len(w["rod_offset"]) - 1
        sim = RodSim(w, precision="mixed", graph_steps=0)
        res = {"n_particles": n, "n_bonds": n - R}
        sim.launch_mode("separate")
        sim.step(2)
        timed = {}
        for k in (1, steps + 1):
            sim.timing(True)
            sim.step(k)
            timed[k] = sim.kernel_times()
            sim.timing(False)
        kt = timed[steps + 1]
        res["bond"] = entry(1e3 * kt["bond"][0] / kt["bond"][1], n - R, BYTES["bond"])
        res["pre"] = entry(1e3 * kt["pre"][0] / kt["pre"][1], n, BYTES["pre"])
        # a rebuild step: the cell-list fill and the contact launch that builds
        # the lists; other steps: the walk, after a fill launch that finds the
        # lists current and does nothing (reported as cell_gate_us)
        build_us = 1e3 * (timed[1]["contact"][0] + timed[1]["cells"][0])
        walk_us = 1e3 * (kt["contact"][0] - timed[1]["contact"][0]) / steps
        listed = contact_list_len(w)
        res["contact"] = entry(walk_us, n, BYTES["contact"] + 4.0 * listed)
        res["contact"]["list_entries"] = listed
        res["contact"]["list_build_us"] = build_us
        res["contact"]["cell_gate_us"] = 1e3 * (kt["cells"][0] - timed[1]["cells"][0]) / steps
        sim.launch_mode("batched")
        sim.timing(True)
        sim.step(steps + 1)
        kt = sim.kernel_times()
        sim.timing(False)
        res["kick"] = entry(1e3 * kt["kick"][0] / kt["kick"][1], n, kick_bytes(0))
        sim.free()
        # the bond kernel again with bond damping on every rod
        wd = dict(w, bond_damping=np.tile([0.1, 0.1, 0.1, 0.1], (R, 1)))
        sim = RodSim(wd, precision="mixed", graph_steps=0)
        sim.launch_mode("separate")
        sim.step(2)
        sim.timing(True)
        sim.step(steps)
        kt = sim.kernel_times()
        sim.timing(False)
        sim.free()
        res["bond_damped"] = entry(1e3 * kt["bond"][0] / kt["bond"][1], n - R, BYTES["bond_damped"])
        # and the Hertz-Mindlin search, which walks the cells every step
        wh = dict(w, contact_model="hertz_mindlin", contact_hm=np.array([200.0, 0.3, 0.5, 0.2, 0.2]))
        sim = RodSim(wh, precision="mixed", graph_steps=0)
        sim.launch_mode("separate")
        sim.step(2)
        timed = {}
        for k in (1, steps + 1):
            sim.timing(True)
            sim.step(k)
            timed[k] = sim.kernel_times()
            sim.timing(False)
        per = 2.0 * len(sim.contact_pairs()) / n
        sim.free()
        walk_us = 1e3 * (timed[steps + 1]["contact"][0] - timed[1]["contact"][0]) / steps
        res["contact_hm"] = entry(walk_us, n,
                                  BYTES["contact_hm"] + BYTES["contact_hm_per_contact"] * per)
        res["contact_hm"]["contacts_per_particle"] = per
        res["contact_hm"]["list_build_us"] = 1e3 * (timed[1]["contact"][0] + timed[1]["cells"][0])
        res["contact_hm"]["cell_gate_us"] = 1e3 * (timed[steps + 1]["cells"][0]
                                                   - timed[1]["cells"][0]) / steps
        # dipoles within a cutoff of 3 from the Verlet lists
        wc = dict(w, dipole_on=True, dipole_cutoff=3.0)
        sim = RodSim(wc, precision="mixed", graph_steps=0)
        sim.launch_mode("separate")
        sim.step(2)
        timed = {}
        for k in (1, steps + 1):
            sim.timing(True)
            sim.step(k)
            timed[k] = sim.kernel_times()
            sim.timing(False)
        sim.free()
        walk_us = 1e3 * (timed[steps + 1]["dipole"][0] - timed[1]["dipole"][0]) / steps
        per = cutoff_neighbours(wc)
        res["dipole_cutoff"] = entry(walk_us, n, BYTES["dipole_cutoff"] + 4.0 * per)
        res["dipole_cutoff"].update(
            cutoff=3.0, neighbours_in_list=per, list_build_us=1e3 * timed[1]["dipole"][0],
            pairs_per_s=n * cutoff_pairs(wc) / (walk_us * 1e-6))
        for k in ("bond", "bond_damped", "contact_hm", "dipole_cutoff", "pre", "contact", "kick"):
            res[k]["frac_copy"] = res[k]["GB_s"] / copy["GB_s"]
        res["plain_copy"] = copy
        out.append(res)
    return out


def lbm_leg(n=256, steps=20):
    """The lattice Boltzmann kernel on an n^3 periodic lattice at rest with a
    small body force: time per step from HIP events on the stream it runs on,
    against 304 bytes per cell update (19 populations read and 19 written)."""
    import torch
    from paper_2603_27279_amd import Lattice
    w = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=torch.float64, device="cuda")
    f0 = w.view(19, 1, 1, 1).expand(19, n, n, n).contiguous()
    lat = Lattice(f0, tau=0.8, force=(1e-6, 0.0, 0.0))
    del f0
    lat.step(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / steps
    lat.free()
    cells = n ** 3
    gbs = cells * 304.0 / (us * 1e-6) / 1e9
    return {"lattice": f"{n}^3 D3Q19, FP64", "cells": cells, "us_per_step": us,
            "mlups": cells / us, "bytes_per_cell": 304.0, "GB_s": gbs,
            "frac_hbm": gbs / HBM_PEAK_GBS}


def ibm_leg(grid=16, nsub=10, cycles=20, shape=(96, 128, 128), autotune=True):
    """Cilia immersed in a lattice (rod_lbm_cycles): a grid x grid carpet of
    clamped rods of 16 to 64 particles at pitch 8, in a rotating field, moved 4
    lattice units in from x = y = 0 and 2 up from z = 0, in a periodic lattice
    [nz, ny, nx] = shape at rest, nsub rod steps of dt = 1 / nsub per lattice
    step (mixed precision rods, FP64 fluid), the rods' dipole layout autotuned
    first. Time per cycle from HIP events on the calling stream, beside the
    lattice step alone on the same lattice."""
    import torch
    import workloads
    from paper_2603_27279_amd import Lattice, RodSim
    w = workloads.cilia_carpet(grid=(grid, grid), pitch=8.0, len_range=(16, 64), dt=1.0 / nsub)
    for k in ("x0", "x_ref"):
        w[k] = np.asarray(w[k]) + np.array([4.0, 4.0, 2.0])
    nz, ny, nx = shape
    assert np.all(w["x0"].max(0) < np.array([nx, ny, nz]))
    wt = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=torch.float64, device="cuda")
    f0 = wt.view(19, 1, 1, 1).expand(19, nz, ny, nx).contiguous()
    sim = RodSim(w, precision=w["precision"])
    tune = sim.autotune(None).strip().splitlines()[-1] if autotune else None
    lat = Lattice(f0, tau=0.8)
    del f0
    sim.lbm_cycles(lat, nsub, 2)
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return 1e3 * e0.elapsed_time(e1) / cycles

    us = timed(lambda: sim.lbm_cycles(lat, nsub, cycles))
    us_lat = timed(lambda: lat.step(cycles))
    sim.sync()  # reports non-finite states or list overflow
    n, cells = int(w["n"]), nx * ny * nz
    sim.free()
    lat.free()
    return {"workload": f"{grid}x{grid} cilia carpet (16-64 particles) in a {nx}x{ny}x{nz} periodic lattice",
            "particles": n, "cells": cells, "n_sub": nsub, "us_per_cycle": us,
            "us_lattice_step": us_lat, "us_rods_and_coupling": us - us_lat,
            "particle_steps_per_s": n * nsub / (us * 1e-6), "mlups": cells / us,
            "dipole_layout": tune}


def ewald_leg(grid=32, length=32, box=(64.0, 64.0, 40.0), rcut=16.0, steps=20):
    """Rods in a periodic box with the Ewald sum of their dipoles: the rod array
    at 32 x 32 rods of 32 particles (32,768) at pitch 2, without contact, in a
    64 x 64 x 40 box (the lateral pitch continues across the boundary), real-
    space cutoff 16 (cells of a third of it: 12 per axis in x and y, 7 in z),
    alpha = 3.6 / rcut and kmax
    = ceil(3.6 alpha max(L) / pi) (both truncated tails near exp(-13)). Whole
    steps replayed from a graph, and the Ewald part of a step (its ten
    launches, bracketed by events) on its own."""
    import torch
    import workloads
    from paper_2603_27279_amd import RodSim
    w = workloads.rod_array(grid=(grid, grid), n_per_rod=length, pitch=2.0, contact_on=False)
    alpha = 3.6 / rcut
    w.update(box=np.asarray(box, float), ewald_rcut=rcut, ewald_alpha=alpha,
             ewald_kmax=int(np.ceil(3.6 * alpha * max(box) / np.pi)))
    n = w["n"]
    sim = RodSim(w, precision="mixed", graph_steps=steps)
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    sim.timing(True)
    sim.step(5)
    kt = sim.kernel_times()
    sim.timing(False)
    x_end = np.asarray(sim.state()["x"], dtype=np.float64)
    sim.free()
    ew_ms = kt["dipole"][0] / kt["dipole"][1]
    real_ms = kt["ewald_real"][0] / kt["ewald_real"][1]
    # real-space pairs (i, j) closer than rcut by the minimum image, each
    # evaluated once per particle of the pair (ordered pairs)
    from scipy.spatial import cKDTree
    bx = np.asarray(box, float)
    tree = cKDTree(np.mod(x_end, bx), boxsize=bx)
    ordered = int(tree.count_neighbors(tree, rcut)) - n
    kmax = w["ewald_kmax"]
    nk = sum(1 for a in range(0, kmax + 1) for b in range(-kmax, kmax + 1)
             for c in range(-kmax, kmax + 1)
             if (a > 0 or (a == 0 and (b > 0 or (b == 0 and c > 0)))) and a * a + b * b + c * c <= kmax * kmax)
    return {"workload": f"{grid}x{grid} rods x {length} particles in a periodic "
                        f"{box[0]:g} x {box[1]:g} x {box[2]:g} box, Ewald sum (rcut {rcut:g}, "
                        f"alpha {alpha:.4f}, kmax {kmax}), mixed precision rods",
            "particles": n, "ms_per_step": ms, "particle_steps_per_s": n / (ms * 1e-3),
            "ewald_ms_per_evaluation": ew_ms,
            "real_space_ms_per_evaluation": real_ms,
            "real_space_pairs_per_particle": ordered / n,
            "roofline": {"bound": "alu", "kernel": "k_ew_real<float>",
                         "achieved": ordered * EWALD_PAIR_FLOPS / (real_ms * 1e-3) / 1e12,
                         "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ordered * EWALD_PAIR_FLOPS / (real_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                         "flops_per_pair": EWALD_PAIR_FLOPS, "ordered_pairs": ordered,
                         "traffic": None},
            "reciprocal_vectors_half_space": nk,
            "reciprocal_terms_per_s": 2.0 * nk * n / (ew_ms * 1e-3)}


def copy_bandwidth(mib=512, reps=20):
    """What a plain device-to-device copy reaches on this GPU (bytes read plus
    bytes written per second, median of `reps` launches): the practical ceiling
    the memory-bound kernels are compared with, besides the vendor peak."""
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3)
    us = sorted(times)[len(times) // 2]
    gbs = 2 * 8 * n / (us * 1e-6) / 1e9
    del a, b
    return {"MiB_each_way": mib, "us": us, "GB_s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}


def helix_loop(gamma, ke_tol=1e-9, max_steps=200_000, check_every=2000, dlam=0.1, lam_max=3.5,
               precision="mixed"):
    """The magnetic helix's loading-unloading cycle (results, "Helical rods with
    dipole-dipole interactions"): lambda_m from 0 to lam_max and back in steps
    of dlam, each setting held by the quasi-static ramp (rod_ramp) until the
    helix is at rest. Reports the distance between the helix ends along the
    screw axis over L for every setting, the steps each took, and where the
    largest jumps occur on the way up (detachment) and down (contraction).
    Prints one progress line per setting to stderr."""
    import torch
    import workloads
    from paper_2603_27279_amd import RodSim
    up = np.round(np.arange(0.0, lam_max + 1e-9, dlam), 10)
    lams = np.concatenate([up, up[::-1][1:]])
    w = workloads.magnetic_helix(gamma=gamma)
    f = workloads.helix_ramp_fields(w, lams)
    sim = RodSim(dict(w, field=f[:1]), precision=precision, graph_steps=100)
    t0 = time.perf_counter()
    dist, steps = [], []
    for k in range(len(lams)):
        r = sim.ramp(f[k:k + 1], max_steps=max_steps, check_every=check_every, ke_tol=ke_tol,
                     watch=[0, w["n"] - 1])
        dist.append(float(abs(r["x_watch"][0, 1, 2] - r["x_watch"][0, 0, 2]) / w["helix"]["length"]))
        steps.append(int(r["steps"][0]))
        print(f"helix gamma={gamma:g} lambda_m={lams[k]:.2f}: distance/L {dist[-1]:.4f}, "
              f"{steps[-1]} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.free()
    n = len(up)
    d_up, d_down = np.array(dist[:n]), np.array(dist[n - 1:][::-1])
    jump_up = int(np.argmax(np.diff(d_up))) + 1
    jump_down = int(np.argmax(-np.diff(d_down[::-1]))) + 1
    return {"workload": f"magnetic helix, N = {w['n']}, gamma = {gamma:g}, {precision}",
            "lambda_m": up.tolist(), "distance_up": d_up.tolist(), "distance_down": d_down.tolist(),
            "steps": steps, "settings_at_step_limit": int(sum(s >= max_steps for s in steps)),
            "detach_lambda_m": float(up[jump_up]),
            "contract_lambda_m": float(up[::-1][jump_down]),
            "total_steps": int(sum(steps)), "wall_s": wall,
            "us_per_step": 1e6 * wall / max(1, sum(steps))}


TERMS = (("bond", 1), ("dipole", 2), ("zeeman", 4), ("contact", 8), ("damping", 16),
         ("total", 63))


def _member0(w):
    """The first member of an ensemble workload as a workload of its own (its
    rods, particles and field column; no arithmetic)."""
    off = np.asarray(w["rod_offset"])
    mem = np.asarray(w["rod_member"])
    R = int(np.count_nonzero(mem == 0))
    n = int(off[R])
    v = dict(w)
    v.update(n=n, rod_offset=off[:R + 1].copy(), rod_member=mem[:R].copy(), n_members=1,
             rod_params=np.asarray(w["rod_params"])[:R].copy(),
             field=np.ascontiguousarray(np.asarray(w["field"])[:, :1, :]))
    for k in ("x_ref", "x0", "v0", "w0", "q0", "m_body", "bc"):
        v[k] = np.asarray(w[k])[:n].copy()
    v["name"] = w["name"] + "_member0"
    return v


def error_table(steps=100):
    """Error of the GPU path against the FP64 oracle per quantity, on both
    paths: ||dF||_inf / ||F||_inf and ||dT||_inf / ||T||_inf of each force term
    alone and of their sum, at the initial level and at the GPU's state after
    `steps` steps (both sides evaluating the same state); and after `steps`
    steps of each side, x relative to the motion ||x_T - x_0||_inf, q relative
    to its change ||q_T - q_0||_inf, and v, w, F, T relative to their own
    ||.||_inf. Terms whose reference is zero are reported as null."""
    import workloads
    from paper_2603_27279_amd import RodSim
    import oracle

    def rel(a, b):
        den = float(np.max(np.abs(b))) if b.size else 0.0
        return None if den == 0.0 else float(np.max(np.abs(a - b))) / den

    cases = [("cantilever", workloads.cantilever()),
             ("twisted_rod", workloads.twisted_rod()),
             ("adjoint_rod", workloads.adjoint_rod()),
             ("cilia_carpet_2x2", workloads.cilia_carpet(grid=(2, 2))),
             ("ensemble_member0", _member0(workloads.ensemble())),
             ("coiled_rods", workloads.coiled_rods()),
             ("periodic_rods", workloads.periodic_rods(n_rods=8, length=16))]
    out = {}

    def per_term(sim, w, g, row, tag):
        # each force term alone at the given state (the GPU's own), both sides
        for term, mask in TERMS:
            Fo, To = oracle.forces(w, g["x"], g["q"], g["v"], g["w"], mask=mask, step=g["step"])
            F, T = sim.eval_forces(mask)
            row[f"{tag}F_{term}"] = rel(F.cpu().numpy().T, Fo)
            row[f"{tag}T_{term}"] = rel(T.cpu().numpy().T, To)

    for name, w in cases:
        print(f"[error-table] {name}: oracle, {steps} steps", file=sys.stderr, flush=True)
        stT = oracle.run(w, steps)
        for prec in ("fp64", "mixed"):
            sim = RodSim(w, precision=prec)
            row = {"n_particles": int(w["n"])}
            per_term(sim, w, sim.state(), row, "")
            sim.step(steps)
            sim.sync()
            g = sim.state()
            per_term(sim, w, g, row, f"step{steps}_")
            sim.free()
            row["x"] = rel(g["x"] - w["x0"], stT["x"] - w["x0"])
            row["q"] = rel(g["q"] - w["q0"], stT["q"] - w["q0"])
            for k in ("v", "w", "F", "T"):
                row[k] = rel(g[k], stT[k])
            out[f"{name}/{prec}"] = row
            print(f"[error-table] {name} {prec}", file=sys.stderr, flush=True)
    return {"steps": steps, "rows": out}


def copy_calibration():
    """A plain device copy of a known size (256 MiB read, 256 MiB written, three
    times), for scaling the FETCH_SIZE and WRITE_SIZE counters to bytes."""
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": 8 * n,
                                           "bytes_written_per_launch": 8 * n, "launches": 3}}),
          flush=True)


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo) and the number of
    logical CPUs the OS reports."""
    name = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def measured_peaks():
    """Arithmetic ceilings measured on this GPU by rod_probe_fma (independent FMA
    chains in vector registers, unpacked FP32 as the library's own code; FP64)."""
    import ctypes
    import torch
    from paper_2603_27279_amd import _lib as L
    lib = L.load()
    out = {}
    for key, prec, dt in (("fp32_fma_tflops", L.ROD_MIXED, torch.float32),
                          ("fp64_fma_tflops", L.ROD_FP64, torch.float64)):
        sink = torch.zeros(1, dtype=dt, device="cuda")
        tf = ctypes.c_double()
        L.check(lib.rod_probe_fma(prec, ctypes.c_void_p(sink.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.byref(tf)))
        out[key] = tf.value
    return out


def graph_plan(graph_steps, steps):
    """Graph length for a timed call of `steps` steps: at most `steps`, so that
    the call replays whole graphs (rod_step replays only calls of at least the
    graph length). Returns (graph length, steps replayed, steps run eagerly)."""
    gs = max(0, min(int(graph_steps), int(steps)))
    replayed = (steps // gs) * gs if gs > 0 else 0
    return gs, replayed, steps - replayed


def workload_leg(name, prec, steps, warmup, graph_steps, timing_steps, per_rod_steps,
                 tune_cache=None, autotune=True, dipole_cutoff=0.0, separate=True, peaks=None):
    """One workload: whole steps replayed from captured HIP graphs and timed by
    wall clock between stream synchronisations; then the launches of the same
    number of steps timed one by one with HIP events on the library's stream
    (eager), for the dominant kernel's roofline; optionally the plain per-rod
    loop over a few steps."""
    import torch
    import workloads
    from paper_2603_27279_amd import RodSim
    w = workloads.make(name)
    if dipole_cutoff > 0:
        w["dipole_cutoff"] = dipole_cutoff
    n = w["n"]
    pairs = ordered_pairs(w) if w["dipole_on"] and not dipole_cutoff else 0
    gs, replayed, _ = graph_plan(graph_steps, steps)
    sim = RodSim(w, precision=prec, graph_steps=gs)
    tune = None
    if autotune:
        report = sim.autotune(tune_cache).strip().splitlines()
        for line in report[:-1]:  # the candidates' timings (none for a cached choice)
            print(f"[bench] {name} {prec} autotune: {line}", file=sys.stderr, flush=True)
        tune = report[-1]
    # the warm-up holds at least one whole graph, so that its capture is never
    # part of the timed steps
    warm = max(warmup, gs)
    sim.step(warm)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ms_step = 1e3 * secs / steps

    # Kernel durations: every launch stamps a pair of HIP events with its own
    # start and end, on the library's stream (eager launches of the same step).
    t_steps = max(1, min(timing_steps, steps))
    sim.timing(True)
    sim.step(t_steps)
    kt = sim.kernel_times()
    sim.timing(False)
    kt_sep = None
    if separate:
        sim.launch_mode("separate")
        sim.step(1)  # untimed: the separate kernels' first launch loads their code
        sim.sync()
        sim.timing(True)
        sim.step(min(t_steps, 5))
        kt_sep = sim.kernel_times()
        sim.timing(False)
        sim.launch_mode("batched")
    sim.sync()
    roof = None
    if pairs:
        # dominant kernel of the step: the fused force kernel (it holds the
        # dipole work of either layout), else the separate dipole kernel
        cls = "forces" if kt["forces"][1] else "dipole"
        t_k = 1e-3 * kt[cls][0] / kt[cls][1]
        real = "float" if prec == "mixed" else "double"
        small = "small-member" in (tune or "")
        if cls == "forces":
            kname = f"k_forces<{real}, {'true' if n < 65536 else 'false'}>"
        else:
            kname = f"k_dipole_small<{real}>" if small else f"k_dipole<{real}>"
        peak = FP32_PEAK_TFLOPS if prec == "mixed" else FP64_PEAK_TFLOPS
        achieved = FLOP_PER_PAIR * pairs / t_k / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kname, name, prec, layout_key(tune)),
                "traffic_unit": "bytes per launch", "kernel": kname,
                "kernel_us": 1e6 * t_k, "launches_timed": int(kt[cls][1]),
                "kernel_us_covers": "the launch's own events; with the spatial layout they also "
                                    "bracket the chunk-box kernel launched just before it"
                                    if "spatial" in (tune or "") else "the launch's own events",
                "flops_counted": "dipole pair arithmetic only (bond and contact work in the "
                                 "same launch is not counted)" if cls == "forces" else "dipole pairs",
                "pair_evals_per_s": pairs / t_k,
                "flop_per_pair": FLOP_PER_PAIR, "pairs_per_launch": pairs}
        if peaks:
            mp = peaks["fp32_fma_tflops" if prec == "mixed" else "fp64_fma_tflops"]
            roof["measured_peak"] = mp
            roof["frac_measured_peak"] = achieved / mp
    batching = None
    n_rods = len(w["rod_offset"]) - 1
    if n_rods > 1 and per_rod_steps > 0:
        # the same step as a plain per-rod loop (every kernel once per rod, eager)
        k = max(1, min(steps, per_rod_steps))
        sim.launch_mode("per_rod")
        sim.step(1)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(k)
        sim.sync()
        torch.cuda.synchronize()
        ms_rod = 1e3 * (time.perf_counter() - t0) / k
        sim.launch_mode("batched")
        batching = {"n_rods": n_rods, "per_rod_ms_per_step": ms_rod, "per_rod_steps": k,
                    "batched_ms_per_step": ms_step, "speedup": ms_rod / ms_step}
    sim.free()
    return {
        "w": w, "value": n * steps / secs, "ms_per_step": ms_step, "steps": steps,
        "warmup_steps_run": warm, "graph_steps": gs, "graph_replayed_steps": replayed,
        "eager_steps": steps - replayed, "pairs": pairs, "tune": tune,
        "pair_evals_per_s": pairs * steps / secs if pairs else None,
        "kernel_us": {k: 1e3 * ms / c for k, (ms, c) in kt.items() if c},
        "kernel_us_separate_terms": (None if kt_sep is None else
                                     {k: 1e3 * ms / c for k, (ms, c) in kt_sep.items() if c}),
        "roofline": roof, "batching": batching,
    }


def leg_summary(name, prec, r):
    """The keyed form of a workload leg in the bench line."""
    return {"workload": WORKLOADS[name], "precision": prec, "n_particles": r["w"]["n"],
            "particle_steps_per_s": r["value"], "ms_per_step": r["ms_per_step"],
            "steps": r["steps"], "graph_steps": r["graph_steps"],
            "graph_replayed_steps": r["graph_replayed_steps"],
            "pair_evals_per_s": r["pair_evals_per_s"], "dipole_layout": r["tune"],
            "kernel_us": r["kernel_us"], "roofline": r["roofline"], "batching": r["batching"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="rod_array", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--graph-steps", type=int, default=200,
                    help="steps per captured graph (at most --steps, so that the timed "
                         "steps replay whole graphs)")
    ap.add_argument("--timing-steps", type=int, default=200,
                    help="eager steps timed launch by launch (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the FP64 oracle per workload on the host cores")
    ap.add_argument("--no-per-rod", action="store_true",
                    help="skip the per-rod loop comparison (multi-rod workloads)")
    ap.add_argument("--per-rod-steps", type=int, default=3)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other workloads (FP64 rod array, twisted rod, cilia "
                         "carpet, ensemble)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines cache of autotuner choices (default: tune every run)")
    ap.add_argument("--no-microbench", action="store_true",
                    help="skip the bond/contact/integration kernels at millions of particles")
    ap.add_argument("--microbench-sizes", default="64,128",
                    help="comma-separated grid sides of the dipole-free rod array (x 1024 "
                         "particles per rod): 64 -> 4.2M particles, 128 -> 16.8M")
    ap.add_argument("--no-lbm", action="store_true",
                    help="skip the lattice Boltzmann kernel on a 256^3 lattice")
    ap.add_argument("--no-ibm", action="store_true",
                    help="skip the cilia carpet immersed in a lattice (rod_lbm_cycles)")
    ap.add_argument("--no-ewald", action="store_true",
                    help="skip the rods in a periodic box with the Ewald dipole sum")
    ap.add_argument("--ibm", action="store_true",
                    help="only run the immersed cilia carpet and print it as JSON")
    ap.add_argument("--error-table", action="store_true",
                    help="only measure the per-quantity error against the FP64 oracle (initial "
                         "forces per term, 100-step state) on both paths and print it as JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy (counter calibration) and exit")
    ap.add_argument("--dipole-cutoff", type=float, default=0.0,
                    help="dipole-dipole interaction only within this distance (0: all pairs; "
                         "no roofline line then: the pair count is not the all-pairs one)")
    ap.add_argument("--helix-loop", type=float, default=None, metavar="GAMMA",
                    help="only run the magnetic helix's quasi-static loading-unloading cycle "
                         "at this dipole strength (about 3 minutes) and print it as JSON")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_timings:
        print(json.dumps({"oracle_timings": oracle_timings()}))
        return
    if args.error_table:
        print(json.dumps({"error_table": error_table()}))
        return
    if args.helix_loop is not None:
        print(json.dumps({"helix_loop": helix_loop(args.helix_loop)}))
        return
    if args.ibm:
        print(json.dumps({"ibm": ibm_leg()}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("--steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import workloads

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    peaks = measured_peaks()
    progress(f"measured FMA ceilings {peaks}")
    prec = args.precision or workloads.make(args.workload)["precision"]
    head = workload_leg(args.workload, prec, args.steps, args.warmup, args.graph_steps,
                        args.timing_steps, 0 if args.no_per_rod else args.per_rod_steps,
                        args.tune_cache, not args.no_autotune, args.dipole_cutoff, peaks=peaks)
    w = head["w"]
    n = w["n"]
    progress(f"{args.workload} {prec}: {head['ms_per_step']:.3f} ms per step")

    legs = None
    if not args.no_legs and args.workload == "rod_array" and not args.dipole_cutoff:
        legs = {}
        # the rod array on the FP64 path (the paper's own arithmetic)
        r = workload_leg("rod_array", "fp64", 5, 2, 5, 5, 0, args.tune_cache,
                         not args.no_autotune, separate=False, peaks=peaks)
        legs["rod_array_fp64"] = leg_summary("rod_array", "fp64", r)
        progress(f"rod_array fp64: {r['ms_per_step']:.3f} ms per step")
        for name, steps, gsteps, prs in (("twisted_rod", 2000, 200, 0),
                                         ("cilia_carpet", 100, 50, args.per_rod_steps),
                                         ("ensemble", 200, 100, 0)):
            pr = workloads.make(name)["precision"]
            r = workload_leg(name, pr, steps, gsteps, gsteps, min(steps, 50),
                             0 if args.no_per_rod else prs, args.tune_cache,
                             not args.no_autotune, separate=False, peaks=peaks)
            legs[name] = leg_summary(name, pr, r)
            progress(f"{name} {pr}: {r['ms_per_step']:.4f} ms per step")

    adj = None if args.no_adjoint else adjoint_leg()
    micro = None
    if not args.no_microbench:
        micro = hbm_microbench([int(v) for v in args.microbench_sizes.split(",") if v])
        progress("memory-bound kernels done")

    lbm_res = None
    if not args.no_lbm:
        lbm_res = lbm_leg()
        if micro:
            lbm_res["frac_copy"] = lbm_res["GB_s"] / micro[0]["plain_copy"]["GB_s"]
    ibm_res = None if args.no_ibm else ibm_leg()
    ewald_res = None if args.no_ewald else ewald_leg()

    cpu = None
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": head["warmup_steps_run"],
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair/bond arithmetic, f64 state and sums" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_particles": n,
                   "ordered_dipole_pairs_per_step": head["pairs"], "precision": prec,
                   "graph_steps": head["graph_steps"],
                   "graph_replayed_steps": head["graph_replayed_steps"],
                   "eager_steps": head["eager_steps"], "dipole_layout": head["tune"],
                   "dipole_cutoff": args.dipole_cutoff or None},
        "pair_evals_per_s": head["pair_evals_per_s"],
        "kernel_us": head["kernel_us"],
        "kernel_us_separate_terms": head["kernel_us_separate_terms"],
        "roofline": head["roofline"],
        "measured_peaks": peaks,
        "batching": head["batching"],
        "legs": legs,
        "lbm": lbm_res,
        "ibm": ibm_res,
        "ewald": ewald_res,
        "adjoint": adj,
        "hbm_kernels": micro,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
