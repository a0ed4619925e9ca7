"""Throughput benchmark of the dimensional-LBM hot path on one MI355X.

Workload: the stationary-bubble case (D2Q9 MRT pressure populations + D2Q9
conservative Allen-Cahn populations, 256 x 256 periodic cell, liquid/gas
density ratio ~43 300, viscosity ratio ~470, radii cycling over 20/30/40/50
nodes with seeded centre jitter) run as a batch of independent replicas, FP32
deviation storage.  One step = one stream-collide update of every node of
every replica; by default the library's two-step kernel performs two steps
per launch (--fusion 1 times the single-step kernel instead).  Inputs are
synthetic and resident in HBM before timing starts.

Prints ONE JSON line (see the keys below).  ``--gpus`` above 1 is refused:
this benchmark measures one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lattice update (each population read once and written
# once): z 9 + h 9 + low part of h_0 + (phi u) 2, read + write
BYTES_PER_LU = {"fp32": (9 + 9 + 1 + 2) * 4 * 2, "fp64": (9 + 9 + 2) * 8 * 2}
# FP32 storage with FP64 step arithmetic moves the FP32 bytes
BYTES_PER_LU["fp32_arith64"] = BYTES_PER_LU["fp32"]
# heated channel (D2Q9 f + D2Q5 g), read + write
CHAN_BYTES_PER_LU = {"fp32": (9 + 5) * 4 * 2, "fp64": (9 + 5) * 8 * 2}
# D3Q19 momentum, read + write
D3_BYTES_PER_LU = {"fp32": 19 * 4 * 2, "fp64": 19 * 8 * 2}
# 3D two-phase: h 19 (+ low part of h_0 in FP32) + z 19 + (phi u) 3, read + write
P3_BYTES_PER_LU = {"fp32": (19 + 1 + 19 + 3) * 4 * 2, "fp64": (19 + 19 + 3) * 8 * 2}
# the files whose contents decide the step kernel's machine code and the
# buffer layout it streams through
KERNEL_SOURCES = ("paper_2302_04120_amd/csrc/lbm_kernels.hip", "paper_2302_04120_amd/csrc/lbm_device.h",
                  "paper_2302_04120_amd/csrc/lbm_internal.h", "paper_2302_04120_amd/csrc/build.py",
                  "paper_2302_04120_amd/csrc/lbm_api.hip")


def kernel_source_hash():
    """SHA-256 over the step kernel's sources and build flags: the counter
    traffic stored beside the profiles is reported only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(L, steps):
    """HIP events on the library's stream around lbm_step(steps), and the
    host wall time of the same interval: (event ms, wall s)."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(L.stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(L.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), time.perf_counter() - t0


def sustained(L, nodes, ms_per_step, windows=5, seconds=1.0, even=True):
    """Throughput over `windows` windows of at least `seconds` each: the
    median, min and max MLUPS (HIP events) and the steps per window."""
    n = max(2, int(np.ceil(seconds * 1e3 / max(ms_per_step, 1e-6))))
    if even:
        n += n & 1
    rates = []
    for _ in range(windows):
        ms, _ = timed(L, n)
        rates.append(nodes * n / (ms * 1e-3) / 1e6)
    return dict(median_mlups=float(np.median(rates)), min_mlups=float(min(rates)),
                max_mlups=float(max(rates)), windows=windows, steps_per_window=n)


def direct_launches(L):
    """Roofline-sized legs launch every step directly: their kernels run for
    milliseconds, so replaying captured graphs saves nothing, and the one-time
    capture would fall inside the timed steps (the library captures a graph
    on the first call of at least twice its graph length)."""
    L.set_graph_steps(0)


def run_gpu(batch, steps, warmup, prec, n=256, fusion=0, windows=0):
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini, _ = WL.bubble(n=n, batch=batch, seed=0)
    L = lbm.Lattice("phase", n, n, batch=batch, prec=prec)
    if batch >= 64:  # the small paper-sized batches stay launch-bound: graphs help them
        direct_launches(L)
    L.set_step_fusion(fusion)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    del ini
    phase0 = L.reduce(("phase",))["phase"]
    L.step(warmup)
    stream = L.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    nodes = batch * n * n
    out = dict(wall=wall, ev_ms=ev_ms, nodes=nodes, kernel_ms=ev_ms / steps,
               bytes_gb=L.bytes / 1e9)
    if windows:
        out["sustained"] = sustained(L, nodes, ev_ms / steps, windows)
    red = L.reduce(("phase", "nonfinite"))
    if red["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    # sum of phi per replica, FP64 reduction: drift over every step of the run
    # (warm-up, timed steps and the sustained windows)
    out["phi_sum_drift"] = float((abs(red["phase"] - phase0) / abs(phase0)).max())
    out["phi_sum_steps"] = int(L.t)
    L.close()
    return out


def run_wide(cells, steps, warmup, prec, fusion=0):
    """One periodic domain of cells x cells bubble cells (256^2 each, radii
    cycling, jitter per cell): 32 x 32 gives the 8192^2 bubble array.  Its
    rows are wider than 256 nodes, so the two-step kernel takes them in
    x-tiles of 250 stored columns."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini, _ = WL.bubble_array(cells, 256, seed=0)
    n = cells * 256
    L = lbm.Lattice("phase", n, n, prec=prec)
    direct_launches(L)
    L.set_step_fusion(fusion)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    del ini
    L.step(warmup)
    ms, wall = timed(L, steps)
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    L.close()
    nodes = n * n
    spl = 2 if fusion != 1 else 1
    launch_ms = ms / steps * spl
    return dict(mlups=nodes * steps / (ms * 1e-3) / 1e6, grid="%dx%d" % (n, n),
                ms_per_step=ms / steps, launch_ms=launch_ms,
                hbm_frac=BYTES_PER_LU[prec] * nodes / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                kernel="k_phase_tb2<%s, true, %s>" % ("float" if prec == "fp32" else "double",
                                                      "true" if n % 64 == 0 else "false")
                if spl == 2 else "k_phase")


def run_channel(nx, ny, steps, warmup, prec, fusion=1):
    """The heated-channel step (D2Q9 MRT flow + D2Q5 thermal, velocity inlet,
    pressure outlet, flux walls) on a roofline-sized grid; fusion 2 runs two
    steps per launch (the state crosses HBM once per two steps)."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini = WL.channel(nx=nx, ny=ny)
    L = lbm.Lattice("channel", nx, ny, prec=prec,
                    bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    direct_launches(L)
    L.set_params(prm)
    L.set_step_fusion(fusion)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    del ini
    L.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(L.stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(L.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1) / steps
    nodes = nx * ny
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    L.close()
    S = "float" if prec == "fp32" else "double"
    two = fusion != 1  # the library's choice at this size is the two-step kernel
    per_step = CHAN_BYTES_PER_LU[prec] * nodes / (2 if two else 1)  # bytes a step moves
    return dict(mlups=nodes * steps / wall / 1e6, kernel_ms=kernel_ms,
                hbm_frac=per_step / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                grid="%dx%d" % (nx, ny), fusion=fusion,
                kernel=("k_chan_tb2<%s, %s, false, 5>" % (S, "true" if nx % 64 == 0 else "false")
                        if two else "k_chan_step<%s, 5>" % S))


def run_d3(n, steps, warmup, prec, mrt=True):
    """The D3Q19 momentum step (dimensional MRT with Guo forcing) on an n^3
    periodic box of water with a random velocity field."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini = WL.box3d(n, n, n, seed=0, F=(30.0, 20.0, -10.0), mrt=mrt)
    L = lbm.Lattice("d3q19", n, n, prec=prec, nz=n)
    direct_launches(L)
    L.set_params(prm)
    L.init3d(ini["rho"], ini["ux"], ini["uy"], ini["uz"])
    del ini
    L.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(L.stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(L.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    kernel_ms = e0.elapsed_time(e1) / steps
    nodes = n ** 3
    L.close()
    gbs = D3_BYTES_PER_LU[prec] * nodes / (kernel_ms * 1e-3) / 1e9
    return dict(mlups=nodes * steps / wall / 1e6, kernel_ms=kernel_ms, hbm_GBps=gbs,
                hbm_frac=gbs / HBM_PEAK_GBS, grid="%d^3" % n, collision="mrt" if mrt else "bgk",
                kernel="k_d3_step<%s>" % ("float" if prec == "fp32" else "double"))


def run_p3(n, steps, warmup, prec, cell=64, R_nodes=16.0):
    """The 3D two-phase step (phi pass + step kernel) on an n^3 periodic box
    filled with air spheres of radius R_nodes in water, one per cell^3 (the
    air-water system of the Sec. 4.3 property table, density ratio 842)."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    props = {k: v for k, v in WL.TWO_PHASE_SYSTEMS["air_water_25C"].items()
             if k not in ("zeta_l", "zeta_g")}
    prm, ini = WL.bubble3d(n=cell, R_nodes=R_nodes, seed=0, **props)
    reps = (1, n // cell, n // cell, n // cell)
    ini = {k: np.tile(v, reps) for k, v in ini.items()}
    L = lbm.Lattice("phase3d", n, n, prec=prec, nz=n)
    direct_launches(L)
    L.set_params(prm)
    L.init3d(ini["p"], ini["ux"], ini["uy"], ini["uz"], ini["phi"])
    del ini
    L.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(L.stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(L.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    step_ms = e0.elapsed_time(e1) / steps
    nodes = n ** 3
    L.close()
    gbs = P3_BYTES_PER_LU[prec] * nodes / (step_ms * 1e-3) / 1e9
    return dict(mlups=nodes * steps / wall / 1e6, step_ms=step_ms, state_GBps=gbs,
                state_frac=gbs / HBM_PEAK_GBS, grid="%d^3" % n,
                kernels="k_p3_phi<%s> + k_p3_step<%s,false>" % ((("float",) * 2) if prec == "fp32"
                                                               else (("double",) * 2)))


def run_layered_batch(batch, steps, warmup, prec):
    """C4's layered two-phase channel (4 x 512 nodes, walls) as a batch of
    independent replicas: the roofline-sized form of a launch-bound case."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini, _ = WL.layered(nx=4, ny=512, batch=batch, seed=0)
    L = lbm.Lattice("phase", 4, 512, batch=batch, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
    direct_launches(L)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    del ini
    L.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(L.stream)
    t0 = time.perf_counter()
    L.step(steps)
    e1.record(L.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations after the timed steps")
    step_ms = e0.elapsed_time(e1) / steps
    nodes = batch * 4 * 512
    L.close()
    gbs = BYTES_PER_LU[prec] * nodes / (step_ms * 1e-3) / 1e9
    return dict(mlups=nodes * steps / wall / 1e6, step_ms=step_ms, hbm_GBps=gbs,
                hbm_frac=gbs / HBM_PEAK_GBS, replicas=batch, grid="4x512")


def run_c4_single(steps=20000, warmup=200, prec="fp32"):
    """One C4 replica (4 x 512 nodes, walls), launch-bound: microseconds per
    step with graph replay of single-step launches and with the many-steps
    kernel (step fusion mode 3), and whether the two end in the same state."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini, _ = WL.layered(nx=4, ny=512, batch=1, seed=0)
    out = {}
    states = {}
    for name, fusion, graph in (("graph_replay", 1, 64), ("many_steps", 3, 0)):
        L = lbm.Lattice("phase", 4, 512, batch=1, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
        L.set_step_fusion(fusion)
        L.set_graph_steps(graph)
        L.set_params(prm)
        L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
        L.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(L.stream)
        L.step(steps)
        e1.record(L.stream)
        torch.cuda.synchronize()
        out[name + "_us_per_step"] = e0.elapsed_time(e1) / steps * 1e3
        states[name] = L.save_state()
        L.close()
    out["bit_identical"] = states["graph_replay"] == states["many_steps"]
    out["steps"] = steps
    return out


def run_c4_steady(system="sat_water_25C", prec="fp32", decay_times=6.5, chunk=2_000_000):
    """C4's layered Poiseuille flow at the paper's finest grid (dx = 1.25 um,
    dt = 12.5 ns, W = 20 dx = 25 um, 512 nodes across: H = 0.64 mm) run from
    rest to steady state with the many-steps kernel: decay_times times the
    liquid layer's slowest decay time 4 h^2 / (pi^2 nu_l).  Reports the E2 of
    the final profile against the steady momentum balance of Eq.
    NSE_for_layered_poiseuille integrated with the simulated phi (diffuse
    interface) and with a sharp interface at the initial height, and the
    relative change over the last chunk of steps."""
    import math
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from layered_ref import diffuse_profile, sharp_profile
    props = {k: v for k, v in WL.TWO_PHASE_SYSTEMS[system].items()
             if k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma")}
    ny = 512
    prm, ini, offs = WL.layered(nx=4, ny=ny, seed=0, dx=1.25e-6, dt=1.25e-8, W_nodes=20.0, **props)
    L = lbm.Lattice("phase", 4, ny, prec=prec, bc=(0, 0, lbm.BC_WALL, lbm.BC_WALL))
    L.set_step_fusion(3)
    L.set_params(prm)
    L.init(ini["p"], ini["ux"], ini["uy"], None, ini["phi"])
    H = ny * prm["dx"]
    h = 0.5 * H
    steps = int(math.ceil(decay_times * 4 * h * h / (math.pi ** 2 * prm["nu_l"]) / prm["dt"]))
    done, prev = 0, None
    t0 = time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        if done + n >= steps:
            prev = L.macros(("ux",))["ux"][0, :, 0]
        L.step(n)
        done += n
        log("bench: c4 steady %s: %d / %d steps" % (system, done, steps))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if L.reduce(("nonfinite",))["nonfinite"].sum() != 0:
        raise RuntimeError("non-finite populations")
    m = L.macros(("ux", "phi"))
    L.close()
    u, phi = m["ux"][0, :, 0], m["phi"][0, :, 0]
    y = (np.arange(ny) + 0.5) * prm["dx"]

    def e2(ref, num):
        return float(100.0 * np.sqrt(np.sum((ref - num) ** 2) / np.sum(ref ** 2)))

    return dict(system=system, prec=prec, steps=steps, us_per_step=wall / steps * 1e6,
                E2_vs_diffuse_percent=e2(diffuse_profile(y, phi, prm, H), u),
                E2_vs_sharp_percent=e2(sharp_profile(y, offs[0], prm, H), u),
                last_chunk_rel_change=float(np.abs(u - prev).max() / np.abs(u).max()),
                u_max=float(np.abs(u).max()))


def adjoint_cost(steps=20000, ckpt=500, prec="fp32"):
    """Adjoint/forward cost on the C5 heated channel (1600 x 80 nodes, flow from
    rest): plain forward time, record time (forward + checkpoints) and the
    reverse time of lbm_grad (recompute of every segment + adjoint steps)."""
    import torch
    from paper_2302_04120_amd import lbm, workloads as WL
    prm, ini = WL.adjoint_channel()
    nx, ny = 1600, 80
    L = lbm.Lattice("channel", nx, ny, prec=prec,
                    bc=(lbm.BC_VEL_INLET, lbm.BC_P_OUTLET, lbm.BC_WALL, lbm.BC_WALL),
                    flow=True, thermal=True)
    L.set_params(prm)
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    L.step(200)
    torch.cuda.synchronize()
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    t0 = time.perf_counter()
    L.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    L.init(ini["rho"], ini["ux"], ini["uy"], ini["T"])
    t0 = time.perf_counter()
    L.record(steps, ckpt, nx // 2)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.grad()
    t_grad = time.perf_counter() - t0
    L.close()
    return dict(forward_s=t_fwd, record_s=t_rec, grad_s=t_grad,
                adjoint_over_forward=t_grad / t_fwd,
                record_plus_grad_over_forward=(t_rec + t_grad) / t_fwd,
                forward_mlups=nx * ny * steps / t_fwd / 1e6)


def host_cpu():
    """Logical CPUs visible to this process and the CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(seconds=8.0):
    """The FP64 oracle on one 256 x 256 replica of the same workload: on one
    thread, and the same source with its OpenMP row loops on every host core
    (identical state after the same steps, checked)."""
    import oracle as O
    from paper_2302_04120_amd import workloads as WL
    prm, ini, _ = WL.bubble(n=256, batch=1, seed=0)
    host = host_cpu()

    def timed_oracle(threads):
        ph = O.Phase(256, 256, prm, threads=threads)
        ph.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds:
            ph.step(10)
            steps += 10
        return ph, steps, time.perf_counter() - t0

    ph1, s1, t1 = timed_oracle(0)
    phn, sn, tn = timed_oracle(host["nproc"])
    # same source, same order of operations per node: the states after the
    # same number of steps are identical
    ref = O.Phase(256, 256, prm)
    ref.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
    ref.step(sn)
    identical = all(np.array_equal(a, b) for a, b in zip(ref.get_state(), phn.get_state()))
    single = dict(value=256 * 256 * s1 / t1 / 1e6, unit="MLUPS", cores=1, steps=s1)
    base = dict(value=256 * 256 * sn / tn / 1e6, unit="MLUPS", cores=phn.threads, kind="oracle",
                sample="one 256x256 replica of the bubble workload, %d steps, FP64, the oracle's "
                       "OpenMP build on %d threads (rows split per node loop)" % (sn, phn.threads),
                single_thread=single, identical_to_single_thread=bool(identical), host=host)
    return base, parity_vs_oracle(prm, ini, ph1.macros(), s1)


def parity_vs_oracle(prm, ini, mo_long, steps_long, steps_short=20):
    """The GPU path on the oracle's sample (replica 0 of the bench workload;
    FP32 deviation storage with the bench's two-step kernel, and FP64).
    Pointwise after a short horizon: max |GPU - oracle| per field relative to
    the field's scale (1 for phi; max |p| or sigma / W for p; max |u| for u).
    After the CPU sample's long horizon, where the model amplifies rounding
    differences (the interface normal flips where grad phi passes through
    zero), the observables: the bubble's pressure jump and the phi sum."""
    import numpy as np
    import oracle as O
    from paper_2302_04120_amd import lbm
    o = O.Phase(256, 256, prm)
    o.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
    o.step(steps_short)
    mo = o.macros()
    scale_p = max(float(np.abs(mo["p"]).max()), prm["sigma"] / prm["W"])
    scale_u = max(float(np.abs(mo["ux"]).max()), float(np.abs(mo["uy"]).max()), 1e-300)
    scales = {"phi": 1.0, "p": scale_p, "ux": scale_u, "uy": scale_u}
    gas, liq = mo_long["phi"] < 0.01, mo_long["phi"] > 0.99
    jump = lambda m: float(m["p"][gas].mean() - m["p"][liq].mean())
    out = {"pointwise_steps": steps_short, "long_steps": steps_long, "replica": 0,
           "oracle_dP_Pa": jump(mo_long)}
    for prec, fusion in (("fp32", 2), ("fp64", 1)):
        L = lbm.Lattice("phase", 256, 256, batch=1, prec=prec)
        L.set_step_fusion(fusion)
        L.set_params(prm)
        L.init(ini["p"][:1], ini["ux"][:1], ini["uy"][:1], None, ini["phi"][:1])
        L.step(steps_short)
        g = L.macros(tuple(scales))
        r = {"pointwise": {k: float(np.abs(g[k][0] - mo[k]).max() / sc) for k, sc in scales.items()}}
        # the velocity against the storage's resolution of the gas momentum:
        # one rounding unit of the stored pressure populations (p / c_s^2)
        # stands for eps c max(|p|, sigma / W) / c_s^2 / rho_g of velocity
        c = prm["dx"] / prm["dt"]
        eps = 2.0 ** -23 if prec == "fp32" else 2.0 ** -52
        u_res = eps * c * scale_p / (c * c / 3.0) / prm["rho_g"]
        du = max(float(np.abs(g[k][0] - mo[k]).max()) for k in ("ux", "uy"))
        r["u_abs_err_mps"] = du
        r["u_resolution_mps"] = u_res
        r["u_err_in_resolution_units"] = du / u_res
        L.step(steps_long - steps_short)
        g = {k: v[0] for k, v in L.macros(("p", "phi")).items()}
        r["dP_rel"] = abs(jump(g) / jump(mo_long) - 1.0)
        r["phi_sum_rel"] = abs(float(g["phi"].sum()) / float(mo_long["phi"].sum()) - 1.0)
        L.close()
        out[prec] = r
    return out


def copy_calibration(nbytes, reps=5):
    """A plain device copy of known size (torch's own copy kernel), used to
    scale rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                      "reps": reps}), flush=True)


def copy_ceiling(nbytes=4 << 30, reps=7):
    """What this GPU's HBM delivers to simple kernels (GB/s): the practical
    ceiling of a kernel that reads and writes its state once."""
    import ctypes
    lib_path = os.path.join(ROOT, "paper_2302_04120_amd", "libhbm_probe.so")
    if not os.path.exists(lib_path):
        raise RuntimeError("libhbm_probe.so not built: run __graft_entry__.build()")
    L = ctypes.CDLL(lib_path)
    L.hbm_probe_run.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.hbm_probe_name.restype = ctypes.c_char_p
    n = L.hbm_probe_count()
    out = (ctypes.c_double * n)()
    rc = L.hbm_probe_run(nbytes, reps, out)
    if rc != 0:
        raise RuntimeError("hbm_probe_run failed: HIP error %d" % rc)
    res = {L.hbm_probe_name(i).decode(): out[i] for i in range(n)}
    best = {kind: max((k for k in res if k.startswith(kind)), key=res.get)
            for kind in ("copy", "read", "write", "planes")}
    res["best"] = {kind: {"probe": k, "GBps": res[k], "frac_of_peak": res[k] / HBM_PEAK_GBS}
                   for kind, k in best.items()}
    res["best_copy_frac_of_peak"] = max(res[best["copy"]], res[best["planes"]]) / HBM_PEAK_GBS
    res["buffer_bytes"] = nbytes
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 200; 20000 for --leg c4single)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 20; 200 for --leg c4single)")
    ap.add_argument("--batch", type=int, default=1024, help="256x256 replicas per step")
    ap.add_argument("--prec", default="fp32", choices=("fp32", "fp64", "fp32_arith64"))
    ap.add_argument("--fusion", type=int, default=2, choices=(0, 1, 2),
                    help="2 two-step kernel (default), 1 single-step, 0 library's choice (the "
                         "two-phase workloads and --leg channel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and batch-4 legs")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_phase_step.json"))
    ap.add_argument("--leg", choices=("channel", "adjoint", "d3q19", "phase3d", "layered", "c4single",
                                      "c4steady", "wide"),
                    default=None,
                    help="only run one secondary leg and print its figures (for profiling)")
    ap.add_argument("--systems", default="sat_water_25C,air_water_25C",
                    help="two-phase systems of the c4steady leg (comma-separated)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy of BYTES (counter calibration)")
    ap.add_argument("--copy-ceiling", action="store_true",
                    help="only run the HBM bandwidth probe (copies and one-way streams, 4 GiB)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 20000 if args.leg == "c4single" else 200
    if args.warmup is None:
        args.warmup = 200 if args.leg == "c4single" else 20
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return 0
    if args.copy_ceiling:
        print(json.dumps(copy_ceiling()), flush=True)
        return 0
    if args.prec == "fp32_arith64" and (args.leg not in (None, "layered", "c4single", "c4steady")
                                        or (args.leg is None and args.fusion == 2)):
        print("--prec fp32_arith64 applies to the two-phase legs (with --fusion 0 or 1 for the "
              "bubble workload)", file=sys.stderr)
        return 2
    if args.leg == "channel":
        print(json.dumps(run_channel(16384, 2048, args.steps, args.warmup, args.prec,
                                     args.fusion)), flush=True)
        return 0
    if args.leg == "wide":
        print(json.dumps(run_wide(32, args.steps, args.warmup, args.prec, args.fusion)), flush=True)
        return 0
    if args.leg == "adjoint":
        print(json.dumps(adjoint_cost(prec=args.prec)), flush=True)
        return 0
    if args.leg == "d3q19":
        print(json.dumps(run_d3(256, args.steps, args.warmup, args.prec)), flush=True)
        return 0
    if args.leg == "phase3d":
        print(json.dumps(run_p3(256, args.steps, args.warmup, args.prec)), flush=True)
        return 0
    if args.leg == "layered":
        print(json.dumps(run_layered_batch(4096, args.steps, args.warmup, args.prec)), flush=True)
        return 0
    if args.leg == "c4single":
        print(json.dumps(run_c4_single(args.steps, args.warmup, args.prec)), flush=True)
        return 0
    if args.leg == "c4steady":
        for system in args.systems.split(","):
            print(json.dumps(run_c4_steady(system, args.prec)), flush=True)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        return 2
    if args.steps % 2 and args.fusion == 2:
        print("--steps must be even with the two-step kernel", file=sys.stderr)
        return 2
    log("bench: phase workload batch=%d steps=%d warmup=%d prec=%s fusion=%d" %
        (args.batch, args.steps, args.warmup, args.prec, args.fusion))
    r = run_gpu(args.batch, args.steps, args.warmup, args.prec, fusion=args.fusion,
                windows=0 if args.no_extras else 5)
    mlups = r["nodes"] * args.steps / r["wall"] / 1e6
    bpl = BYTES_PER_LU[args.prec]
    spl = 2 if args.fusion == 2 else 1  # steps per launch
    kname = ("k_phase_tb2<%s, false, true>" % ("float" if args.prec == "fp32" else "double")
             if spl == 2 else
             "k_phase<%s>" % {"fp32": "float,float,false", "fp64": "double,double,false",
                              "fp32_arith64": "float,double,false"}[args.prec])
    launch_ms = r["kernel_ms"] * spl
    # Bytes one launch must move: the stored state (21 FP32 values per node: h,
    # the low part of h_0, z and (phi u)) read once and written once, whatever
    # the number of steps the launch performs -- bpl x nodes.  The two-step
    # kernel keeps the intermediate state on chip, so per lattice update it
    # needs bpl / 2; the step-equivalent rate (bpl per update) is reported
    # beside it and is not a fraction of any peak.
    launch_bytes = bpl * r["nodes"]
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    step_equivalent = bpl * r["nodes"] * spl / (launch_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic):
        with open(args.traffic) as f:
            tr = json.load(f)
        if (tr.get("batch") == args.batch and tr.get("prec") == args.prec
                and tr.get("kernel") == kname
                and tr.get("source_sha256") == kernel_source_hash()):
            traffic = tr.get("bytes_per_launch")
    extras = {}
    if not args.no_extras:
        log("bench: FP64 leg")
        s64 = max(20, args.steps // 4) // 2 * 2
        r64 = run_gpu(max(1, args.batch // 4), s64, 6, "fp64", fusion=args.fusion)
        extras["fp64_mlups"] = r64["nodes"] * s64 / r64["wall"] / 1e6
        # the state (20 FP64 values per node) once in and once out per launch of spl steps
        l64 = r64["kernel_ms"] * spl * 1e-3
        extras["fp64_hbm_frac"] = BYTES_PER_LU["fp64"] * r64["nodes"] / l64 / 1e9 / HBM_PEAK_GBS
        extras["fp64_step_equivalent_GBps"] = BYTES_PER_LU["fp64"] * r64["nodes"] * spl / l64 / 1e9
        log("bench: single-step kernel on the same workload")
        r1 = run_gpu(args.batch, 100, 6, "fp32", fusion=1)
        extras["single_step_fp32"] = dict(
            mlups=r1["nodes"] * 100 / (r1["ev_ms"] * 1e-3) / 1e6, kernel_ms=r1["kernel_ms"],
            hbm_GBps=BYTES_PER_LU["fp32"] * r1["nodes"] / (r1["kernel_ms"] * 1e-3) / 1e9,
            hbm_frac=BYTES_PER_LU["fp32"] * r1["nodes"] / (r1["kernel_ms"] * 1e-3) / 1e9
            / HBM_PEAK_GBS,
            kernel="k_phase<float, float, false, 64, 4>")
        log("bench: paper-sized leg (4 replicas)")
        # launch-bound: graph replay; 128 warm-up steps (twice the graph length)
        # capture the graph before the timed steps
        r4 = run_gpu(4, 1000, 128, args.prec)
        extras["paper_config_batch4_mlups"] = r4["nodes"] * 1000 / r4["wall"] / 1e6
        log("bench: single wide domain leg (8192^2 bubble array)")
        extras["wide_domain_fp32"] = run_wide(32, 100, 10, "fp32")
        log("bench: C4 layered batch leg (4096 x 4 x 512)")
        extras["layered_batch_fp32"] = run_layered_batch(4096, 200, 20, "fp32")
        log("bench: C4 single replica, graph replay and many-steps kernel")
        extras["c4_single_replica"] = run_c4_single()
        log("bench: heated-channel leg (16384 x 2048)")
        extras["channel_fp32"] = run_channel(16384, 2048, 100, 10, "fp32", fusion=2)
        extras["channel_single_step_fp32"] = run_channel(16384, 2048, 100, 10, "fp32", fusion=1)
        extras["channel_fp64"] = run_channel(16384, 2048, 40, 4, "fp64", fusion=2)
        log("bench: D3Q19 leg (256^3)")
        extras["d3q19_fp32"] = run_d3(256, 100, 10, "fp32")
        extras["d3q19_fp64"] = run_d3(256, 40, 4, "fp64")
        log("bench: 3D two-phase leg (256^3)")
        extras["phase3d_fp32"] = run_p3(256, 40, 4, "fp32")
        log("bench: adjoint/forward cost leg (C5 channel)")
        extras["adjoint"] = adjoint_cost()
    cpu = parity = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline and parity of the GPU path on its sample")
        cpu, parity = cpu_baseline()
    line = {
        "metric": "MLUPS (D2Q9 MRT + Allen-Cahn) FP32-dev vs FP64, % HBM roofline; adjoint/fwd cost",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "f64",  # the step's arithmetic type
        "data": "synthetic",
        "config": {"workload": "stationary bubble, D2Q9 MRT z + D2Q9 Allen-Cahn h, 256x256 "
                               "periodic cell, rho_l/rho_g=43290, nu_g/nu_l=471, radii 20/30/40/50 "
                               "nodes, %d replicas per step" % args.batch,
                   "nodes_per_step": r["nodes"],
                   "storage": "fp64-deviation" if args.prec == "fp64" else "fp32-deviation"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_node_per_launch": bpl, "nodes_per_launch": r["nodes"],
                     "launch_bytes": launch_bytes, "kernel": kname, "steps_per_launch": spl,
                     "launch_ms": launch_ms,
                     "lu_per_launch": r["nodes"] * spl,
                     "bytes_per_lu_single_step": bpl,
                     "step_equivalent_GBps": step_equivalent,
                     "hbm_measured_GBps": (traffic / (launch_ms * 1e-3) / 1e9
                                           if traffic is not None else None),
                     "hbm_measured_frac": (traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                           if traffic is not None else None)},
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "phi_sum_drift": r["phi_sum_drift"],
        "phi_sum_steps": r["phi_sum_steps"],
        "sustained": r.get("sustained"),
        "adjoint_over_forward": None,
    }
    line.update(extras)
    if "adjoint" in extras:
        line["adjoint_over_forward"] = extras["adjoint"]["adjoint_over_forward"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
