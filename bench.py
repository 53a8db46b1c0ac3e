"""Benchmark: LLG cell-updates/s of the fused HIP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload block|block_large|block_dmi|film|film_basis|film_large|film_large_basis|cube]

A step is one accepted Dormand-Prince 5(4) step (6 new right-hand sides with
first-same-as-last) of the whole hot path: demag FFT convolution, local terms,
LLG right-hand side, stage combination, float64 error norm and the device-side
step controller.  Inputs are seeded synthetic problems resident in HBM before
the timed region.  The metric follows the paper's benchmark (Sec. 6): cells x
right-hand-side evaluations / wall time.

Printed JSON line extras:
  roofline      the dominant kernel's algorithmic bytes per launch divided by
                its average launch time, against the 8 TB/s HBM peak; launch
                times come from timing-only HIP events on the mesh stream
                around every kernel of a second region of the same number of
                steps (the headline region replays captured graphs, which
                cannot hold per-kernel events);
  kernels       the same for every kernel slot;
  cpu_baseline  the float64 oracle on the host, timed on a bounded sample of
                the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # the block relaxation: 128 x 128 x 32 cells of 2 nm, alpha = 1, random Ku
    # and easy axes, DP45 rtol 1e-5
    "block": dict(tag="block_128x128x32", desc="3D block 128x128x32 cells (2 nm), alpha=1 relaxation, per-cell Ku, DP45 rtol 1e-5",
                  make="block", terms=("exchange", "demag", "anisotropy"), dt0=1e-14),
    # the same recipe at 256 x 256 x 64: the demag working set (~320 MB) no
    # longer fits the 256 MB Infinity Cache
    "block_large": dict(tag="block_256x256x64", desc="3D block 256x256x64 cells (2 nm), alpha=1 relaxation, per-cell Ku, DP45 rtol 1e-5",
                        make="block_large", terms=("exchange", "demag", "anisotropy"), dt0=1e-14),
    # the block with interfacial DMI (D = 3 mJ/m^2 in every cell): the node
    # kernel's DMI instantiation on the same mesh
    "block_dmi": dict(tag="block_128x128x32_dmi",
                      desc="3D block 128x128x32 cells (2 nm), alpha=1 relaxation, per-cell Ku, interfacial DMI "
                           "D=3 mJ/m^2, DP45 rtol 1e-5",
                      make="block_dmi", terms=("exchange", "demag", "anisotropy", "dmi"), dt0=1e-14),
    # the same film under the thin-film basis (one node layer, Sec. 3.3)
    "film_basis": dict(tag="film_256x64x1_filmbasis",
                       desc="thin film 256x64x1 cells (3.9x3.9x3 nm), thin-film basis (one node layer), "
                            "field step (-25,4,0) mT, DP45 rtol 1e-5",
                       make="film_basis", terms=("exchange", "demag", "zeeman"), dt0=1e-13),
    # a 512 x 512 x 1 film (the largest single-layer grid of 1024-point
    # transforms) under both bases
    "film_large": dict(tag="film_512x512x1",
                       desc="thin film 512x512x1 cells (3.9x3.9x3 nm), 3D basis, field step (-25,4,0) mT, "
                            "DP45 rtol 1e-5",
                       make="film_large", terms=("exchange", "demag", "zeeman"), dt0=1e-13),
    "film_large_basis": dict(tag="film_512x512x1_filmbasis",
                             desc="thin film 512x512x1 cells (3.9x3.9x3 nm), thin-film basis (one node layer), "
                                  "field step (-25,4,0) mT, DP45 rtol 1e-5",
                             make="film_large_basis", terms=("exchange", "demag", "zeeman"), dt0=1e-13),
    "film": dict(tag="film_256x64x1", desc="thin film 256x64x1 cells (3.9x3.9x3 nm), field step (-25,4,0) mT, DP45 rtol 1e-5",
                 make="film", terms=("exchange", "demag", "zeeman"), dt0=1e-13),
    "cube": dict(tag="cube_16x16x4", desc="16x16x4 cells (2 nm), random start, DP45 rtol 1e-5",
                 make="standard_cube", terms=("exchange", "demag"), dt0=1e-14),
}


# DP45 node-kernel launches per accepted step run stages 2..7 (the first
# stage of a step is the last of the one before): stage s writes k_s and,
# below 7, y_{s+1}, and reads the earlier k_j with non-zero weights
# (1, 2, 3, 4, 4, 5 of them)
DP45_WRITES = 11.0 / 6.0
DP45_READS = 19.0 / 6.0


# the oracle's term bits (its own numbering)
ORACLE_TERMS = {"exchange": 1, "demag": 2, "anisotropy": 4, "zeeman": 8, "dmi": 16}


def make_workload(synth, W):
    if W["make"] == "block_large":
        return synth.block(n=(256, 256, 64))
    if W["make"] == "block_dmi":
        return synth.block(D=3e-3)
    if W["make"] == "film_basis":
        return synth.as_film(synth.film())
    if W["make"] == "film_large":
        return synth.film(n=(512, 512, 1))
    if W["make"] == "film_large_basis":
        return synth.as_film(synth.film(n=(512, 512, 1)))
    return getattr(synth, W["make"])()


def byte_model(n, pad, nn, zeeman, stage_writes=DP45_WRITES, stage_reads=DP45_READS, dmi=False):
    """Algorithmic bytes per launch of each kernel slot (inputs + outputs once).
    zeeman: the static applied field is part of the cell-field source; dmi:
    the node kernel also reads D per cell."""
    n1, n2, n3 = n
    p1, p2, p3 = pad
    k1 = p1 // 2 + 1
    nc = n1 * n2 * n3
    c8 = 8  # complex64
    out = {}
    out["xfwd"] = 12 * nn + 4 * nc + 3 * n3 * n2 * k1 * c8
    if n3 > 1:
        out["yfwd"] = 3 * n3 * n2 * k1 * c8 + 3 * n3 * p2 * k1 * c8
        tensor = 6 * (p3 // 2 + 1) * (p2 // 2 + 1) * k1 * 4
        out["conv"] = 2 * 3 * n3 * p2 * k1 * c8 + tensor
        out["yinv"] = 3 * n3 * p2 * k1 * c8 + 3 * n3 * n2 * k1 * c8
    else:
        tensor = 4 * (p2 // 2 + 1) * k1 * 4
        out["conv"] = 2 * 3 * n2 * k1 * c8 + tensor
    # spectrum rows in, cell weight in, one float4 source per cell out (plus
    # the static Zeeman float4 in when the field has one)
    out["xinv"] = 3 * n3 * n2 * k1 * c8 + 4 * nc + 16 * nc + (16 * nc if zeeman else 0)
    # per cell: packed {2A, u} and the float4 source; per node: stage input,
    # state, coefficients (1/M, gamma', alpha), the stage outputs written,
    # earlier k_j read
    cell = 16 * nc + 16 * nc + (4 * nc if dmi else 0)
    out["stencil"] = cell + 12 * nn * (1 + 1 + 1 + stage_writes + stage_reads)
    return out


def counter_traffic(kernel, tag):
    """HBM bytes per launch of one kernel on one workload from a committed
    rocprofv3 counter summary, if the kernel source has not changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters_%s_%s.md" % (kernel, tag))
    src = os.path.join(ROOT, "paper_2411_11725_amd", "csrc", "demag.hip" if kernel != "stencil" else "stencil.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    b = re.search(r"hbm bytes per launch: ([0-9.eE+]+)", text)
    if not m or not b:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(1):
        return None
    return float(b.group(1))


def _oracle_problem(p):
    import numpy as np

    import oracle

    mesh = oracle.Mesh(p["n"], p["h"], basis=p.get("basis", "3d"))
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    mat = oracle.Material(Ms=f(p["Ms"]), A=f(p["A"]), alpha=f(p["alpha"]), gamma=p["gamma"],
                          Ku=f(p["Ku"]), easy=f(p["easy"]), h_cell=f(p["h_cell"]),
                          h_uniform=f(p["h_uniform"]), drive_mask=f(p["drive_mask"]),
                          drive_amp=f(p["drive_amp"]), drive_freq=p["drive_freq"],
                          drive_phase=p["drive_phase"], D=f(p.get("D")))
    return mesh, mat, f(p["m0"])


def _oracle_worker(args):
    """One host process: tensor set-up (untimed), a barrier, then `evals`
    oracle right-hand sides; returns (start, end) wall-clock times."""
    p, terms_mask, evals, barrier = args
    import oracle
    from oracle.field import demag_cell_field

    mesh, mat, m = _oracle_problem(p)
    demag_cell_field(mesh, mat, m)
    barrier.wait()
    t0 = time.time()
    for _ in range(evals):
        oracle.llg_rhs(mesh, mat, m, 0.0, terms_mask)
    return t0, time.time()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, terms_mask, evals=14, par_evals=3, max_cores=16):
    """The float64 oracle's right-hand sides of the same workload on the host:
    one process (numpy, one thread), then one process per available core
    (at most max_cores, the host share of one GPU) evaluating concurrently;
    the tensor set-up is excluded from both."""
    import multiprocessing as mp

    import oracle
    from oracle.field import demag_cell_field

    os.environ["OMP_NUM_THREADS"] = "1"
    mesh, mat, m = _oracle_problem(p)
    t0 = time.perf_counter()
    demag_cell_field(mesh, mat, m)            # tensor and its spectrum: set-up, not timed
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(evals):
        oracle.llg_rhs(mesh, mat, m, 0.0, terms_mask)
    dt = time.perf_counter() - t0
    one = mesh.n_cells * evals / dt
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("fork")
    with ctx.Manager() as man:
        barrier = man.Barrier(cores)
        with ctx.Pool(cores) as pool:
            spans = pool.map(_oracle_worker, [(p, terms_mask, par_evals, barrier)] * cores, chunksize=1)
    wall = max(b for _, b in spans) - min(a for a, _ in spans)
    allc = mesh.n_cells * par_evals * cores / wall
    return {"value": allc, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": "%d concurrent host processes (one numpy thread each), %d float64 right-hand sides "
                      "of the full %dx%dx%d mesh each; tensor set-up excluded" % (cores, par_evals, *p["n"]),
            "one_core": {"value": one, "unit": "cell-updates/s", "cores": 1,
                         "sample": "%d float64 right-hand sides of the full mesh in one process "
                                   "(%.1f s tensor set-up excluded)" % (evals, setup)}}


def serving_bench(B, synth, count, t_end, nmax, max_active, n_streams=4, attempts=8):
    """Continuous-batching server against a plain one-at-a-time loop on the
    same Poisson request stream (arrival times honoured by both): solves/s and
    p50 / p99 latency (completion minus arrival), and the largest difference
    between the two sets of final states."""
    import numpy as np
    import torch

    reqs = synth.serving_requests(count, nmax=nmax)
    nns = [(q["n"][0] + 1) * (q["n"][1] + 1) * (q["n"][2] + 1) for _, q in reqs]
    # batched: each request is submitted when it arrives, results polled after
    srv = B.nm_server_create(max_active=max_active, n_streams=n_streams, attempts_per_launch=attempts)
    outs_b, lat_b = [], []
    try:
        t0 = B.nm_server_clock()
        tickets = []
        for (ta, q) in reqs:
            while B.nm_server_clock() - t0 < ta:
                time.sleep(2e-4)
            tickets.append(B.nm_serve_submit(srv, q, t_end=t_end))
        t_last = t0
        for i, (tk, nn) in enumerate(zip(tickets, nns)):
            m = np.empty(3 * nn, dtype=np.float32)
            r = B.nm_serve_poll(srv, tk, timeout_ms=600000, m_out=m)
            if r is None or r.status != B.NM_OK:
                raise RuntimeError("served solve failed: %s" % (None if r is None else r.status))
            outs_b.append(m)
            lat_b.append(r.t_done - r.t_submit)
            t_last = max(t_last, r.t_done)
            if (i + 1) % 64 == 0:
                print("serving: batched %d/%d polled" % (i + 1, count), file=sys.stderr, flush=True)
        wall_b = t_last - t0
        print("serving: batched %d solves in %.2f s" % (count, wall_b), file=sys.stderr, flush=True)
    finally:
        B.nm_server_destroy(srv)
    # plain loop: one mesh at a time, created, stepped to t_end and read back
    lat_p, diff = [], 0.0
    t0 = time.perf_counter()
    for (ta, q), mb in zip(reqs, outs_b):
        while time.perf_counter() - t0 < ta:
            time.sleep(2e-4)
        mesh = B.mesh_from_problem(q, device="cuda:0")
        m = torch.as_tensor(q["m0"], device="cuda:0").contiguous()
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=t_end)
        mp = m.cpu().numpy().ravel()
        B.nm_mesh_destroy(mesh)
        lat_p.append(time.perf_counter() - t0 - ta)
        diff = max(diff, float(np.abs(mp - mb).max()))
        if len(lat_p) % 64 == 0:
            print("serving: plain loop %d/%d done" % (len(lat_p), count), file=sys.stderr, flush=True)
    wall_p = time.perf_counter() - t0
    print("serving: plain loop %d solves in %.2f s" % (count, wall_p), file=sys.stderr, flush=True)
    pct = lambda a, q: float(np.percentile(np.asarray(a), q))
    cells = [q["n"][0] * q["n"][1] * q["n"][2] for _, q in reqs]
    return {
        "stream": "%d solves, Poisson arrivals at 200/s, nx, ny log-uniform in [32, %d], nz in 1..8, "
                  "3 nm cells, DP45 rtol 1e-5 to t = %.2g s" % (count, nmax, t_end),
        "cells_mean": float(np.mean(cells)), "max_active": max_active, "streams": n_streams,
        "attempts_per_launch": attempts,
        "batched": {"solves_per_s": count / wall_b, "p50_s": pct(lat_b, 50), "p99_s": pct(lat_b, 99),
                    "wall_s": wall_b},
        "plain_loop": {"solves_per_s": count / wall_p, "p50_s": pct(lat_p, 50), "p99_s": pct(lat_p, 99),
                       "wall_s": wall_p},
        "speedup": wall_p / wall_b,
        "max_abs_diff_m": diff,
    }


def adjoint_bench(B, synth, nsteps, ckpt):
    """Inverse-problem workload (the 256x128x1 magnonic strip, RK4 dt 5e-14 s,
    10 GHz drive, loss = -time average of the mean m_z^2 over a 16x16 output
    region): forward trajectory with checkpoints, then the adjoint sweep that
    gives the gradient with respect to the per-cell field map."""
    import torch

    from paper_2411_11725_amd.adjoint import LLGTrajectory, LLGTrajectoryContinuous

    p = synth.magnonic()
    mesh = B.mesh_from_problem(p, device="cuda:0")
    n1, n2, n3 = p["n"]
    try:
        theta = torch.zeros((3, n3, n2, n1), device="cuda:0", requires_grad=True)
        m0 = torch.as_tensor(p["m0"], device="cuda:0").contiguous()
        region = torch.zeros((n3 + 1, n2 + 1, n1 + 1), dtype=torch.bool, device="cuda:0")
        region[:, 56:72, 192:208] = True
        # warm-up: records the stepping and adjoint-segment graphs
        w = LLGTrajectory.apply(theta, m0, mesh, 5e-14, ckpt, ckpt, 1, B.NM_T_ALL)
        (-(w[:, 2][:, region] ** 2).mean()).backward()
        theta.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        traj = LLGTrajectory.apply(theta, m0, mesh, 5e-14, nsteps, ckpt, 1, B.NM_T_ALL)
        loss = -(traj[:, 2][:, region] ** 2).mean()
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        gnorm = float(theta.grad.norm())
        # the continuous adjoint rebuilds m by integrating backwards, which
        # amplifies the damped modes (alpha up to 0.5 at the absorbing edges)
        # by exp(alpha gamma' H t): over the full trajectory it overflows, so
        # it is timed and compared on the first cont_steps steps only
        cont_steps = min(nsteps, 400)
        theta.grad = None
        traj = LLGTrajectory.apply(theta, m0, mesh, 5e-14, cont_steps, ckpt, 1, B.NM_T_ALL)
        (-(traj[:, 2][:, region] ** 2).mean()).backward()
        g_disc = theta.grad.clone()
        theta.grad = None
        w = LLGTrajectoryContinuous.apply(theta, m0, mesh, 5e-14, ckpt, 1, B.NM_T_ALL)
        (-(w[:, 2][:, region] ** 2).mean()).backward()
        theta.grad = None
        torch.cuda.synchronize()
        traj = LLGTrajectoryContinuous.apply(theta, m0, mesh, 5e-14, cont_steps, 1, B.NM_T_ALL)
        loss = -(traj[:, 2][:, region] ** 2).mean()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t_cont = time.perf_counter() - t0
        gap = float((theta.grad - g_disc).norm() / g_disc.norm())
    finally:
        B.nm_mesh_destroy(mesh)
    cells = n1 * n2 * n3
    return {"workload": "magnonic strip %dx%dx%d cells, RK4 dt 5e-14 s, %d steps, checkpoint every %d, "
                        "gradient w.r.t. the per-cell field map" % (n1, n2, n3, nsteps, ckpt),
            "forward_steps_per_s": nsteps / t_fwd, "backward_steps_per_s": nsteps / t_bwd,
            "backward_over_forward": t_bwd / t_fwd,
            "forward_cell_updates_per_s": 4 * cells * nsteps / t_fwd, "grad_norm": gnorm,
            "continuous_steps": cont_steps,
            "continuous_backward_steps_per_s": cont_steps / t_cont,
            "continuous_vs_discrete_gradient_rel_diff": gap}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="block", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-count", type=int, default=48,
                    help="solves in the serving stream (0: skip the serving measurement)")
    ap.add_argument("--serve-nmax", type=int, default=256)
    ap.add_argument("--serve-tend", type=float, default=0.2e-9)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-attempts", type=int, default=8)
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=4000,
                    help="RK4 steps of the adjoint measurement (0: skip it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 plain device copies of 256 MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        n = 64 * 1024 * 1024
        a = torch.ones(n, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the hot path runs on a single GPU "
              "(multi-GPU sharding is design only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2411_11725_amd import synth

    W = WORKLOADS[args.workload]
    p = make_workload(synth, W)
    # the host baseline runs first, before this process touches the GPU (its
    # worker processes are forked)
    cpu = None
    if not args.no_cpu_baseline and not args.serve_only:
        cpu = cpu_baseline(p, sum(ORACLE_TERMS[t] for t in W["terms"]))
        print("cpu baseline: done", file=sys.stderr, flush=True)

    import torch

    from paper_2411_11725_amd import binding as B

    if args.serve_only:
        torch.cuda.set_device(0)
        print(json.dumps({"serving": serving_bench(B, synth, args.serve_count, args.serve_tend, args.serve_nmax,
                                                   args.serve_active, args.serve_streams, args.serve_attempts)}))
        return
    # the serving stream runs first, in a fresh process state
    serving = None
    if args.serve_count > 0:
        torch.cuda.set_device(0)
        serving = serving_bench(B, synth, args.serve_count, args.serve_tend, args.serve_nmax,
                                args.serve_active, args.serve_streams, args.serve_attempts)
    tmask = {"exchange": B.NM_T_EXCHANGE, "demag": B.NM_T_DEMAG, "anisotropy": B.NM_T_ANIS,
             "zeeman": B.NM_T_ZEEMAN, "dmi": B.NM_T_DMI}
    terms = sum(tmask[t] for t in W["terms"])
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mesh = B.mesh_from_problem(p, device="cuda:0", stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nn, nc, pad = B.nm_mesh_info(mesh)
    m = torch.as_tensor(p["m0"], device="cuda:0").contiguous()
    clk = B.nm_clock(0.0, W["dt0"], 0, 0, 0, 0.0)
    t_cap = 20e-9
    B.nm_llg_step(mesh, m, clk, B.NM_DP45, terms, t_end=t_cap, max_steps=args.warmup)
    torch.cuda.synchronize()
    # timed region: the stepping loop replays one captured HIP graph per batch
    rhs0, acc0, rej0 = clk.rhs_evals, clk.accepted, clk.rejected
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.nm_llg_step(mesh, m, clk, B.NM_DP45, terms, t_end=t_cap, max_steps=args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print("timed region: %.3f s" % elapsed, file=sys.stderr, flush=True)
    rhs = clk.rhs_evals - rhs0
    steps = clk.accepted - acc0
    # graph replays of the region: 16 attempts each, then powers of two
    attempts = steps + clk.rejected - rej0
    replays = attempts // 16 + bin(attempts % 16).count("1")
    value = nc * rhs / elapsed
    # per-kernel region: the same number of steps with every kernel bracketed
    # by timing-only HIP events on the mesh stream (direct launches)
    B.nm_profile_enable(mesh, True)
    B.nm_llg_step(mesh, m, clk, B.NM_DP45, terms, t_end=t_cap, max_steps=args.steps)
    prof = B.nm_profile_read(mesh)
    B.nm_profile_enable(mesh, False)

    bm = byte_model(p["n"], pad, nn, "zeeman" in W["terms"], dmi="dmi" in W["terms"])
    kernels = {}
    for slot, (ms, cnt) in prof.items():
        if cnt == 0 or slot not in bm:
            continue
        avg_s = ms / cnt * 1e-3
        kernels[slot] = {"launches": cnt, "avg_us": avg_s * 1e6, "bytes_per_launch": bm[slot],
                         "gbs": bm[slot] / avg_s / 1e9, "frac": bm[slot] / avg_s / 1e9 / HBM_PEAK_GBS}
    dom = max(kernels, key=lambda k: prof[k][0])
    ach = kernels[dom]["gbs"]
    traffic = counter_traffic(dom, W["tag"])
    B.nm_mesh_destroy(mesh)

    out = {
        "metric": "LLG cell-updates/s", "value": value, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": elapsed / max(steps, 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded; float64 tensor set-up and error norm)",
        "config": {"workload": W["desc"], "cells": nc, "nodes": nn, "padded": list(pad),
                   "rhs_evals": rhs, "integrator": "DP45", "terms": list(W["terms"]),
                   "setup_s": setup_s},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic},
        "kernels": kernels,
        "timing": "value: the timed region of K accepted DP45 steps, replayed as captured HIP graphs (about %d "
                  "replays, each followed by a read-back of the device controller); kernels and roofline: a "
                  "second region of the same K steps with direct launches, every kernel bracketed by HIP "
                  "events on the mesh stream" % replays,
    }
    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_bench(B, synth, args.adjoint_steps, 100)
        print("adjoint: done", file=sys.stderr, flush=True)
    if serving is not None:
        out["serving"] = serving
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
