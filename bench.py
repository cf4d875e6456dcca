"""Throughput of the kinetic bounds + limiter hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload tri2m] [--no-cpu-baseline]

One step = kbl_compute_bounds + kbl_limit over the whole workload, inputs
already resident in HBM.  The default workload is the largest one that the
method is exercised on: 2,000,000 P2 triangles with uneven vertex-neighbour
stencils and a 64 x 64 per-stencil velocity grid.  Prints ONE JSON line with
- the FP64 throughput in elements/s (`value`) and the roofline of the
  dominant kernel (the FP64 bounds pass, bound by VALU issue) measured with
  HIP events on the launch stream;
- the same step with each mixed-precision form of the bounds (FP32
  envelopes; FP32 VALU, FP16 MFMA or BF16 MFMA contraction), each against
  its own VALU ceiling, and the MFMA forms' matrix-core rate;
- the FP64 and mixed steps on the 1024^2-quad workload with a global 64 x 64
  grid, and the FP64 backward on the 512^2-quad workload;
- the FP64 CPU oracle timed on a bounded element sample, on all host cores
  and on one core.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs, 2.4 GHz peak engine clock, 64 VALU lanes per CU per clock
# for FP64 (and unpacked FP32) add/min/max.  One lane-op per clock per lane.
N_CU = 256
CLOCK_HZ = 2.4e9
LANES_PER_CU = 64
VALU_PEAK_OPS = N_CU * CLOCK_HZ * LANES_PER_CU          # 3.93e13 lane-ops/s
HBM_PEAK = 8.0e12

METRIC = "element-bounds+limit/s at stated tol, FP64 vs mixed; % VALU/MFMA roofline"

WORKLOAD_TEXT = {
    "quad256": ("2D Euler gamma=1.4, 256x256 periodic quads, p=3 (4x4 Gauss-Legendre nodes), "
                "5-element face stencils (80 states), 48x48 per-stencil velocity grid (k=4), "
                "r_fac=1e-3, 4-quadrant Riemann field rho in [0.1,10], p in [0.1,100], |U|<=3 "
                "+1% smooth perturbation"),
    "quad1024_sine": ("2D Euler gamma=1.4, 1024x1024 periodic quads, p=3, 80-state stencils, "
                      "64x64 global velocity grid on [-12,12]^2 sqrt(theta_max), sine + Sod-jump field"),
    "tri2m": ("2D Euler gamma=1.4, 2,000,000 jittered P2 triangles (6 nodes) on a periodic "
              "1000x1000 lattice, vertex-neighbour stencils (11-16 elements, CSR), 64x64 "
              "per-stencil velocity grid (k=4), r_fac=1e-3, radial shock rho ratio 1e3, "
              "p ratio 1e5 +1% smooth perturbation"),
    "quad512": ("2D Euler gamma=1.4, 512x512 periodic quads, p=3, 80-state stencils, 48x48 "
                "per-stencil velocity grid (k=4), 4-quadrant Riemann field"),
    "line64": ("1D Euler gamma=1.4, 64 elements, p=3, 12-state stencils, 64-node global velocity "
               "grid on [-12,12] sqrt(theta_max), sine + Sod jump"),
    "hex32": ("3D Euler gamma=1.4, 32^3 periodic hexahedra, p=2 (3x3x3 Gauss-Legendre nodes), "
              "7-element face stencils (189 states), 24^3 per-stencil velocity grid (k=4), "
              "r_fac=1e-3, 8-octant Riemann field rho in [0.1,10], p in [0.1,100], |U|<=3 "
              "+1% smooth perturbation"),
}


# sources of the FP64 bounds kernels, per velocity dimension
KERNEL_SOURCES = {
    2: ("paper_2407_20966_amd/csrc/bounds_fp64.hip", "paper_2407_20966_amd/csrc/bounds_common.h",
        "paper_2407_20966_amd/csrc/kbl_internal.h", "paper_2407_20966_amd/csrc/exp2_table.h"),
    3: ("paper_2407_20966_amd/csrc/bounds_fp64_3d.hip",
        "paper_2407_20966_amd/csrc/bounds_common.h", "paper_2407_20966_amd/csrc/kbl_internal.h",
        "paper_2407_20966_amd/csrc/exp2_table.h"),
}
TRAFFIC_FILE = "profiles/bounds_fp64_traffic.txt"


def kernel_sources_sha(dim: int) -> str:
    """sha256 of the FP64 bounds kernel's sources (identifies what was profiled)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[dim]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel: str, grid_threads: int, workload: str, dim: int):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by the copy-kernel calibration) and the grid size the
    counters were taken at, or (None, None) when there is no entry for this
    kernel and workload, or the kernel's sources changed since the counters
    were taken (per-entry sha256).  An entry at this launch's grid size is
    preferred; else one of the same kernel at another grid size (the autotuner
    may pick a persistent grid: the same element work, so the same bytes up to
    L2 reuse)."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path) or dim not in KERNEL_SOURCES:
        return None, None
    entries, cur = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line == "[entry]":
            cur = {}
            entries.append(cur)
            continue
        if "=" in line and cur is not None:
            k, v = line.split("=", 1)
            cur[k.strip()] = v.strip()
    sha = kernel_sources_sha(dim)
    other = (None, None)
    for e in entries:
        try:
            if e["kernel"] == kernel and e["workload"] == workload and e["source_sha256"] == sha:
                g = int(e["grid_threads"])
                if g == grid_threads:
                    return float(e["bytes_per_launch"]), g
                if other[0] is None:
                    other = (float(e["bytes_per_launch"]), g)
        except (KeyError, ValueError):
            continue
    return other


def _counter_per_dispatch(csv_path: str, counter: str):
    """{dispatch id: (kernel name, grid size, value)} of one counter from a
    rocprofv3 counter-collection CSV (rows of one dispatch summed)."""
    import csv
    out = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            k = r["Dispatch_Id"]
            name, grid, v = out.get(k, (r["Kernel_Name"], int(r["Grid_Size"]), 0.0))
            out[k] = (name, grid, v + float(r["Counter_Value"]))
    return dict(sorted(out.items(), key=lambda kv: int(kv[0])))


def write_traffic(workload: str, fetch_csv: str, write_csv: str) -> dict:
    """Turns a FETCH_SIZE run and a WRITE_SIZE run of bench.py (each with
    --copy-calibration) into an entry of the traffic file, replacing an entry
    of the same workload, kernel and grid and the workload's entries of older
    sources.  Calibration: the device copy reads
    as many bytes as it writes, and WRITE_SIZE counts the bytes written, so
    FETCH_SIZE is scaled by WRITE/FETCH of the copy.  The profiled launch is
    the kernel and grid of the last FP64 bounds dispatch (the timed launches;
    the autotuner's candidates run before them)."""
    import synth
    fetch = _counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _counter_per_dispatch(write_csv, "WRITE_SIZE")

    def copy_kib(d):
        v = [x[2] for x in d.values() if "copyBuffer" in x[0]]
        if not v:
            raise SystemExit("no calibration copy in the counter runs (use --copy-calibration)")
        return v[-1]

    scale = copy_kib(write) / copy_kib(fetch)

    def bounds_launches(d):
        runs, last = {}, None
        for name, grid, v in d.values():               # in dispatch order
            if "bounds_fp64_" in name and "bwd" not in name:
                kname = name.replace("void kbl::(anonymous namespace)::", "").split("(kbl")[0]
                runs.setdefault((kname, grid), []).append(v)
                last = (kname, grid)
        # the timed launches come last (after the autotuner's candidates)
        return last, runs[last]

    (kname, grid), fv = bounds_launches(fetch)
    (kname_w, grid_w), wv = bounds_launches(write)
    if (kname, grid) != (kname_w, grid_w):
        raise SystemExit(f"the two runs profiled different launches: {kname} {grid} / "
                         f"{kname_w} {grid_w}")
    f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
    wl = synth.make_workload(workload)
    nv = wl.dim + 2
    alg = (wl.n_nodes * nv * 8 + (wl.n_elem + 1) * 4 + wl.nnz * 4 + 2 * nv * wl.n_elem * 8
           + wl.n_elem * 4)
    nbytes = (f_kib * scale + w_kib) * 1024.0
    entry = {"workload": workload, "kernel": kname, "grid_threads": str(grid),
             "source_sha256": kernel_sources_sha(wl.dim),
             "fetch_kib_per_dispatch": f"{f_kib:.1f}", "write_kib_per_dispatch": f"{w_kib:.1f}",
             "fetch_scale": f"{scale:.4f}", "bytes_per_launch": f"{nbytes:.0f}",
             "algorithmic_bytes_per_launch": str(alg)}
    path = os.path.join(ROOT, TRAFFIC_FILE)
    head, blocks = [], []
    for line in open(path):
        if line.strip() == "[entry]":
            blocks.append([])
        (blocks[-1] if blocks else head).append(line)
    keep = []
    for b in blocks:
        kv = dict(l.strip().split(" = ", 1) for l in b if " = " in l)
        same = (kv.get("workload"), kv.get("kernel"), kv.get("grid_threads")) == \
            (workload, kname, str(grid))
        stale = kv.get("workload") == workload and kv.get("source_sha256") != entry["source_sha256"]
        if not (same or stale):   # counters of older sources are never used again
            keep.append(b)
    with open(path, "w") as fh:
        fh.writelines(head)
        for b in keep:
            fh.writelines(b)
        fh.write("[entry]\n")
        for k, v in entry.items():
            fh.write(f"{k} = {v}\n")
        fh.write(f"# ratio {nbytes / alg:.3f}\n")
    return entry


def pair_ops(dim: int) -> int:
    """Algorithmic VALU lane-ops per (stencil state, velocity node) pair, FP64.

    2D: the log-Maxwellian is separable, q = A[jx] + B[jy]: two adds (q and
    q + ln(theta delta/2)) and four running min/max.  3D: the same with
    q = A[jx] + (B[jy] + C[jz]), the bracket shared by all x nodes (its add
    is not counted).  1D: sub, mul, fma, fma, then four min/max.
    """
    return 8 if dim == 1 else 6


# Mixed precision (FP32 envelopes, 2D): the same two adds per pair, but the
# four running extrema take two states per step with the three-input
# v_min3_f32 / v_max3_f32, one issue slot per extremum and pair of states:
# 2 + 4/2 = 4 issue slots per pair at the unpacked FP32 VALU rate.
MIXED_PAIR_OPS = 4
# Dense FP16/BF16 matrix-core peak of MI355X (no sparsity).
MFMA_PEAK_FLOPS = 2.5e15


def mfma_flops_issued(wl, precision: int, tile: int, kbl) -> float:
    """Matrix-core flops one mixed bounds launch issues in its y-stage
    contraction: per element, each x tile of 16 nodes and each of the four
    envelopes runs KS k-steps of 16x16x16 MFMAs, 3 per k-step for the FP16
    hi/lo split, 6 for the BF16 three-way split (8192 flops each)."""
    txw, ks, nw = kbl._lib.MIXED_TILES[tile]
    per_k = 3 if precision == kbl.PREC_MIXED_FP16 else 6
    return float(wl.n_elem) * txw * nw * 4 * ks * per_k * 2 * 16 * 16 * 16


def kernel_shape(kbl, dim, tuned, n_elem, n_cu):
    """Kernel name and grid threads of the FP64 bounds launch for an
    autotuned choice (None, None without one)."""
    if dim == 1 or not tuned:
        return ("bounds_fp64_1d" if dim == 1 else f"bounds_fp64_{dim}d"), None
    blocks = kbl._lib.launch_workgroups(tuned, n_elem, n_cu)
    if dim == 2:
        bx, by, tx, ty, md = kbl._lib.FP64_TILES[tuned["tile"]]
        return f"bounds_fp64_2d<{bx}, {by}, {tx}, {ty}, {md}>", blocks * bx * by
    bx, by, bz, tx, ty, tz = kbl._lib.FP64_TILES_3D[tuned["tile"]]
    return f"bounds_fp64_3d<{bx}, {by}, {bz}, {tx}, {ty}, {tz}>", blocks * bx * by * bz


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, target_s: float = 12.0, one_core_s: float = 5.0):
    """The oracle (bounds + limit) on a seeded element sample of the workload,
    sized to take about target_s of wall time on all host cores, then on one
    core (OpenMP limited to one thread) for about one_core_s."""
    import ctypes
    import oracle
    oracle.build(force=False)
    oracle._load()
    try:
        gomp = ctypes.CDLL("libgomp.so.1")      # the OpenMP runtime liboracle links
        gomp.omp_get_max_threads.restype = ctypes.c_int
    except OSError:
        gomp = None
    rng = np.random.default_rng(12345)

    def run(n):
        sample = np.sort(rng.choice(wl.n_elem, n, replace=False))
        t0 = time.perf_counter()
        rb, _ = oracle.workload_bounds(wl, elems=sample)
        oracle.workload_limit(wl, rb, elems=sample)
        return time.perf_counter() - t0

    def sized(target):
        # grow the calibration sample until it takes at least 0.5 s, then size
        n, dt = 16, 0.0
        while n < wl.n_elem:
            dt = run(n)
            if dt >= 0.5:
                break
            n = min(wl.n_elem, n * 4)
        n = int(min(wl.n_elem, max(16, n * target / max(dt, 1e-6))))
        return n, run(n)

    threads = gomp.omp_get_max_threads() if gomp else (
        int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0)))
    n, dt = sized(target_s)
    out = {"value": n / dt, "unit": "elements/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} seeded random elements of {wl.name} (bounds + limit), {dt:.1f} s wall "
                     f"on {threads} threads, FP64 direct-form oracle (gcc -O2, OpenMP over "
                     f"elements)",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    if gomp is not None:
        gomp.omp_set_num_threads(1)
        n1, dt1 = sized(one_core_s)
        gomp.omp_set_num_threads(threads)
        out["one_core"] = {"value": n1 / dt1, "unit": "elements/s", "cores": 1,
                           "sample": f"{n1} seeded random elements, {dt1:.1f} s wall"}
    return out


def _time_events(torch, stream, fn, steps, warmup):
    """Average ms of fn() over `steps` calls, HIP events on the launch stream."""
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_variants(args, kbl, torch, synth, wl, st, rp, cl, tg, vg, stream, ms_step, b_ms):
    """The method's variants on the same inputs (and the node-level stencil on
    its own workload): per-state energy integrand, strict bounds (r = 0),
    independent limiting, solution + flux point stencils."""
    dev = st.device
    steps = max(2, args.steps // 2)
    out = {}
    bnd = torch.empty((8, wl.n_elem), dtype=torch.float64, device=dev)
    bst = torch.empty(wl.n_elem, dtype=torch.int32, device=dev)
    lim = torch.empty_like(tg)
    # energy bounds from the per-state integrand: 7 ops per pair (g = EA EB,
    # h + c, product, four min/max) in value space
    prm_e = kbl.make_params(wl.gamma, r_fac=wl.r_fac, energy_perstate=True)
    ms = _time_events(torch, stream, lambda: kbl.compute_bounds(
        st, rp, cl, wl.n_s, vg, prm_e, out=bnd, status=bst, stream=stream), steps, args.warmup)
    ops = wl.pairs() * 7
    out["energy_perstate"] = {"bounds_ms": ms, "vs_default_bounds": ms / b_ms,
                              "ops_per_pair": 7, "frac": ops / (ms * 1e-3) / VALU_PEAK_OPS}
    # strict bounds: same kernels, r_fac = 0; report how many more elements limit
    prm0 = kbl.make_params(wl.gamma, r_fac=0.0)
    prm1 = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    al = torch.empty((2, wl.n_elem), dtype=torch.float64, device=dev)

    def step0():
        kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm0, out=bnd, status=bst, stream=stream)
        kbl.limit(tg, bnd, wl.node_weights, wl.n_s, prm0, out=lim, alpha=al, stream=stream)
    ms0 = _time_events(torch, stream, step0, steps, args.warmup)
    lim0 = int((al[0] < 1).sum())
    kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm1, out=bnd, status=bst, stream=stream)
    kbl.limit(tg, bnd, wl.node_weights, wl.n_s, prm1, out=lim, alpha=al, stream=stream)
    torch.cuda.synchronize()
    lim1 = int((al[0] < 1).sum())
    out["strict_r0"] = {"ms_per_step": ms0, "value": wl.n_elem / (ms0 * 1e-3),
                        "limited_elements": lim0, "limited_elements_relaxed": lim1}
    # independent limiting (limiter only; bounds from the default method)
    prm_i = kbl.make_params(wl.gamma, r_fac=wl.r_fac, independent_alpha=True)
    msi = _time_events(torch, stream, lambda: kbl.limit(
        tg, bnd, wl.node_weights, wl.n_s, prm_i, out=lim, stream=stream), steps, args.warmup)
    out["independent_alpha"] = {"limit_ms": msi,
                                "limit_hbm_frac": (2 * tg.numel() * 8 + bnd.numel() * 8)
                                / (msi * 1e-3) / HBM_PEAK}
    # node-level stencils of solution + flux points (256^2 quads, 48 states each)
    if not args.no_fr:
        print("[bench] generating quad256_fr", file=sys.stderr, flush=True)
        fr = synth.make_workload("quad256_fr")
        fst = torch.from_numpy(fr.states).to(dev)
        frp = torch.from_numpy(fr.rowptr).to(dev)
        fcl = torch.from_numpy(fr.cols).to(dev)
        ftg = torch.from_numpy(fr.target).to(dev)
        fg = fr.grid
        fvg = kbl.make_vgrid(fg.mode, fg.n[:2], fg.lo, fg.hi, fg.k)
        fb = torch.empty((8, fr.n_elem), dtype=torch.float64, device=dev)
        fs = torch.empty(fr.n_elem, dtype=torch.int32, device=dev)
        flim = torch.empty_like(ftg)

        def fstep():
            kbl.compute_bounds_nodes(fst, frp, fcl, fvg, prm1, out=fb, status=fs, stream=stream)
            kbl.limit(ftg, fb, fr.v_weights, fr.n_v, prm1, out=flim, stream=stream)
        msf = _time_events(torch, stream, fstep, steps, args.warmup)
        # the bounds launch alone, averaged over the same number of steps
        fbms = _time_events(torch, stream, lambda: kbl.compute_bounds_nodes(
            fst, frp, fcl, fvg, prm1, out=fb, status=fs, stream=stream), steps, args.warmup)
        out["node_stencil_fr"] = {
            "workload": "quad256_fr: 256x256 periodic quads, p=3, per element 16 solution "
                        "points + 16 own flux points + 16 neighbour flux points (48 states), "
                        "48x48 per-stencil grid, V = 32 nodes (flux points weight 0)",
            "ms_per_step": msf, "value": fr.n_elem / (msf * 1e-3), "unit": "elements/s",
            "bounds_ms": fbms, "frac": fr.pairs() * 6 / (fbms * 1e-3) / VALU_PEAK_OPS}
        print(f"[bench] node-stencil FR: {msf:.3f} ms/step (bounds {fbms:.3f} ms)",
              file=sys.stderr, flush=True)
        # Riemann-averaged states of every face pair, checked against the bounds
        P = fr.meta["face_pairs"]
        pni, pnj = torch.from_numpy(P["ni"]).to(dev), torch.from_numpy(P["nj"]).to(dev)
        pn = torch.from_numpy(P["normals"]).to(dev)
        pe = torch.from_numpy(P["elem"]).to(dev)
        kbl.compute_bounds_nodes(fst, frp, fcl, fvg, prm1, out=fb, status=fs, stream=stream)
        msr = _time_events(torch, stream, lambda: kbl.riemann_states(
            fst, pni, pnj, pn, prm1, bounds=fb, elem=pe, stream=stream), steps, args.warmup)
        _, rst = kbl.riemann_states(fst, pni, pnj, pn, prm1, bounds=fb, elem=pe, stream=stream)
        torch.cuda.synchronize()
        npairs = int(pni.numel())
        # bytes per pair: two gathered states, ids, normal, element id, the
        # element's bounds, the averaged state and the status written
        bpp = 2 * 4 * 8 + 2 * 4 + 2 * 8 + 4 + 8 * 8 + 4 * 8 + 4
        out["riemann_states_fr"] = {
            "pairs": npairs, "ms": msr, "pairs_per_s": npairs / (msr * 1e-3),
            "hbm_frac_upper": npairs * bpp / (msr * 1e-3) / HBM_PEAK,
            "outside_bounds": int((rst != 0).sum().item()),
            "what": "Riemann-averaged state (Thm. 4.3) of every flux-point pair, wavespeed "
                    "estimate, checked against the element bounds"}
        print(f"[bench] riemann states: {msr:.3f} ms for {npairs} pairs, "
              f"{out['riemann_states_fr']['outside_bounds']} outside the bounds",
              file=sys.stderr, flush=True)
        del fst, ftg, flim
    print(f"[bench] variants: energy {ms:.3f} ms, strict {ms0:.3f} ms/step, independent limit "
          f"{msi:.3f} ms", file=sys.stderr, flush=True)
    return out


def time_3d(args, kbl, torch, synth, stream):
    """The same step on a 3D velocity grid (hex32): the d = 3 kernel whose cost
    the paper's conclusion flags."""
    dev = torch.device("cuda:0")
    print("[bench] generating hex32", file=sys.stderr, flush=True)
    wl = synth.make_workload("hex32")
    g = wl.grid
    st = torch.from_numpy(wl.states).to(dev)
    rp = torch.from_numpy(wl.rowptr).to(dev)
    cl = torch.from_numpy(wl.cols).to(dev)
    tg = torch.from_numpy(wl.target).to(dev)
    vg = kbl.make_vgrid(g.mode, g.n[:3], g.lo, g.hi, g.k)
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    bnd = torch.empty((10, wl.n_elem), dtype=torch.float64, device=dev)
    bst = torch.empty(wl.n_elem, dtype=torch.int32, device=dev)
    lim = torch.empty_like(tg)
    tuned = None
    if not args.no_autotune:
        c = kbl.autotune_bounds(st, rp, cl, wl.n_s, vg, prm, sample_elems=8192, stream=stream)
        tuned = kbl._lib.decode_autotune(c)
        print(f"[bench] autotuned hex32: {tuned}", file=sys.stderr, flush=True)
    steps = max(2, args.steps // 2)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]

    def step(e=None):
        if e is not None:
            e[0].record(stream)
        kbl.compute_bounds(st, rp, cl, wl.n_s, vg, prm, out=bnd, status=bst, stream=stream)
        if e is not None:
            e[1].record(stream)
        kbl.limit(tg, bnd, wl.node_weights, wl.n_s, prm, out=lim, stream=stream)
        if e is not None:
            e[2].record(stream)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(ev[i])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    b_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    l_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    kname, gthreads = kernel_shape(kbl, 3, tuned, wl.n_elem, n_cu)
    ops = wl.pairs() * pair_ops(3)
    print(f"[bench] hex32: {ms:.3f} ms/step (bounds {b_ms:.3f} ms, limit {l_ms:.3f} ms)",
          file=sys.stderr, flush=True)
    traffic, traffic_grid = (profiled_traffic(kname, gthreads, "hex32", 3) if gthreads
                             else (None, None))
    out = {"workload": f"hex32: {WORKLOAD_TEXT['hex32']}", "n_elem": wl.n_elem,
           "value": wl.n_elem / (ms * 1e-3), "unit": "elements/s", "ms_per_step": ms,
           "bounds_ms": b_ms, "limit_ms": l_ms, "kernel": kname, "grid_threads": gthreads,
           "pairs_per_launch": wl.pairs(), "ops_per_pair": pair_ops(3),
           "frac": ops / (b_ms * 1e-3) / VALU_PEAK_OPS, "traffic": traffic,
           "traffic_unit": "bytes per launch", "traffic_grid_threads": traffic_grid, "launch": tuned,
           "parity_tol": 1e-12}
    del st, tg, lim
    return out


def time_fr1d(args, kbl, torch, stream):
    """One SSP-RK3 step of the 1D FR solver with the kinetic bounds and limiter
    after every stage (Sec. 5), on the paper's finest Sod mesh (p = 3,
    N = 3200, velocity grid k = 8 with 2048 nodes)."""
    from synth import fr1d_problems as probs
    pr = probs.sod(3, 3200)
    s = kbl.FR1D(pr.p, pr.n_elem, pr.x0, pr.x1, pr.gamma, bc=pr.bc, left=pr.left,
                 right=pr.right, r_fac=1e-3, n_u=2048, k=8.0, stream=stream)
    s.set_solution(pr.U0)
    h = (pr.x1 - pr.x0) / pr.n_elem
    dt = 0.1 * h / ((2 * pr.p + 1) * s.max_speed())
    steps = max(20, 10 * args.steps)
    ms = _time_events(torch, stream, lambda: s.step(dt), steps, max(2, args.warmup))
    # the same with the CFL time step taken every step (one host sync each)
    t0 = time.perf_counter()
    for _ in range(steps):
        sp = s.max_speed()
        s.step(0.1 * h / ((2 * pr.p + 1) * sp))
    torch.cuda.synchronize()
    ms_cfl = 1e3 * (time.perf_counter() - t0) / steps
    # the CFL time step computed on the device, steps replayed from a HIP graph
    # in batches of 50 (no host sync per step; the capture is included)
    g = kbl.FR1D(pr.p, pr.n_elem, pr.x0, pr.x1, pr.gamma, bc=pr.bc, left=pr.left,
                 right=pr.right, r_fac=1e-3, n_u=2048, k=8.0, stream=stream)
    g.set_solution(pr.U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_graph = g.run_device(10 * steps * dt, 0.1, batch=50)
    torch.cuda.synchronize()
    ms_graph = 1e3 * (time.perf_counter() - t0) / max(n_graph, 1)
    del g
    pairs = 3 * (pr.n_elem * (pr.p + 5) + 2 * (pr.p + 3)) * 2048
    print(f"[bench] fr1d sod p=3 N=3200: {ms:.3f} ms/step ({ms_cfl:.3f} with the CFL sync, "
          f"{ms_graph:.3f} with the device CFL step in HIP graphs over {n_graph} steps)",
          file=sys.stderr, flush=True)
    return {"workload": "Sod shock tube, FR p=3, 3200 elements, HLLC, SSP-RK3 with the kinetic "
                        "bounds (k=8, 2048 velocity nodes, node stencils of 10 states) and the "
                        "squeeze limiter after every stage",
            "ms_per_step": ms, "steps_per_s": 1e3 / ms, "ms_per_step_with_cfl_sync": ms_cfl,
            "ms_per_step_device_cfl_graph": ms_graph, "graph_steps": n_graph,
            "element_stages_per_s": 3 * pr.n_elem / (ms * 1e-3),
            "bounds_pairs_per_step": pairs,
            "launches_per_step": 14}


class Dev:
    """A workload's inputs resident on the device, and output buffers."""

    def __init__(self, kbl, torch, wl, dev):
        g = wl.grid
        self.wl = wl
        self.st = torch.from_numpy(wl.states).to(dev)
        self.rp = torch.from_numpy(wl.rowptr).to(dev)
        self.cl = torch.from_numpy(wl.cols).to(dev)
        self.tg = torch.from_numpy(wl.target).to(dev)
        self.vg = kbl.make_vgrid(g.mode, g.n[: wl.dim], g.lo, g.hi, g.k)
        self.bounds = torch.empty((2 * (wl.dim + 2), wl.n_elem), dtype=torch.float64, device=dev)
        self.bstat = torch.empty(wl.n_elem, dtype=torch.int32, device=dev)
        self.lim = torch.empty_like(self.tg)
        self.alpha = torch.empty((2, wl.n_elem), dtype=torch.float64, device=dev)
        self.lstat = torch.empty(wl.n_elem, dtype=torch.int32, device=dev)


def time_step(kbl, torch, d, prm_b, prm_l, stream, steps, warmup):
    """One step = bounds + limit, timed over `steps` after `warmup`: wall ms
    per step (host clock around synchronisations) and the average bounds and
    limit launch times (HIP events recorded on the launch stream)."""
    wl = d.wl

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        kbl.compute_bounds(d.st, d.rp, d.cl, wl.n_s, d.vg, prm_b, out=d.bounds, status=d.bstat,
                           stream=stream)
        if ev is not None:
            ev[1].record(stream)
        kbl.limit(d.tg, d.bounds, wl.node_weights, wl.n_s, prm_l, out=d.lim, alpha=d.alpha,
                  status=d.lstat, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t0) / steps
    b_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    l_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    return wall, b_ms, l_ms


def autotune(args, kbl, d, prm, stream, label, sample=65536):
    """Untimed: picks the tile and launch shape for this problem shape."""
    if args.no_autotune:
        return None
    wl = d.wl
    c = kbl.autotune_bounds(d.st, d.rp, d.cl, wl.n_s, d.vg, prm, sample_elems=sample,
                            stream=stream)
    t = kbl._lib.decode_autotune(c)
    print(f"[bench] autotuned {label}: {t}", file=sys.stderr, flush=True)
    return t


def limit_hbm_frac(d, l_ms):
    """Limiter launch against HBM peak: solution read, limited solution,
    bounds, alpha and status written or read once."""
    wl = d.wl
    byts = 2 * wl.target.nbytes + d.bounds.numel() * 8 + d.alpha.numel() * 8 + d.lstat.numel() * 4
    return byts / (l_ms * 1e-3) / HBM_PEAK


def fp64_leg(args, kbl, torch, d, stream, n_cu, label, steps):
    """FP64 step on one workload: throughput and the bounds kernel's roofline."""
    wl = d.wl
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    tuned = autotune(args, kbl, d, prm, stream, f"{label} fp64")
    ms, b_ms, l_ms = time_step(kbl, torch, d, prm, prm, stream, steps, args.warmup)
    print(f"[bench] {label} fp64: {ms:.3f} ms/step (bounds {b_ms:.3f} ms, limit {l_ms:.3f} ms)",
          file=sys.stderr, flush=True)
    ops = wl.pairs() * pair_ops(wl.dim)
    achieved = ops / (b_ms * 1e-3)
    kname, grid_threads = kernel_shape(kbl, wl.dim, tuned, wl.n_elem, n_cu)
    traffic, traffic_grid = (profiled_traffic(kname, grid_threads, wl.name, wl.dim)
                             if grid_threads else (None, None))
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
            "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS, "traffic": traffic,
            "traffic_unit": "bytes per launch", "traffic_source": TRAFFIC_FILE,
            "traffic_grid_threads": traffic_grid, "kernel": kname, "grid_threads": grid_threads,
            "ops_per_launch": ops, "pairs_per_launch": wl.pairs(),
            "ops_per_pair": pair_ops(wl.dim), "kernel_ms": b_ms, "limit_ms": l_ms,
            "limit_hbm_frac": limit_hbm_frac(d, l_ms)}
    return {"ms_per_step": ms, "value": wl.n_elem / (ms * 1e-3), "unit": "elements/s",
            "bounds_ms": b_ms, "limit_ms": l_ms, "launch": tuned, "roofline": roof,
            "parity_tol": 1e-12}


def mixed_legs(args, kbl, torch, d, stream, label, steps, ms_fp64, b_fp64):
    """The same step with each mixed-precision form of the bounds (the
    limiter stays FP64)."""
    wl = d.wl
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    out = {}
    forms = (("fp32_valu", kbl.PREC_MIXED_FP32), ("fp16_mfma", kbl.PREC_MIXED_FP16),
             ("bf16_mfma", kbl.PREC_MIXED_BF16))
    for name, prec in forms:
        if name not in args.mixed_forms.split(","):
            continue
        prm_m = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=prec)
        tuned = autotune(args, kbl, d, prm_m, stream, f"{label} {name}")
        ms, b_ms, l_ms = time_step(kbl, torch, d, prm_m, prm, stream, steps, args.warmup)
        ops = wl.pairs() * MIXED_PAIR_OPS
        e = {"value": wl.n_elem / (ms * 1e-3), "unit": "elements/s", "ms_per_step": ms,
             "bounds_ms": b_ms, "limit_ms": l_ms,
             "roofline": {"bound": "alu", "achieved": ops / (b_ms * 1e-3) / 1e12,
                          "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
                          "frac": ops / (b_ms * 1e-3) / VALU_PEAK_OPS,
                          "ops_per_pair": MIXED_PAIR_OPS},
             "speedup_vs_fp64": ms_fp64 / ms, "bounds_speedup_vs_fp64": b_fp64 / b_ms,
             "launch": tuned, "parity_tol": 1e-5}
        if prec != kbl.PREC_MIXED_FP32:
            tile = tuned["tile"] if tuned else None
            if tile is None:
                g = wl.grid.n
                n = max(g[0], g[1])
                tile = 0 if n <= 16 else 1 if n <= 32 else 3 if n <= 48 else 5
            fl = mfma_flops_issued(wl, prec, tile, kbl)
            e["mfma"] = {"flops_issued_per_launch": fl,
                         "achieved": fl / (b_ms * 1e-3) / 1e12, "peak": MFMA_PEAK_FLOPS / 1e12,
                         "unit": "TFLOP/s", "frac": fl / (b_ms * 1e-3) / MFMA_PEAK_FLOPS}
        out[name] = e
        print(f"[bench] {label} mixed {name}: {ms:.3f} ms/step (bounds {b_ms:.3f} ms, "
              f"frac {e['roofline']['frac']:.3f})", file=sys.stderr, flush=True)
    return out


def backward_leg(args, kbl, torch, synth, stream, name="quad512"):
    """The hand-written backward of bounds + limiter on the differentiation
    workload, J = sum w rho_limited; the forward's bounds and status are
    handed over (as the autograd Function does)."""
    dev = torch.device("cuda:0")
    print(f"[bench] generating {name}", file=sys.stderr, flush=True)
    d = Dev(kbl, torch, synth.make_workload(name), dev)
    wl = d.wl
    prm = kbl.make_params(wl.gamma, r_fac=wl.r_fac)
    autotune(args, kbl, d, prm, stream, f"{name} fp64")
    steps = max(2, args.steps // 2)
    ms_fwd, b_fwd, _ = time_step(kbl, torch, d, prm, prm, stream, steps, args.warmup)
    G = torch.zeros_like(d.tg)
    G[0] = torch.from_numpy(np.random.default_rng(7).standard_normal(wl.n_nodes)).to(dev)

    def limited_fraction(p, tg):
        fb, _ = kbl.compute_bounds(d.st, d.rp, d.cl, wl.n_s, d.vg, p, stream=stream)
        _, _, ls = kbl.limit(tg, fb, wl.node_weights, wl.n_s, p, stream=stream)
        counts = kbl.status_summary(ls, stream=stream).cpu()
        return float(counts[3]) / wl.n_elem        # bit 3: KBL_ST_LIMITED (alpha < 1)

    def time_backward(p, tg=None):
        tg = d.tg if tg is None else tg
        fb = torch.empty_like(d.bounds)
        fs = torch.empty_like(d.bstat)
        kbl.compute_bounds(d.st, d.rp, d.cl, wl.n_s, d.vg, p, out=fb, status=fs, stream=stream)

        def bstep():
            return kbl.bounds_limit_backward(d.st, d.rp, d.cl, wl.n_s, d.vg, p, tg,
                                             wl.node_weights, G, fwd_bounds=fb, fwd_status=fs,
                                             stream=stream)

        for _ in range(max(1, args.warmup)):
            res = bstep()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            bstep()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, res

    bms, res = time_backward(prm)
    gref = res[0] + res[1]
    frac = limited_fraction(prm, d.tg)
    # the forward step again after the backward timings; the reference is
    # the faster of the two (a slow outlier makes the ratio look better)
    ms_fwd2, b_fwd2, _ = time_step(kbl, torch, d, prm, prm, stream, steps, args.warmup)
    fwd_runs = [ms_fwd, ms_fwd2]
    if ms_fwd2 < ms_fwd:
        ms_fwd, b_fwd = ms_fwd2, b_fwd2
    # Every element limited: the solution's deviation from the stencil
    # states amplified 1e4 times (the kinetic bounds are wide; at 1e3 about
    # two thirds of the elements bind a bound).  This is the dense cost of
    # the bounds adjoint, which the default target exercises only where the
    # limiter binds.
    tg_dense = d.st + 1e4 * (d.tg - d.st)
    dms, dres = time_backward(prm, tg_dense)
    # elements per binding bound: the nonzero entry of each row of dJ/dbounds
    rows = ["rho_min"] + [f"m{j}_min" for j in range(wl.dim)] + ["E_min", "rho_max"] + \
           [f"m{j}_max" for j in range(wl.dim)] + ["E_max"]
    binding = dict(zip(rows, (dres[2] != 0).sum(dim=1).tolist()))
    dense = {"ms_per_call": dms, "vs_forward_step": dms / ms_fwd,
             "limited_fraction": limited_fraction(prm, tg_dense),
             "elements_per_binding_bound": binding,
             "what": "the same call with every element limited: target = states + "
                     "1e4 (target - states)"}
    del tg_dense
    print(f"[bench] {name} backward, every element limited: {dms:.3f} ms/call "
          f"({100 * dense['limited_fraction']:.1f}% limited)", file=sys.stderr, flush=True)
    out = {"workload": f"{name}: {WORKLOAD_TEXT[name]}", "n_elem": wl.n_elem,
           "value": wl.n_elem / (bms * 1e-3), "unit": "elements/s", "ms_per_call": bms,
           "forward_ms_per_step": ms_fwd, "forward_bounds_ms": b_fwd,
           "forward_ms_per_step_runs": fwd_runs,
           "vs_forward_step": bms / ms_fwd, "limited_fraction": frac,
           "what": "kbl_bounds_limit_backward given the forward bounds: limiter backward, "
                   "bounds backward (envelopes and winners recomputed where a bound binds; "
                   "elements with a zero bounds adjoint contribute exactly zero), gather; "
                   "FP64; J = sum w rho_limited, w ~ N(0, 1)",
           "all_limited": dense}
    print(f"[bench] {name} backward: {bms:.3f} ms/call (forward step {ms_fwd:.3f} ms, "
          f"{100 * frac:.1f}% of the elements limited)", file=sys.stderr, flush=True)
    if not args.no_mixed:
        prm_m = kbl.make_params(wl.gamma, r_fac=wl.r_fac, precision=kbl.PREC_MIXED_FP32)
        mms, mres = time_backward(prm_m)
        gmix = mres[0] + mres[1]
        scale = float(gref.abs().max())
        diff = (gmix - gref).abs()
        out["mixed_fp32"] = {
            "ms_per_call": mms, "speedup_vs_fp64": bms / mms,
            "max_err_rel_to_max_grad": float(diff.max()) / scale,
            "p99_err_rel_to_max_grad": float(torch.quantile(diff.flatten()[:1 << 24].float(),
                                                            0.99)) / scale,
            "what": "gradient of the mixed forward (FP32 envelopes and winners, FP64 shares and "
                    "chain rule), compared with the FP64 gradient"}
        print(f"[bench] {name} mixed backward: {mms:.3f} ms/call, max err "
              f"{float(diff.max()) / scale:.2e} of the max gradient", file=sys.stderr, flush=True)
    return out


def workload_config(name, wl):
    sizes = wl.stencil_sizes()
    cfg = {"workload": f"{name}: {WORKLOAD_TEXT.get(name, '')}", "n_elem": wl.n_elem,
           "nodes_per_elem": wl.n_s, "velocity_grid": list(wl.grid.n[: wl.dim]),
           "grid_mode": "stencil" if wl.grid.mode == 1 else "global",
           "pairs_per_pass": wl.pairs()}
    if sizes.min() != sizes.max():
        h = np.bincount(sizes)
        cfg["stencil_elements"] = {"min": int(sizes.min()), "max": int(sizes.max()),
                                   "mean": float(sizes.mean()),
                                   "histogram": {str(k): int(h[k]) for k in range(len(h)) if h[k]}}
    else:
        cfg["stencil_elements"] = int(sizes[0])
    return cfg


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tri2m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision timings")
    ap.add_argument("--mixed-forms", default="fp32_valu,fp16_mfma,bf16_mfma",
                    help="comma-separated mixed forms to time (profiling runs)")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward timing")
    ap.add_argument("--no-second", action="store_true",
                    help="skip the 1024^2-quad global-grid leg")
    ap.add_argument("--no-fr", action="store_true", help="skip the node-level stencil timing")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D velocity-grid timing")
    ap.add_argument("--solver", action="store_true", help="also time the 1D FR solver step")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the variant timings (energy reading, r = 0, independent "
                         "limiting, node-level stencils)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default launch configuration instead of an autotuned one")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no timing: turn the counter CSVs of a FETCH_SIZE and a WRITE_SIZE "
                         "run on --workload into its entry of " + TRAFFIC_FILE)
    args = ap.parse_args(argv)
    if args.write_traffic:
        e = write_traffic(args.workload, *args.write_traffic)
        print(json.dumps(e))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the bounds path runs on a single MI355X "
              "(there is no multi-GPU path); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_2407_20966_amd as kbl
    import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {n * 8} bytes read, {n * 8} bytes written",
              file=sys.stderr, flush=True)
        del src, dst

    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    wl = synth.make_workload(args.workload)
    d = Dev(kbl, torch, wl, dev)
    head = fp64_leg(args, kbl, torch, d, stream, n_cu, args.workload, args.steps)
    cfg = workload_config(args.workload, wl)
    cfg.update({"precision": "fp64", "parity_tol": 1e-12})
    if head["launch"]:
        cfg["launch"] = {"autotuned": head["launch"],
                         "note": "elements_per_workgroup: elements computed by one "
                                 "workgroup; workgroups_per_cu: persistent grid"}
    out = {"metric": METRIC, "value": head["value"], "unit": "elements/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
           "roofline": head["roofline"]}
    if wl.dim == 2 and not args.no_mixed:
        out["mixed"] = mixed_legs(args, kbl, torch, d, stream, args.workload, args.steps,
                                  head["ms_per_step"], head["bounds_ms"])
    if not args.no_variants and wl.dim == 2:
        out["variants"] = time_variants(args, kbl, torch, synth, wl, d.st, d.rp, d.cl, d.tg,
                                        d.vg, stream, head["ms_per_step"], head["bounds_ms"])
    del d
    torch.cuda.empty_cache()
    second = "quad1024_sine"
    if not args.no_second and args.workload != second:
        print(f"[bench] generating {second}", file=sys.stderr, flush=True)
        wl2 = synth.make_workload(second)
        d2 = Dev(kbl, torch, wl2, dev)
        steps2 = max(2, args.steps // 2)
        leg = fp64_leg(args, kbl, torch, d2, stream, n_cu, second, steps2)
        leg["config"] = workload_config(second, wl2)
        if not args.no_mixed:
            leg["mixed"] = mixed_legs(args, kbl, torch, d2, stream, second, steps2,
                                      leg["ms_per_step"], leg["bounds_ms"])
        out[second] = leg
        del d2, wl2
        torch.cuda.empty_cache()
    if not args.no_backward and wl.dim == 2:
        out["backward"] = backward_leg(args, kbl, torch, synth, stream)
        torch.cuda.empty_cache()
    if not args.no_3d and wl.dim == 2:
        out["three_d"] = time_3d(args, kbl, torch, synth, stream)
    if args.solver and wl.dim == 2:
        out["fr1d_solver"] = time_fr1d(args, kbl, torch, stream)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
