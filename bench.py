"""Throughput of the fused multicomponent LB step on one MI355X.

Workload: neutral binary mixture on a 256^3 periodic D3Q19 lattice, FP32 populations
stored as deviations from rest (f - w rho0), rest density 0.5 per species, 8 seeded
concentration modes (amplitude 1e-3, antiphase between species) plus a shear wave
u_y = 1e-3 sin(2 pi x / 256), tau_visc = 1, Sc = 100 (synthetic inputs from
workloads.binary_multimode, seed 2).  One step = one fused stream-collide launch (pull
streaming, moments, drag, collision, store, FP64 mass partials).  The timed steps run as 5
windows and the median per-step time is reported.  The same workload is also timed with
plain FP32, FP16 and BF16 storage and with stochastically rounded FP32 ("variants").

Prints one JSON line: species-site updates per second (GLUPS), the roofline of the
stream-collide kernel against MI355X HBM bandwidth (with the measured ceiling of a plain
device copy), every other configuration ("configs": the charged ternary slit 64 x 64 x 130
with the direct, SOR and multigrid solvers, the 128 x 128 x 258 slit, 64 batched channels and
the 512^3 binary), and the FP64 CPU oracle, built for this host, timed on a bounded sample of
the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
Q = 19


def code_text(src: str) -> str:
    """C++ source without its comments, whitespace runs folded to one space (string and
    character literals kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the code of the fused step kernel, comments and layout aside (its counters are
    void once the code changes)."""
    h = hashlib.sha256()
    for name in ("lbmix_step_kernel.h", "lbmix_step.hip", "lbmix_step.h", "lbmix_device.h"):
        with open(os.path.join(ROOT, "paper_1507_04891_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(storage: str, n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"stream_collide_{storage}_binary_{n}cubed_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, sc: float, target_s: float = 12.0):
    """The FP64 oracle on the same 256^3 workload, a bounded number of steps, built for this
    host (gcc -O3 -march=native, no FMA contraction, OpenMP) in a temporary directory."""
    import tempfile

    import oracle

    tmpdir = tempfile.mkdtemp(prefix="lbmix_oracle_")
    path = oracle.build(native=True, path=os.path.join(tmpdir, "liblbmix_oracle_native.so"))
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.nspecies, w.omega_visc, w.omega_drag, lib_path=path)
    for s in range(w.nspecies):
        o.set_state(s, w.n[s], w.u[s])
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    extra = max(0, min(20, int(target_s / max(t1, 1e-3)) - 1))
    t0 = time.perf_counter()
    if extra:
        o.step(extra)
    t2 = time.perf_counter() - t0
    del o
    steps = 1 + extra
    elapsed = t1 + t2
    sites = w.nspecies * w.nx * w.ny * w.nz
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": sites * steps / elapsed / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} of the 2000 steps of the {w.nx}^3 binary workload, FP64, "
                     f"{elapsed:.1f} s on {threads} OpenMP threads",
           "cpu_model": cpu_model(), "build": "gcc " + " ".join(oracle.NATIVE_FLAGS)}
    # the same oracle on one thread, one step, in a child process (OpenMP reads its thread
    # count at start-up); the child does not touch the GPU
    code = ("import sys, time; sys.path.insert(0, %r); import oracle, workloads as WL; "
            "w = WL.binary_multimode(n=%d, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=%r, seed=2); "
            "o = oracle.Oracle(w.nx, w.ny, w.nz, w.nspecies, w.omega_visc, w.omega_drag, lib_path=%r); "
            "[o.set_state(s, w.n[s], w.u[s]) for s in range(w.nspecies)]; "
            "t0 = time.perf_counter(); o.step(1); print(time.perf_counter() - t0)") % (ROOT, w.nx, sc, path)
    try:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        one = float(r.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": sites / one / 1e9, "unit": "GLUPS", "cores": 1,
                                "sample": f"1 step of the same workload, {one:.1f} s"}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        out["single_thread"] = {"value": None, "error": str(e)[:200]}
    return out


WINDOWS = 5


def timed_windows(run, stream, steps, windows=WINDOWS):
    """Run `steps` steps as `windows` consecutive windows (run(k) issues k steps on `stream`),
    each bracketed by HIP events; returns the per-step milliseconds of every window."""
    import torch

    sizes = [steps // windows + (1 if i < steps % windows else 0) for i in range(windows)]
    sizes = [k for k in sizes if k > 0]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(sizes) + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i, k in enumerate(sizes):
        run(k)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) / k for i, k in enumerate(sizes)]


def median(v):
    v = sorted(v)
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def copy_ceiling(nbytes=2 << 30):
    """HBM bandwidth of the library's plain device copy (lbmix_device_copy: 16-byte
    non-temporal loads and stores, each byte read once and written once) of nbytes: the median
    of 5 timed copies after 2 untimed ones."""
    import torch

    import paper_1507_04891_amd as P

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        P.device_copy(dst, src, stream)
    ms = timed_windows(lambda k: [P.device_copy(dst, src, stream) for _ in range(k)], stream, 5)
    torch.cuda.synchronize()
    ok = bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    gbs = [2 * nbytes / (t * 1e-3) / 1e9 for t in ms]
    return {"gbs": round(median(gbs), 1), "bytes": nbytes, "kernel": "lbmix_device_copy (plain copy kernel)",
            "frac_of_peak": round(median(gbs) / HBM_PEAK_GBS, 4), "copy_ok": ok}


def time_storage(P, w, storage, steps, warmup, autotune=False, stochastic=None):
    """Time `steps` steps of the workload with one storage form, as 5 windows whose median
    per-step time is reported; one fused launch per step (work-group shape: the library's
    default, or its autotuner's pick)."""
    import torch

    stream = torch.cuda.current_stream()
    lat = P.from_workload(w, storage=storage, stream=stream, stochastic=stochastic)
    shape = lat.autotune(reps=5) if autotune else None
    lat.step(warmup)
    ms = timed_windows(lat.step, stream, steps)
    totals = lat.mass_totals()
    nodes = w.nx * w.ny * w.nz
    assert all(abs(t / (0.5 * nodes) - 1) < 1e-5 for t in totals), (storage, totals)
    del lat
    torch.cuda.empty_cache()
    sites = w.nspecies * nodes
    esize = P.ELEMENT_BYTES[P.STORAGE[storage]]
    ms_per_step = median(ms)
    achieved = 2 * Q * esize * sites / (ms_per_step * 1e-3) / 1e9   # 19 reads + 19 writes
    return {"glups": sites / (ms_per_step * 1e-3) / 1e9, "ms_per_step": ms_per_step,
            "window_ms": [round(t, 5) for t in ms], "achieved_gbs": achieved,
            "frac": achieved / HBM_PEAK_GBS, "launch": shape}


def lattice_config(P, w, storage, steps, warmup, poisson=None, charged=False):
    """ms/step (median of 5 windows), GLUPS and the step's HBM fraction (the stream-collide's
    algorithmic bytes, plus the potential read and charge write of a charged run, over the
    whole step's time) of one workload; with a Poisson solve, its work per step too."""
    import torch

    stream = torch.cuda.current_stream()
    lat = P.from_workload(w, storage=storage, stream=stream, poisson=poisson)
    lat.step(warmup)
    st0 = lat.stats()
    ms = timed_windows(lat.step, stream, steps)
    st1 = lat.stats()
    nodes = int(st1["fluid_nodes"])
    sites = w.nspecies * nodes
    esize = P.ELEMENT_BYTES[P.STORAGE[storage]]
    t = median(ms)
    nbytes = 2 * Q * esize * sites + (16 * nodes if charged else 0)
    out = {"storage": storage, "ms_per_step": round(t, 5), "spread_ms": [round(min(ms), 5), round(max(ms), 5)],
           "glups": round(sites / (t * 1e-3) / 1e9, 3),
           "step_hbm_frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if poisson:
        out["poisson"] = poisson.get("method", "sor")
        out["poisson_work_per_step"] = round((st1["total_sweeps"] - st0["total_sweeps"]) / steps, 2)
        out["last_residual"] = st1["last_residual"]
    del lat
    torch.cuda.empty_cache()
    return out


def bench_configs(P, WL, steps, warmup):
    """Every configuration beyond the headline, each timed as 5 windows of `steps` steps."""
    import torch

    out = {}
    mark = lambda k: print(f"config {k} done", file=sys.stderr, flush=True)
    slit = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    for st in ("f32s", "f16s"):
        k = f"charged_slit_64x64x130_direct_{st}"
        out[k] = lattice_config(P, slit, st, steps, warmup, dict(method="direct"), charged=True)
        mark(k)
    k = "charged_slit_64x64x130_sor_f32s"
    out[k] = lattice_config(P, slit, "f32s", steps, warmup,
                            dict(method="sor", rel_tol=1e-8, max_sweeps=1000000, check_every=10), charged=True)
    mark(k)
    k = "charged_slit_64x64x130_sor_f32"
    out[k] = lattice_config(P, slit, "f32", steps, warmup,
                            dict(method="sor", rel_tol=1e-8, max_sweeps=1000000, check_every=10), charged=True)
    mark(k)
    k = "charged_slit_64x64x130_multigrid_f32s"
    out[k] = lattice_config(P, slit, "f32s", steps, warmup,
                            dict(method="multigrid", rel_tol=1e-8, max_sweeps=100000, warm_start="extrapolated"),
                            charged=True)
    mark(k)
    del slit
    big = WL.charged_slit(nx=128, ny=128, nz=258, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    for st in ("f16s", "f32s"):
        k = f"charged_slit_128x128x258_direct_{st}"
        out[k] = lattice_config(P, big, st, steps, warmup, dict(method="direct"), charged=True)
        mark(k)
    del big
    ch = WL.batched_channels()
    for st in ("f32s", "f16s"):
        k = f"channels_64x32x32xW_direct_{st}"
        out[k] = lattice_config(P, ch, st, steps, warmup, dict(method="direct"), charged=True)
        out[k]["fluid_nodes"] = sum(ch.widths) * ch.nx * ch.ny
        mark(k)
    # the stated fallback of the batched form: multigrid to 1e-8 (the channel form: lateral
    # coarsening, z-line relaxation), extrapolated warm start
    k = "channels_64x32x32xW_multigrid_f32s"
    out[k] = lattice_config(P, ch, "f32s", steps, max(warmup, 20),
                            dict(method="multigrid", rel_tol=1e-8, max_sweeps=1000, warm_start="extrapolated"),
                            charged=True)
    mark(k)
    del ch
    w = WL.binary_multimode(n=512, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=100.0, seed=4)
    for st in ("f16s", "bf16s", "f32s"):
        k = f"binary_512cubed_{st}"
        out[k] = lattice_config(P, w, st, steps, warmup)
        mark(k)
    del w
    torch.cuda.empty_cache()
    return out


DTYPE = {"f64": "f64", "f32": "f32", "f32s": "f32", "f16s": "f16", "bf16s": "bf16"}


def bench_slit(args):
    """The charged ternary slit: 64 x 64 x 130 (walls z = 0, 129), solvent + cation + anion,
    lambda_D = 8, sigma = -1e-4 per wall, E_x = 1e-4, Sc = 100, Poisson to 1e-8 every step;
    with --size large the precision configuration's slit, 128 x 128 x 258.
    Prints its own JSON line (step time with and without the Poisson solve, solver work)."""
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    nxy, nz = (128, 258) if args.size == "large" else (64, 130)
    w = WL.charged_slit(nx=nxy, ny=nxy, nz=nz, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4,
                        sc=100.0)
    stream = torch.cuda.current_stream()
    out = {"workload": f"charged ternary slit {nxy}x{nxy}x{nz} (fluid {nxy}x{nxy}x{nz - 2}), Sc=100, lambda_D=8, "
                       "sigma=-1e-4, E_x=1e-4, Poisson rel. residual 1e-8 per step",
           "storage": args.storage}
    lat = P.from_workload(w, storage=args.storage, stream=stream,
                          poisson=dict(rel_tol=1e-8, max_sweeps=1000000, check_every=args.check_every,
                                       method=args.poisson, warm_start=args.warm_start))
    out["launch"] = lat.autotune(reps=3) if args.autotune else None
    out["graph"] = bool(args.graph)
    if args.graph:
        lat.set_step_graph(True)
    t0 = time.perf_counter()
    lat.step(args.warmup)
    torch.cuda.synchronize()
    out["warmup_s"] = round(time.perf_counter() - t0, 3)
    st0 = lat.stats()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    lat.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    st1 = lat.stats()
    sites = 3 * nxy * nxy * (nz - 2)
    out.update({"ms_per_step": round(ms, 4), "glups": round(sites / (ms * 1e-3) / 1e9, 4),
                "poisson_work_per_step": round((st1["total_sweeps"] - st0["total_sweeps"]) / args.steps, 2),
                "poisson_method": args.poisson, "warm_start": args.warm_start,
                "last_residual": st1["last_residual"]})
    print(json.dumps(out), flush=True)


def bench_channels(args):
    """The batched charged channels: 64 slit channels of 32 x 32 x W (W ~ U{32..256}, seed 5,
    9.2 M fluid nodes), wall charges ~ -U[1e-4, 1e-3], Sc 10 / 100 / 1000, lambda_D = 8,
    E_x = 1e-4, one fused stream-collide launch for all channels plus the Poisson solve of
    every channel each step.  Prints its own JSON line."""
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    w = WL.batched_channels()
    stream = torch.cuda.current_stream()
    lat = P.from_workload(w, storage=args.storage, stream=stream,
                          poisson=dict(rel_tol=1e-8, max_sweeps=1000000, check_every=args.check_every,
                                       method=args.poisson))
    shape = lat.autotune(reps=3) if args.autotune else None
    if args.graph:
        lat.set_step_graph(True)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    st0 = lat.stats()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    lat.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    st1 = lat.stats()
    nodes = sum(w.widths) * w.nx * w.ny
    sites = w.nspecies * nodes
    print(json.dumps({"workload": f"{len(w.widths)} charged slit channels {w.nx}x{w.ny}xW, W in "
                                  f"{min(w.widths)}..{max(w.widths)} (seed 5), {nodes} fluid nodes, Sc 10/100/1000",
                      "storage": args.storage, "poisson_method": args.poisson, "launch": shape, "graph": args.graph,
                      "ms_per_step": round(ms, 4), "glups": round(sites / (ms * 1e-3) / 1e9, 3),
                      "poisson_work_per_step": round((st1["total_sweeps"] - st0["total_sweeps"]) / args.steps, 2),
                      "last_residual": st1["last_residual"]}), flush=True)


def bench_warmstart(args):
    """Learned warm start on the charged ternary slit 64 x 64 x 130 (f32s): train the network
    (5 -> 16 -> 16 -> 16 -> 1, 3 x 3 x 3, BF16 operands with FP32 accumulation; inputs: the
    residual of the extrapolated guess, its coarse-grid solution, two potential increments and
    the wall mask) for --train-steps steps on exact corrections of the extrapolated guess, then
    time multigrid and red-black SOR to 1e-8 per step from the previous potential, the
    extrapolation and the learned guess (the direct solve alongside).  Prints one JSON line."""
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    stream = torch.cuda.current_stream()
    net = P.Net(5, 16, 4, seed=1)
    lat = P.from_workload(w, storage=args.storage, stream=stream, poisson=dict(method="direct"))
    lat.step(200)   # train on developed dynamics, not on the first transient
    t0 = time.perf_counter()
    losses = lat.train_warm_start(net, args.train_steps, lr=1e-3)
    torch.cuda.synchronize()
    out = {"workload": "charged ternary slit 64x64x130, Sc=100, lambda_D=8, multigrid to rel. residual 1e-8",
           "storage": args.storage, "network": "5-16-16-16-1, 3x3x3, BF16 operands, FP32 accumulate, %d parameters" % net.num_params,
           "train_steps": args.train_steps, "train_s": round(time.perf_counter() - t0, 2),
           "output_scale": net.output_scale(),
           "loss_first50": float(losses[3:53].mean()), "loss_last50": float(losses[-50:].mean())}
    for name, method, warm in [("direct", "direct", "previous"), ("previous", "multigrid", "previous"),
                               ("extrapolated", "multigrid", "extrapolated"), ("learned", "multigrid", "learned"),
                               ("sor previous", "sor", "previous"), ("sor extrapolated", "sor", "extrapolated"),
                               ("sor learned", "sor", "learned")]:
        lat = P.from_workload(w, storage=args.storage, stream=stream,
                              poisson=dict(method=method, rel_tol=1e-8, max_sweeps=100000))
        if warm == "learned":
            lat.set_warm_start_net(net)
        lat.set_poisson(method=method, rel_tol=1e-8, max_sweeps=100000, warm_start=warm)
        lat.step(max(args.warmup, 200))   # the developed dynamics the network was trained on
        torch.cuda.synchronize()
        st0 = lat.stats()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        lat.step(args.steps)
        end.record(stream)
        torch.cuda.synchronize()
        st1 = lat.stats()
        out[name] = {"ms_per_step": round(start.elapsed_time(end) / args.steps, 4),
                     "cycles_per_step": round((st1["total_sweeps"] - st0["total_sweeps"]) / args.steps, 3),
                     "last_residual": st1["last_residual"]}
        print(f"{name} done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def bench_precision_large(args):
    """Transport coefficients at the precision configuration's full size: 512^3 periodic
    binary, multimode noise (8 modes, seed 4) and shear wave, Sc 100.  D from the decay of
    concentration mode m = 7 (wavenumber 2 pi 7 / 512 along x, which the shear flow u_y(x)
    does not advect), nu from the shear wave u_y(x), each storage form against FP64 storage
    over the same steps: 200 to --steps (4000 unless --steps is above 200)."""
    import math

    import numpy as np
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    n = 512
    w = WL.binary_multimode(n=n, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=100.0, seed=4)
    ax = np.arange(n)
    km, kx = 2 * math.pi * 7 / n, 2 * math.pi / n
    t1 = 200
    t2 = args.steps if args.steps > t1 else 4000   # the window's end (--steps above 200, else 4000)
    out = {"workload": f"binary 512^3 multimode (seed 4), Sc 100; D from mode m=7 along x, nu from the shear "
                       f"wave; steps {t1}..{t2}"}

    def amps(lat):
        n0, j0 = lat.moments(0)
        _, j1 = lat.moments(1)
        c = np.cos(km * ax)[None, None, :]
        sn = np.sin(km * ax)[None, None, :]
        dn = n0 - 0.5
        a_m = math.hypot(float((dn * c).sum()), float((dn * sn).sum()))
        a_s = float(((j0[1] + j1[1]) * np.sin(kx * ax)[None, None, :]).sum())
        return a_m, a_s

    for st, sr in [("f64", None), ("f32s", None), ("f32s", True), ("f16s", True), ("bf16s", True), ("f32", None)]:
        lat = P.from_workload(w, storage=st, stochastic=sr, seed=7)
        lat.step(t1)
        a1 = amps(lat)
        lat.step(t2 - t1)
        a2 = amps(lat)
        del lat
        torch.cuda.empty_cache()
        key = st + ("" if sr is None else " SR")
        out[f"D {key}"] = -math.log(a2[0] / a1[0]) / (t2 - t1) / km ** 2 if a2[0] > 0 and a1[0] > 0 else None
        out[f"nu {key}"] = -math.log(a2[1] / a1[1]) / (t2 - t1) / kx ** 2
        print(f"{key} done", file=sys.stderr, flush=True)
    for key in list(out):
        if key == "workload" or " f64" in key or out[key] is None:
            continue
        ref = out[key.split(" ")[0] + " f64"]
        out["err " + key] = out[key] / ref - 1.0 if ref else None
    print(json.dumps(out), flush=True)


def bench_electrokinetics(args):
    """The paper's charged-slit experiment (Sec. IV) at full size: 64 x 64 x 130, solvent +
    cation + anion, lambda_D = 8, sigma = -1e-4 per wall, E_x = 1e-4, Sc = 100, direct
    Poisson solve, `steps` steps from rest, each storage form.  Prints one JSON line: the
    electro-osmotic mobility u_centre / E_x against Helmholtz-Smoluchowski, the mass flow
    I_m and the electro-osmotic current I_eo against twice the paper's half-channel formulas
    (eqs. theomassflow, theo), the conductivity I / (E_x H) against its conduction part
    (D / v_T^2) sum (n+ + n-) / H plus I_eo / (E_x H), and the step time."""
    import math

    import numpy as np
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = WL.charged_slit(nx=64, ny=64, nz=130, n_ion=1e-3, debye_length=8.0, sigma=-1e-4, Ex=1e-4, sc=100.0)
    Ex, sigma, H = w.E[0], w.sigma[0], w.nz - 2
    nu = (w.tau_visc - 0.5) / 3.0
    kB = 4 * math.pi * w.bjerrum
    kd = 1.0 / 8.0
    out = {"workload": "charged ternary slit 64x64x130 (fluid 64x64x128), lambda_D=8, sigma=-1e-4, E_x=1e-4, "
                       "Sc=100, direct Poisson solve, from rest", "steps": args.steps}
    for name in args.storage.split(","):
        # storage[:sr][:narrow]: stochastic rounding of an FP32 form; FP32 collision arithmetic
        st, *flags = name.split(":")
        sr = True if "sr" in flags else None
        lat = P.from_workload(w, storage=st, stream=stream, stochastic=sr, poisson=dict(method="direct"),
                              wide="narrow" not in flags)
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        lat.step(args.steps)
        s1.record(stream)
        torch.cuda.synchronize()
        pr = lat.zprofiles()
        psi = lat.potential().mean(axis=(1, 2))
        lat.step(1)
        pr = (0.5 * (pr + lat.zprofiles()))[:, :, 1:-1]
        psi = (0.5 * (psi + lat.potential().mean(axis=(1, 2))))[1:-1]
        n = pr[:, 0]
        rho = n.sum(0)
        ux = pr[:, 1].sum(0) / rho
        hs = Ex * (psi - (psi[0] + 0.5 * kB * sigma)) / (kB * nu * rho)
        c = lambda v: 0.5 * (v[H // 2 - 1] + v[H // 2])
        Im = float((rho * ux).sum())
        Im_th = 2 * (Ex * sigma / nu) / kd ** 2 * (1 - (kd * H / 2) / math.tanh(kd * H / 2))
        Ieo = float(((n[1] - n[2]) * ux).sum())
        eta = nu * rho.mean()
        Ieo_th = -2 * (Ex * sigma ** 2 / (eta * kd * math.tanh(kd * H / 2) ** 2)) * (
            (math.sinh(kd * H) + kd * H) / (4 * math.cosh(kd * H / 2) ** 2)
            - math.sinh(kd * H / 2) / math.cosh(kd * H / 2))
        I = float((pr[1, 1] - pr[2, 1]).sum())
        tau_d = 1.0 / w.omega_drag
        cond = (tau_d - 0.5) * float((n[1] + n[2]).sum()) * Ex
        out[name] = {"ms_per_step": round(s0.elapsed_time(s1) / args.steps, 4),
                   "mobility": c(ux) / Ex, "mobility_hs": c(hs) / Ex, "err_mobility_vs_hs": c(ux) / c(hs) - 1,
                   "I_m": Im, "I_m_paper": Im_th, "err_I_m": Im / Im_th - 1,
                   "I_eo": Ieo, "I_eo_paper": Ieo_th, "err_I_eo": Ieo / Ieo_th - 1,
                   "conductivity": I / (Ex * H), "conduction_plus_convection": (cond + Ieo) / (Ex * H),
                   "err_conductivity": I / (cond + Ieo) - 1, "ohmic_over_eo": (I - Ieo) / Ieo,
                   "mass_drift": [float(v) for v in lat.mass_totals() / np.array([a.sum() for a in w.n]) - 1]}
        del lat
        print(f"{name} done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """Transport coefficients with every storage form against FP64 storage: the mutual
    diffusivity D from a decaying concentration wave (Sc 10 and 100; D = v_T^2 (1/omega_drag
    - 1/2)), the viscosity nu from a shear wave (nu = v_T^2 (1/omega_visc - 1/2)), and the
    electro-osmotic mobility u_centre / E_x of a charged 16 x 16 x 32 slit at Sc 100 (steady
    state, time-averaged).  Prints one JSON line of values and relative errors."""
    import math

    import numpy as np
    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    L = 128
    k = 2 * math.pi / L
    basis = np.sin(k * np.arange(L))[None, None, :]
    # (storage, stochastic rounding, density deviation carried in FP64); "narrow": FP32
    # collision arithmetic throughout
    forms = [("f64", None, True), ("f32", None, True), ("f32s", None, True), ("f32s", None, False),
             ("f32s", True, True), ("f16s", True, True), ("f16s", True, False), ("f16s", False, True),
             ("bf16s", True, True), ("bf16s", True, False)]
    name = lambda st, sr, wd=True: st + ("" if sr is None else (" SR" if sr else " RNE")) + ("" if wd else " narrow")
    out = {"workload": "D: binary sine 128x64x64 (amp 1e-3); nu: shear wave 128x64x64, tau 0.8; "
                       "mobility: charged slit 16x16x34, lambda_D 4, sigma -1e-4, E_x 1e-5, Sc 100"}
    def diffusivity(w, st, sr, wd, seed, t1, t2):
        lat = P.from_workload(w, storage=st, stochastic=sr, seed=seed, wide=wd)
        lat.step(t1)
        a1 = float(((lat.moments(0)[0] - 0.5) * basis).sum())
        lat.step(t2 - t1)
        a2 = float(((lat.moments(0)[0] - 0.5) * basis).sum())
        return -math.log(a2 / a1) / (t2 - t1) / k ** 2 if a2 / a1 > 0 else None

    def mobility(w, st, sr, wd, seed):
        lat = P.from_workload(w, storage=st, stochastic=sr, seed=seed, poisson=dict(method="direct"), wide=wd)
        lat.step(28000)
        acc = None
        for _ in range(20):
            lat.step(100)
            pr = lat.zprofiles()
            acc = pr if acc is None else acc + pr
        pr = acc / 20
        rho = pr[:, 0, 1:-1].sum(0)
        return float(pr[:, 1, 1:-1].sum(0)[16] / rho[16] / 1e-5)

    sine = {}
    for sc, t1, t2 in [(10.0, 300, 6300), (100.0, 2000, 22000)]:
        sine[sc] = WL.binary_sine(L, 64, 64, amp=1e-3, tau_visc=1.0, sc=sc), t1, t2
        for st, sr, wd in forms:
            out[f"D Sc={sc:g} {name(st, sr, wd)}"] = diffusivity(sine[sc][0], st, sr, wd, 7, t1, t2)
            print(f"D Sc={sc:g} {name(st, sr, wd)} done", file=sys.stderr, flush=True)
    shape = (64, 64, L)
    u = np.zeros((3,) + shape)
    u[1] = 1e-3 * basis
    w = WL.Workload("shear", L, 64, 64, "periodic", [0.5, 0.5], [0, 0], 0.8, WL.tau_drag_for_schmidt(0.8, 100.0),
                    [np.full(shape, 0.5)] * 2, [u, u])
    for st, sr, wd in forms:
        lat = P.from_workload(w, storage=st, stochastic=sr, seed=7, wide=wd)
        amp = lambda: sum(float((lat.moments(q)[1][1] * basis).sum()) for q in range(2))
        lat.step(100)
        a1 = amp()
        lat.step(3000)
        out[f"nu {name(st, sr, wd)}"] = -math.log(amp() / a1) / 3000 / k ** 2
        del lat
    slit = WL.charged_slit(nx=16, ny=16, nz=34, n_ion=1e-3, debye_length=4.0, sigma=-1e-4, Ex=1e-5, sc=100.0)
    for st, sr, wd in forms:
        out[f"mobility {name(st, sr, wd)}"] = mobility(slit, st, sr, wd, 7)
        print(f"mobility {name(st, sr, wd)} done", file=sys.stderr, flush=True)
    # spread over rounding streams of the stochastically rounded 16-bit forms: relative errors
    # against FP64 for 8 seeds, their mean and sample standard deviation
    seeds = list(range(7, 15))
    w, t1, t2 = sine[100.0]
    for st in ("f16s", "bf16s"):
        errs = {"D Sc=100": [diffusivity(w, st, True, True, s, t1, t2) / out["D Sc=100 f64"] - 1 for s in seeds],
                "mobility": [mobility(slit, st, True, True, s) / out["mobility f64"] - 1 for s in seeds]}
        for q, e in errs.items():
            out[f"streams {q} {st} SR"] = {"seeds": seeds, "err": e, "mean": float(np.mean(e)),
                                           "std": float(np.std(e, ddof=1))}
        print(f"streams {st} done", file=sys.stderr, flush=True)
    for key in list(out):
        if key == "workload" or " f64" in key or key.startswith("streams") or out[key] is None:
            continue
        ref = out[key.split(" ")[0] + (" " + key.split(" ")[1] if key.startswith("D") else "") + " f64"]
        out["err " + key] = out[key] / ref - 1.0
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--storage", default="f32s",
                    help="f32s (FP32 deviations from rest, the default), f32, f16s, bf16s, f64")
    ap.add_argument("--sc", type=float, default=100.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (slits, channels, 512^3)")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--config-steps", type=int, default=50, help="timed steps of each other configuration")
    ap.add_argument("--config-warmup", type=int, default=10)
    ap.add_argument("--graph", action="store_true", help="replay steps as captured HIP graphs")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library pick the work-group shape of the step (default: its default shape)")
    ap.add_argument("--workload", default="binary",
                    choices=["binary", "slit", "channels", "precision", "warmstart", "electrokinetics"],
                    help="binary: the 256^3 throughput benchmark (default); slit: the charged slit; "
                         "channels: 64 charged slit channels in one lattice")
    ap.add_argument("--poisson", default="sor", choices=["sor", "multigrid", "direct"])
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--train-steps", type=int, default=300, help="training steps of the warm-start network")
    ap.add_argument("--size", default="small", choices=["small", "large"],
                    help="precision workload: small lattices (default) or the 512^3 configuration; "
                         "slit workload: 64x64x130 (default) or 128x128x258")
    ap.add_argument("--warm-start", default="previous", choices=["previous", "extrapolated"])
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (3 times), the reference "
                         "kernel for scaling HBM counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the lattice would be "
              "split into slabs with halo exchange; not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "slit":
        bench_slit(args)
        return
    if args.workload == "channels":
        bench_channels(args)
        return
    if args.workload == "precision":
        if args.size == "large":
            bench_precision_large(args)
        else:
            bench_precision(args)
        return
    if args.workload == "warmstart":
        bench_warmstart(args)
        return
    if args.workload == "electrokinetics":
        bench_electrokinetics(args)
        return

    import torch

    import paper_1507_04891_amd as P
    import workloads as WL

    torch.cuda.set_device(0)
    w = WL.binary_multimode(n=args.n, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=args.sc, seed=2)
    head = time_storage(P, w, args.storage, args.steps, args.warmup, autotune=args.autotune)
    out = {
        "metric": "species-site updates/s (GLUPS), %HBM peak",
        "value": round(head["glups"], 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": f"neutral binary D3Q19 {args.n}^3 periodic, {args.storage} populations, "
                               f"Sc={args.sc:g}, tau_visc=1, multimode noise + shear wave (seed 2)",
                   "species": 2, "lattice": [args.n] * 3, "storage": args.storage, "schmidt": args.sc,
                   "launch": head["launch"], "timing": f"median per-step time of {WINDOWS} windows over "
                                                       f"the {args.steps} timed steps"},
        "window_ms_per_step": head["window_ms"],
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["frac"], 4),
                     "traffic": traffic_from_profile(args.storage, args.n)},
    }
    if not args.no_variants:
        var = {}
        for st in ("f32", "f16s", "bf16s"):
            if st == args.storage:
                continue
            r = time_storage(P, w, st, args.steps, args.warmup, autotune=args.autotune)
            var[st] = {"glups": round(r["glups"], 3), "ms_per_step": round(r["ms_per_step"], 5),
                       "window_ms_per_step": r["window_ms"], "hbm_frac": round(r["frac"], 4),
                       "speedup_vs_headline": round(r["glups"] / head["glups"], 3), "launch": r["launch"]}
        # shifted FP32 with stochastically rounded stores
        r = time_storage(P, w, "f32s", args.steps, args.warmup, autotune=args.autotune, stochastic=True)
        var["f32s_stochastic"] = {"glups": round(r["glups"], 3), "ms_per_step": round(r["ms_per_step"], 5),
                                  "window_ms_per_step": r["window_ms"], "hbm_frac": round(r["frac"], 4),
                                  "speedup_vs_headline": round(r["glups"] / head["glups"], 3), "launch": r["launch"]}
        out["variants"] = var
    if not args.no_copy_ceiling:
        cc = copy_ceiling()
        cc["headline_frac_of_copy"] = round(head["achieved_gbs"] / cc["gbs"], 4)
        out["roofline"]["copy_ceiling"] = cc
    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 2 ** 30)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
        del src, dst
    if not args.no_configs:
        del w
        torch.cuda.empty_cache()
        out["configs"] = bench_configs(P, WL, args.config_steps, args.config_warmup)
        w = WL.binary_multimode(n=args.n, amp=1e-3, nmodes=8, shear=1e-3, tau_visc=1.0, sc=args.sc, seed=2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.sc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
