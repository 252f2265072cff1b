"""Benchmark of the fused RLBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the metric's FP32-vs-FP64 configuration): 512 x 512 periodic
lattice, spherical 26-direction stencil, tau = 0.55, eps = 1 and
beta ~ N(0, 0.005^2) per component (seed 1), stirring force on the shell
|k| in [4, 6] with amplitude 1e-5 redrawn every step from Philox (seed 2).
A step is the whole hot path: force table + fused stream / moments / FP64
Landau / equilibrium / collision / force / store.  Inputs are resident in
HBM before timing starts.

The headline value is the FP32-population step in MLUPS.  The same line
carries the FP64, F16S and BF16S forms of the step (MLUPS, kernel GB/s and
their field error against the FP64 path after the same steps), the z-folded
stencil (17 stored populations, exact for the one-layer lattice) in F32 and
F16S, the same kernels on HBM-resident lattices (2048^2 and 8192^2) and on
the 256-lattice ensemble, a plain device copy of one 2048^2 step's bytes (the
practical streaming rate), the roofline of the FP32 step kernel (per-launch
duration from HIP events around every launch; HBM traffic from the committed
rocprofv3 counter summary when it matches the kernel sources) and the FP64
NumPy oracle timed on the host cores for a bounded sample.  Every form is
timed in the kernel form the library's autotuner picks on a scratch lattice
of the same configuration.  Kernel GB/s are algorithmic bytes (2 Q s per site
and step) per launch over the launch's duration; a two-step launch counts both
steps' bytes and moves about half of them through HBM (the committed traffic
counters show it).
Everything except the JSON line goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
Q = 26
BYTES = {"F64": 8, "F32": 4, "F16S": 2, "BF16S": 2}
STEPS_PER_LAUNCH = {"march2": 2}         # kernel forms that advance more than one step per launch
METRIC = "MLUPS + HBM GB/s (% peak): FP32/FP16-storage vs FP64 step at stated field error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources the step kernel is built from (for counter data)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_06187_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(tag="forced512_F32", kind=None):
    """HBM bytes per launch of the step kernel on a workload, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on
    the current kernel sources and (when kind is given) on the same kernel
    form (tile / staged / march / march2); else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sha, val = None, None
    for line in open(path):
        f = line.split()
        if len(f) == 2 and f[0] == "kernel_src_sha":
            sha = f[1]
        elif len(f) >= 3 and f[0] == tag and f[1] == "traffic_bytes_per_launch":
            form = f[3].split(":")[0] if len(f) >= 4 else None
            if kind is None or form is None or form == kind:
                val = int(f[2])
    if sha != kernel_source_hash():
        return None
    return val


def make_lattice(rl, wl, storage, torch, stencil="SPH26"):
    import workloads
    A, klo, khi, fseed = wl.forcing
    lat = rl.Lattice(wl.n, wl.n, wl.tau, stencil=stencil, storage=storage,
                     forcing=rl.Forcing(A, klo, khi, fseed))
    e, bx, by = workloads.initial_fields(wl)
    dev = lambda a: torch.from_numpy(a).to("cuda:0")  # noqa: E731
    lat.set_state(dev(e), dev(bx), dev(by))
    del e, bx, by
    return lat


def time_steps(lat, torch, steps, warmup, chunk):
    lat.set_graph_chunk(chunk)
    lat.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    lat.step(steps)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def field_error(a, b):
    """Normwise error of fields a against reference b (eps; beta as a vector)."""
    ea, xa, ya, _ = [t.cpu().numpy() for t in a]
    eb, xb, yb, _ = [t.cpu().numpy() for t in b]
    vmax = max(np.abs(xb).max(), np.abs(yb).max())
    return {"eps": float(np.abs(ea - eb).max() / np.abs(eb).max()),
            "beta": float(max(np.abs(xa - xb).max(), np.abs(ya - yb).max()) / vmax)}


def tune_form(rl, wl, storage, torch, stencil, tune_steps):
    """The library's autotuner run on a scratch lattice of the same
    configuration; returns the kernel form it keeps."""
    scratch = make_lattice(rl, wl, storage, torch, stencil)
    form = scratch.autotune(tune_steps)
    scratch.close()
    del scratch
    torch.cuda.empty_cache()
    return form


def run_form(rl, torch, wl, storage, steps, warmup, chunk, prof_n, stencil="SPH26",
             tune_steps=0, form=None):
    tuned = form is None and tune_steps > 0
    if tuned:
        form = tune_form(rl, wl, storage, torch, stencil, tune_steps)
    lat = make_lattice(rl, wl, storage, torch, stencil)
    if form is not None:
        lat.set_kernel(*form)
    ms = time_steps(lat, torch, steps, warmup, chunk)
    kind = lat.kernel()
    spl = STEPS_PER_LAUNCH.get(kind[0], 1)          # the two-step form advances 2 per launch
    n_prof = max(1, prof_n // spl)                  # the same number of steps for every form
    kms = lat.profile_step_kernel(n_prof)
    sites = wl.n * wl.n
    algo = 2 * lat.Q * BYTES[storage] * sites
    out = {
        "storage": storage,
        "stencil": stencil,
        "ms_per_step": ms,
        "mlups": sites / (ms * 1e-3) / 1e6,
        "kernel_ms": kms,
        "steps_per_launch": spl,
        "kernel_gbs": spl * algo / (kms * 1e-3) / 1e9,
        "step_gbs": algo / (ms * 1e-3) / 1e9,
        "steps_done": warmup + steps + n_prof * spl,
    }
    out["kernel_frac_hbm_peak"] = out["kernel_gbs"] / HBM_PEAK_GBS
    out["kernel_form"] = list(kind)
    out["autotuned"] = tuned
    return lat, out


def run_ensemble(rl, torch, steps, warmup, chunk=20):
    """The 256-lattice ensemble (sides from {64, 128, 256}, tau in [0.51, 0.8]),
    FP32 populations, one persistent launch per step, graph replay; the
    library's autotuner picks the kernel form and shape first."""
    import workloads
    spec = workloads.ensemble()
    sizes = [(n, n) for n, _ in spec]
    taus = [t for _, t in spec]
    frs = [rl.Forcing(1e-5, 2.0, 4.0, r) for r in range(len(spec))]
    ens = rl.Ensemble(sizes, taus, storage="F32", forcings=frs)
    for r, (n, _) in enumerate(spec):
        e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=r)
        ens.set_state(r, *(torch.from_numpy(a).to("cuda:0") for a in (e, bx, by)))
    form = ens.autotune(10)
    ens.set_graph_chunk(chunk)
    ens.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    ens.step(steps)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    sites = sum(n * n for n, _ in spec)
    out = {"realizations": len(spec), "sites": sites, "ms_per_step": ms,
           "mlups": sites / (ms * 1e-3) / 1e6,
           "step_gbs": 2 * Q * BYTES["F32"] * sites / (ms * 1e-3) / 1e9,
           "unstable": ens.check() != rl.OK, "kernel_form": list(form)}
    ens.close()
    return out


def copy_ceiling(torch, nbytes, reps=20):
    """Device-to-device copy of nbytes (torch's copy: the runtime's copy
    kernel), back to back: read + write bytes per second, the practical
    streaming rate of the machine's HBM for a buffer of that size."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        (b if i % 2 == 0 else a).copy_(a if i % 2 == 0 else b)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_each_way": 4 * n, "ms": ms, "gbs": 2 * 4 * n / (ms * 1e-3) / 1e9}


def cpu_baseline(wl, n_steps):
    """The FP64 oracle on the same workload, single thread, a few steps."""
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import rlbm as orlbm
    from oracle import stencil as ostencil
    st = ostencil.sph26()
    A, klo, khi, fseed = wl.forcing
    force = dict(amplitude=A, k_lo=klo, k_hi=khi, seed=fseed)
    e, bx, by = workloads.initial_fields(wl)
    with threadpool_limits(limits=1):
        F = orlbm.set_state(e, bx, by, st)
        t = time.perf_counter()
        for s in range(n_steps):
            F = orlbm.step(F, st, wl.tau, 1.0, force, s)
        dt = time.perf_counter() - t
    return {"value": wl.n * wl.n * n_steps / dt / 1e6, "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_steps} steps of the {wl.n}x{wl.n} forced workload, FP64 NumPy "
                      f"oracle on one host core ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the HBM-resident 2048^2 / 8192^2 lines")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--tune-steps", type=int, default=None,
                    help="steps per candidate of the library's autotuner, run on a scratch "
                         "lattice before each form is timed (scaled down as 512/n on the "
                         "larger lattices, at least 16; 0: the library's default form). "
                         "Default 40, and 0 with --only")
    ap.add_argument("--form", default=None, metavar="KIND:PARAM",
                    help="with --only: time this kernel form (e.g. march:22 or tile:4)")
    ap.add_argument("--only", default=None, metavar="WORKLOAD:STORAGE[:STENCIL]",
                    help="time one form only (e.g. forced2048:F32 or "
                         "forced2048:F32:SPH26_ZFOLD), for profiler runs")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run a plain device copy of this many bytes 3 times "
                         "(counter calibration under rocprofv3 --pmc)")
    a = ap.parse_args()
    if a.tune_steps is None:
        a.tune_steps = 0 if a.only else 40
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(a lattice would be split into row slabs, one per GPU); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2101_06187_amd as rl
    import workloads

    rl.lib()
    log("device:", torch.cuda.get_device_name(0))
    if a.copy_bytes:
        n = a.copy_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy: 3 x {4 * n} bytes")
        del src, dst
    if a.only:
        name, storage, *st = a.only.split(":")
        w = workloads.WORKLOADS[name]
        form = None
        if a.form:
            kind, param = a.form.split(":")
            form = (kind, int(param))
        tune = a.tune_steps or 0
        lat, r = run_form(rl, torch, w, storage, a.steps, a.warmup, 50, min(a.steps, 200),
                          st[0] if st else "SPH26",
                          tune_steps=max(16, tune * 512 // w.n) if tune else 0, form=form)
        r["unstable"] = lat.check() != rl.OK
        log(f"{name} {storage}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_ms'] * 1e3:.2f} us "
            f"= {r['kernel_gbs']:.0f} GB/s")
        print(json.dumps({"only": a.only, **r}), flush=True)
        return
    wl = workloads.WORKLOADS["forced512"]
    chunk = 50

    forms = {}
    lats = {}
    for storage in ("F32", "F64", "F16S", "BF16S"):
        lat, r = run_form(rl, torch, wl, storage, a.steps, a.warmup, chunk, 500,
                          tune_steps=a.tune_steps)
        lats[storage] = lat
        forms[storage] = r
        log(f"{storage}: {r['mlups']:.0f} MLUPS, {r['ms_per_step'] * 1e3:.2f} us/step, "
            f"kernel {r['kernel_ms'] * 1e3:.2f} us = {r['kernel_gbs']:.0f} GB/s")
    ref = lats["F64"].fields()
    for storage in ("F32", "F16S", "BF16S"):
        forms[storage]["field_error_vs_f64"] = field_error(lats[storage].fields(), ref)
        log(storage, "field error vs F64 path:", forms[storage]["field_error_vs_f64"])
    for storage in ("F32", "F64", "F16S", "BF16S"):
        forms[storage]["unstable"] = lats[storage].check() != rl.OK
        lats[storage].close()
    del lats
    torch.cuda.empty_cache()

    # The z-folded stencil (17 stored populations, exact for the one-layer
    # lattice): same workload, same step, fewer bytes per site.
    for storage in ("F32", "F16S"):
        key = storage + "_ZFOLD"
        lat, r = run_form(rl, torch, wl, storage, a.steps, a.warmup, chunk, 500, "SPH26_ZFOLD",
                          tune_steps=a.tune_steps)
        r["field_error_vs_f64"] = field_error(lat.fields(), ref)
        r["unstable"] = lat.check() != rl.OK
        lat.close()
        forms[key] = r
        log(f"{key}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_ms'] * 1e3:.2f} us = "
            f"{r['kernel_gbs']:.0f} GB/s, field error vs F64 {r['field_error_vs_f64']}")
    del ref
    torch.cuda.empty_cache()

    extra = {}
    if not a.no_extra:
        for name, storages, steps in (
                ("forced2048", ("F32", "F16S", "BF16S", "F32_ZFOLD", "F16S_ZFOLD"), 300),
                ("forced8192", ("F32", "F16S", "F32_ZFOLD", "F16S_ZFOLD"), 60)):
            w = workloads.WORKLOADS[name]
            extra[name] = {}
            for key in storages:
                storage, _, fold = key.partition("_")
                lat, r = run_form(rl, torch, w, storage, steps, 20, 20, 20,
                                  "SPH26_ZFOLD" if fold else "SPH26",
                                  tune_steps=max(16, a.tune_steps * 512 // w.n)
                                  if a.tune_steps else 0)
                r["unstable"] = lat.check() != rl.OK
                lat.close()
                del lat
                torch.cuda.empty_cache()
                extra[name][key] = {k: r[k] for k in ("mlups", "ms_per_step", "kernel_ms",
                                                      "steps_per_launch", "kernel_gbs",
                                                      "kernel_frac_hbm_peak", "unstable",
                                                      "kernel_form")}
                extra[name][key]["traffic_bytes_per_launch"] = committed_traffic(
                    f"{name}_{storage}" + ("_SPH26_ZFOLD" if fold else ""), r["kernel_form"][0])
                log(f"{name} {key}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_gbs']:.0f} GB/s "
                    f"({100 * r['kernel_frac_hbm_peak']:.1f}% of HBM peak)")

    if not a.no_extra:
        # the same bytes as one FP32 step of the 2048^2 lattice (read + write 436 MB)
        extra["copy_2048_f32_bytes"] = copy_ceiling(torch, 2048 * 2048 * Q * 4)
        log(f"device copy of 436 MB: {extra['copy_2048_f32_bytes']['gbs']:.0f} GB/s "
            f"({100 * extra['copy_2048_f32_bytes']['gbs'] / HBM_PEAK_GBS:.1f}% of HBM peak)")
        extra["ensemble256"] = run_ensemble(rl, torch, 200, 20)
        torch.cuda.empty_cache()
        log(f"ensemble256 F32: {extra['ensemble256']['mlups']:.0f} MLUPS, "
            f"{extra['ensemble256']['step_gbs']:.0f} GB/s per step")

    head = forms["F32"]
    sites = wl.n * wl.n
    per_launch = head["steps_per_launch"] * 2 * Q * BYTES["F32"] * sites
    traffic = committed_traffic("forced512_F32", head["kernel_form"][0])
    roofline = {"bound": "hbm", "achieved": head["kernel_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": head["kernel_gbs"] / HBM_PEAK_GBS,
                "traffic": traffic,
                "kernel": ("rlbm::%s<StF32, Sph26, unit cfl, forced>"
                           % {"tile": "step_kernel", "staged": "staged_kernel",
                              "march": "march_kernel", "march2": "march2_kernel",
                              "march_pairs": "march_pair_kernel"}[
                               head["kernel_form"][0]]),
                "kernel_form": head["kernel_form"],
                "algorithmic_bytes_per_launch": per_launch,
                "kernel_ms": head["kernel_ms"]}

    cpu = None if a.no_cpu_baseline else cpu_baseline(wl, a.cpu_steps)
    if cpu:
        log("cpu baseline:", cpu)

    line = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "forced512: 512x512 periodic, SPH26 stencil, tau 0.55, "
                               "beta~N(0,0.005^2) seed 1, force shell |k| in [4,6] "
                               "amplitude 1e-5 Philox seed 2, FP32 populations",
                   "lattice": [wl.n, wl.n], "storage": "F32", "parallelism": "single GPU",
                   "graph_chunk": chunk},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "hbm_resident": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
