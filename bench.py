"""Benchmark of the fused RLBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra]

Headline workload (the largest single-GPU configuration): 8192 x 8192
periodic lattice, spherical 26-direction stencil, FP32 populations,
tau = 0.505, eps = 1 and beta ~ N(0, 0.002^2) per component (seed 3),
stirring force on the shell |k| in [32, 40] (910 modes) with amplitude 2e-6
redrawn every step from Philox (seed 2).  A step is the whole hot path (force
tables + fused stream / moments / FP64 Landau / equilibrium / collision /
force / store, one launch per step or per two steps).  Inputs are resident
in HBM before timing starts; the lattice (14 GB of populations) is far larger
than the caches.

The JSON line carries, beside the headline:
  * "forms": every storage form on the same lattice (F64, F32, F16S, BF16S and
    the z-folded stencil) with MLUPS, kernel time per launch and its
    algorithmic bandwidth, the gain over the GPU FP64 step, and each form's
    per-field error (eps, beta, six T^{mu nu} planes) after 8 steps against
    the oracle's fields at 24 sampled sites (stored by
    tests/golden/make_field_windows.py) and after 200 steps against the GPU
    FP64 path on the whole lattice;
  * "forced2048": the same for the 2048^2 workload (HBM-resident too);
  * "forced512": the 512^2 workload, whose buffers fit the Infinity Cache
    (effective GB/s only, not an HBM figure);
  * "ensemble256": the 256-lattice ensemble in one persistent launch per step;
  * "insitu": the 8192^2 and 2048^2 FP32 runs with their in-situ diagnostics
    (energy spectrum and enstrophy every 500 / 1000 steps), MLUPS including
    the diagnostics;
  * "copy": the library's streaming copy of one FP32 step's bytes (the
    practical HBM ceiling) and torch's device copy;
  * "roofline": algorithmic bytes per launch of the step kernel the
    autotuner picked over its mean launch time (HIP events around every
    launch), the committed rocprofv3 traffic when it matches the sources;
  * "cpu_baseline": the FP64 NumPy oracle on one host core, one step of a
    64-row band of the headline lattice; "oracle_all_cores": ensemble
    realizations stepped by the oracle in a process pool.
Every GPU form is timed in the kernel form the library's autotuner picks on a
scratch lattice of the same configuration.  Everything except the JSON line
goes to stderr.
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
BYTES = {"F64": 8, "F32": 4, "F16S": 2, "BF16S": 2}
QS = {"SPH26": 26, "SPH26_ZFOLD": 17}
STEPS_PER_LAUNCH = {"march2": 2}         # kernel forms that advance more than one step per launch
METRIC = "MLUPS + HBM GB/s (% peak): FP32/FP16-storage vs FP64 step at stated field error"
KERNEL_NAMES = {"tile": "step_kernel", "staged": "staged_kernel", "march": "march_kernel",
                "march2": "march2_kernel", "march_pairs": "march_pair_kernel"}
FIELD_STEPS = 8                 # steps before the field error against the oracle
LONG_STEPS = 200                # steps before the field error against the GPU FP64 path
GOLDEN = os.path.join(ROOT, "tests", "golden", "field_windows.json")


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


def committed_traffic(tag="forced8192_F32", kind=None):
    """HBM bytes per launch of the step kernel on a workload, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on
    the current kernel sources and (when kind is given) on the same kernel
    form (tile / staged / march / march2 / march_pairs); else None."""
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


def tune_form(rl, wl, storage, torch, stencil, tune_steps):
    """The library's autotuner run on a scratch lattice of the same
    configuration; returns the kernel form it keeps."""
    scratch = make_lattice(rl, wl, storage, torch, stencil)
    form = scratch.autotune(tune_steps)
    scratch.close()
    del scratch
    torch.cuda.empty_cache()
    return form


def tune_steps_for(wl, tune_steps):
    return max(16, tune_steps * 512 // wl.n) if tune_steps else 0


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
        "algorithmic_bytes_per_launch": spl * algo,
        "kernel_gbs": spl * algo / (kms * 1e-3) / 1e9,
        "step_gbs": algo / (ms * 1e-3) / 1e9,
        "kernel_form": list(kind),
        "autotuned": tuned,
    }
    out["kernel_frac_hbm_peak"] = out["kernel_gbs"] / HBM_PEAK_GBS
    out["unstable"] = lat.check() != rl.OK
    return lat, out


def sampled_fields(lat, xs, ys):
    import torch
    e, bx, by, T = lat.fields()
    iy = torch.as_tensor(ys, device="cuda:0")
    ix = torch.as_tensor(xs, device="cuda:0")
    out = {"eps": e[iy, ix].cpu().numpy(), "beta_x": bx[iy, ix].cpu().numpy(),
           "beta_y": by[iy, ix].cpu().numpy()}
    for i, name in enumerate(("T00", "T0x", "T0y", "Txx", "Txy", "Tyy")):
        out[name] = T[i][iy, ix].cpu().numpy()
    return out


def field_errors(got, want):
    """Normwise per-field errors max |got - want| / max |want|; beta as a
    vector (both components over the largest |beta| component)."""
    out = {}
    for name in ("eps", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy"):
        w = np.asarray(want[name])
        out[name] = float(np.abs(np.asarray(got[name]) - w).max() / np.abs(w).max())
    wx, wy = np.asarray(want["beta_x"]), np.asarray(want["beta_y"])
    vmax = max(np.abs(wx).max(), np.abs(wy).max())
    out["beta"] = float(max(np.abs(np.asarray(got["beta_x"]) - wx).max(),
                            np.abs(np.asarray(got["beta_y"]) - wy).max()) / vmax)
    return out


def whole_fields(lat):
    """The library's fields of the whole lattice, as one dict of device tensors."""
    e, bx, by, T = lat.fields()
    out = {"eps": e, "beta_x": bx, "beta_y": by}
    for i, name in enumerate(("T00", "T0x", "T0y", "Txx", "Txy", "Tyy")):
        out[name] = T[i]
    return out


def whole_field_errors(got, ref):
    """field_errors on device tensors (whole lattice)."""
    out = {}
    for name in ("eps", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy"):
        out[name] = float((got[name] - ref[name]).abs().max() / ref[name].abs().max())
    vmax = float(max(ref["beta_x"].abs().max(), ref["beta_y"].abs().max()))
    out["beta"] = float(max((got["beta_x"] - ref["beta_x"]).abs().max(),
                            (got["beta_y"] - ref["beta_y"]).abs().max())) / vmax
    return out


def field_error_runs(rl, torch, wl, forms, golden):
    """Per storage form: fields after FIELD_STEPS steps against the oracle's
    stored fields at the golden sites, and after LONG_STEPS steps against the
    GPU FP64 path on the whole lattice (each form in its benchmark form)."""
    case = golden["workloads"].get(wl.name) if golden else None
    results = {}
    ref = make_lattice(rl, wl, "F64", torch)
    ref.set_kernel(*forms["F64"]["kernel_form"])
    ref.step(FIELD_STEPS)
    if case:
        results["F64"] = {"vs_oracle_after_%d" % FIELD_STEPS:
                          field_errors(sampled_fields(ref, case["x"], case["y"]), case["fields"])}
    ref.step(LONG_STEPS - FIELD_STEPS)
    ref_f = whole_fields(ref)
    ref.close()
    del ref
    torch.cuda.empty_cache()
    for key, r in forms.items():
        if key == "F64":
            continue
        lat = make_lattice(rl, wl, r["storage"], torch, r["stencil"])
        lat.set_kernel(*r["kernel_form"])
        lat.step(FIELD_STEPS)
        res = {}
        if case:
            res["vs_oracle_after_%d" % FIELD_STEPS] = field_errors(
                sampled_fields(lat, case["x"], case["y"]), case["fields"])
        lat.step(LONG_STEPS - FIELD_STEPS)
        got = whole_fields(lat)
        res["vs_gpu_f64_after_%d" % LONG_STEPS] = whole_field_errors(got, ref_f)
        res["unstable"] = lat.check() != rl.OK
        del got
        lat.close()
        del lat
        torch.cuda.empty_cache()
        results[key] = res
    del ref_f
    torch.cuda.empty_cache()
    return results


def workload_forms(rl, torch, wl, keys, steps, warmup, chunk, prof_n, tune_steps, head=None):
    """Time every storage form of a workload; returns {key: result}."""
    out = {}
    for key in keys:
        storage, _, fold = key.partition("_")
        stencil = "SPH26_ZFOLD" if fold else "SPH26"
        if head is not None and key == "F32":
            out[key] = head
            continue
        lat, r = run_form(rl, torch, wl, storage, steps, warmup, chunk, prof_n, stencil,
                          tune_steps=tune_steps_for(wl, tune_steps))
        lat.close()
        del lat
        torch.cuda.empty_cache()
        tag = f"{wl.name}_{storage}" + ("_SPH26_ZFOLD" if fold else "")
        r["traffic_bytes_per_launch"] = committed_traffic(tag, r["kernel_form"][0])
        out[key] = r
        log(f"{wl.name} {key}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_ms'] * 1e3:.2f} us "
            f"({r['kernel_form'][0]}:{r['kernel_form'][1]}) = {r['kernel_gbs']:.0f} GB/s "
            f"({100 * r['kernel_frac_hbm_peak']:.1f}% of 8 TB/s)")
    if "F64" in out:
        for r in out.values():
            r["gain_vs_gpu_f64"] = r["mlups"] / out["F64"]["mlups"]
    return out


def run_insitu(rl, torch, wl, storage, form, every, cycles, nbins=None):
    """The workload's run with its in-situ diagnostics: the energy spectrum and
    enstrophy every `every` steps (Sec. IV / Sec. V), `cycles` times, in the
    given kernel form; wall time of steps plus diagnostics (the spectrum call
    synchronises), against the steps alone."""
    lat = make_lattice(rl, wl, storage, torch)
    lat.set_kernel(*form)
    nb = nbins or wl.n // 2
    lat.step(every)                          # warm-up, and the spectrum's scratch
    lat.spectrum(nb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(cycles):
        lat.step(every)
        Ek, Z = lat.spectrum(nb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(cycles):
        lat.step(every)
    torch.cuda.synchronize()
    steps_only = time.perf_counter() - t0
    sites = wl.n * wl.n
    out = {"storage": storage, "kernel_form": list(form), "steps_between_diagnostics": every,
           "cycles": cycles, "bins": nb,
           "ms_per_step_with_diagnostics": 1e3 * wall / (cycles * every),
           "ms_per_step_steps_only": 1e3 * steps_only / (cycles * every),
           "diagnostic_ms": 1e3 * (wall - steps_only) / cycles,
           "mlups_with_diagnostics": sites * cycles * every / wall / 1e6,
           "enstrophy_last": Z, "energy_last": float(np.sum(Ek)),
           "unstable": lat.check() != rl.OK}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def copy_ceiling(rl, torch, nbytes, reps=10):
    """The library's streaming copy (16-byte loads and stores, rlbm_stream_copy)
    and torch's device copy of nbytes: read + write bytes per second."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    ms = rl.stream_copy(a, b, reps)
    out = {"bytes_each_way": 4 * n, "library_copy_ms": ms,
           "library_copy_gbs": 2 * 4 * n / (ms * 1e-3) / 1e9}
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    end.record()
    torch.cuda.synchronize()
    tms = start.elapsed_time(end) / reps
    out["torch_copy_ms"] = tms
    out["torch_copy_gbs"] = 2 * 4 * n / (tms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


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
           "step_gbs": 2 * 26 * BYTES["F32"] * sites / (ms * 1e-3) / 1e9,
           "unstable": ens.check() != rl.OK, "kernel_form": list(form)}
    ens.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, rows):
    """The FP64 oracle, single thread, one forced step of a band of `rows`
    rows (full width) of the workload: its stages (stream, moments, Landau,
    equilibrium, collision, force term with the force evaluated at the band's
    sites from the workload's modes) on the band and its two halo rows."""
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import forcing as oforcing
    from oracle import rlbm as orlbm
    from oracle import stencil as ostencil
    st = ostencil.sph26()
    A, klo, khi, fseed = wl.forcing
    e, bx, by = workloads.initial_fields(wl)
    band = np.arange(-1, rows + 1) % wl.n
    e, bx, by = e[band], bx[band], by[band]
    Y, X = np.meshgrid(band.astype(np.float64), np.arange(wl.n, dtype=np.float64), indexing="ij")
    with threadpool_limits(limits=1):
        F = orlbm.set_state(e, bx, by, st)
        t = time.perf_counter()
        Fs = orlbm.stream(F, st, 1.0)
        T, R = orlbm.moments(Fs, st)
        eps, u = orlbm.landau(T)
        beta = u[1:] / u[0]
        Fn = orlbm.collide(Fs, orlbm.equilibrium(eps, beta, st), beta, wl.tau, st)
        fx, fy = oforcing.force_at(wl.n, wl.n, A, klo, khi, fseed, 0, X.ravel(), Y.ravel())
        Fn = Fn + orlbm.force_source(T, R, fx.reshape(X.shape), fy.reshape(X.shape), 1.0, st)
        dt = time.perf_counter() - t
    sites = (rows + 2) * wl.n
    return {"value": sites / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"one forced step of a {rows + 2}-row full-width band ({sites} sites) of the "
                      f"{wl.n}x{wl.n} workload ({len(oforcing.modes(wl.n, wl.n, klo, khi))} "
                      f"force modes), FP64 NumPy oracle on one host core, {dt:.1f} s; the whole "
                      f"lattice would take {wl.n * wl.n / (sites / dt):.0f} s per step "
                      f"(extrapolated)",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def _oracle_realization(args):
    r, n, tau, steps = args
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import rlbm as orlbm
    from oracle import stencil as ostencil
    st = ostencil.sph26()
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=r)
    with threadpool_limits(limits=1):
        F = orlbm.set_state(e, bx, by, st)
        t = time.perf_counter()
        F = orlbm.run(F, st, tau, steps, force=dict(amplitude=1e-5, k_lo=2.0, k_hi=4.0, seed=r),
                      realization=r)
        return n * n * steps, time.perf_counter() - t


def oracle_all_cores(count=64, steps=2):
    """Ensemble realizations 0 .. count-1 stepped by the oracle in a pool of
    one process per usable core (at most 16): aggregate MLUPS."""
    import multiprocessing as mp
    import workloads
    spec = workloads.ensemble()[:count]
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    jobs = [(r, n, tau, steps) for r, (n, tau) in enumerate(spec)]
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_realization, jobs)
    wall = time.perf_counter() - t
    sites = sum(s for s, _ in res)
    return {"value": sites / wall / 1e6, "unit": "MLUPS", "cores": workers, "kind": "oracle",
            "sample": f"{count} realizations of the ensemble workload, {steps} steps each, one "
                      f"FP64 NumPy oracle process per core ({wall:.1f} s wall)",
            "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline form (with its roofline and CPU baseline)")
    ap.add_argument("--cpu-rows", type=int, default=64)
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
                    help="also run the library's streaming copy of this many bytes 3 times "
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
        rl.stream_copy(src, dst, 2)
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
        lat, r = run_form(rl, torch, w, storage, a.steps, a.warmup, 50, min(a.steps, 200),
                          st[0] if st else "SPH26",
                          tune_steps=tune_steps_for(w, a.tune_steps), form=form)
        lat.close()
        log(f"{name} {storage}: {r['mlups']:.0f} MLUPS, kernel {r['kernel_ms'] * 1e3:.2f} us "
            f"= {r['kernel_gbs']:.0f} GB/s")
        print(json.dumps({"only": a.only, **r}), flush=True)
        return

    wl = workloads.WORKLOADS["forced8192"]
    chunk = 10
    head_lat, head = run_form(rl, torch, wl, "F32", a.steps, a.warmup, chunk, 40,
                              tune_steps=tune_steps_for(wl, a.tune_steps))
    head_lat.close()
    del head_lat
    torch.cuda.empty_cache()
    log(f"forced8192 F32 (headline): {head['mlups']:.0f} MLUPS, {head['ms_per_step']:.3f} ms/step, "
        f"kernel {head['kernel_ms'] * 1e3:.1f} us per launch ({head['kernel_form'][0]}:"
        f"{head['kernel_form'][1]}) = {head['kernel_gbs']:.0f} GB/s")

    # the practical streaming ceiling: a copy of one FP32 step's bytes
    copy = copy_ceiling(rl, torch, wl.n * wl.n * 26 * 4)
    log(f"copy of {copy['bytes_each_way'] / 1e9:.2f} GB: library {copy['library_copy_gbs']:.0f} GB/s, "
        f"torch {copy['torch_copy_gbs']:.0f} GB/s")

    kname = KERNEL_NAMES[head["kernel_form"][0]]
    traffic = committed_traffic("forced8192_F32", head["kernel_form"][0])
    head["traffic_bytes_per_launch"] = traffic
    roofline = {"bound": "hbm", "achieved": head["kernel_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": head["kernel_gbs"] / HBM_PEAK_GBS,
                "traffic": traffic,
                "kernel": "rlbm::%s<StF32, Sph26, unit cfl, forced>" % kname,
                "kernel_form": head["kernel_form"],
                "algorithmic_bytes_per_launch": head["algorithmic_bytes_per_launch"],
                "kernel_ms": head["kernel_ms"],
                "frac_of_copy_ceiling": head["kernel_gbs"] / copy["library_copy_gbs"],
                "traffic_gbs": (traffic / (head["kernel_ms"] * 1e-3) / 1e9) if traffic else None}

    golden = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else None
    extra = {"copy": copy}
    forms = {"F32": head}
    if not a.no_extra:
        keys = ("F32", "F64", "F16S", "BF16S", "F32_ZFOLD", "F16S_ZFOLD")
        forms = workload_forms(rl, torch, wl, keys, 40, 10, chunk, 20, a.tune_steps, head=head)
        errs = field_error_runs(rl, torch, wl, forms, golden)
        for k, v in errs.items():
            forms[k]["field_error"] = v
            log(f"forced8192 {k} field error:", json.dumps(v))
        w2 = workloads.WORKLOADS["forced2048"]
        f2 = workload_forms(rl, torch, w2, keys, 300, 20, 20, 20, a.tune_steps)
        for k, v in field_error_runs(rl, torch, w2, f2, golden).items():
            f2[k]["field_error"] = v
            log(f"forced2048 {k} field error:", json.dumps(v))
        extra["forced2048"] = f2
        w5 = workloads.WORKLOADS["forced512"]
        f5 = workload_forms(rl, torch, w5, ("F32", "F64", "F16S", "BF16S", "F32_ZFOLD"),
                            2000, 200, 50, 500, a.tune_steps)
        for r in f5.values():
            r["note"] = ("both buffers fit the 256 MB Infinity Cache: kernel_gbs is an "
                         "effective rate, not HBM traffic")
            r.pop("kernel_frac_hbm_peak", None)
        extra["forced512_cache_resident"] = f5
        extra["ensemble256"] = run_ensemble(rl, torch, 200, 20)
        log(f"ensemble256 F32: {extra['ensemble256']['mlups']:.0f} MLUPS")
        torch.cuda.empty_cache()
        # the configurations' diagnostics cadence: 8192^2 spectrum and enstrophy
        # every 500 steps, 2048^2 spectrum every 1000 steps
        extra["insitu"] = {
            "forced8192": run_insitu(rl, torch, wl, "F32", tuple(head["kernel_form"]), 500, 2),
            "forced2048": run_insitu(rl, torch, w2, "F32", tuple(f2["F32"]["kernel_form"]), 1000, 2),
        }
        for k, v in extra["insitu"].items():
            log(f"{k} F32 with diagnostics every {v['steps_between_diagnostics']} steps: "
                f"{v['mlups_with_diagnostics']:.0f} MLUPS, diagnostic {v['diagnostic_ms']:.1f} ms")

    cpu = None if a.no_cpu_baseline else cpu_baseline(wl, a.cpu_rows)
    if cpu:
        log("cpu baseline:", cpu)
        if not a.no_extra:
            extra["oracle_all_cores"] = oracle_all_cores()
            log("oracle, all cores:", extra["oracle_all_cores"])

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
        "config": {"workload": "forced8192: 8192x8192 periodic, SPH26 stencil (26 populations), "
                               "tau 0.505, beta~N(0,0.002^2) seed 3, force shell |k| in [32,40] "
                               "(910 modes) amplitude 2e-6 Philox seed 2, FP32 populations, "
                               "FP64 Landau frame",
                   "lattice": [wl.n, wl.n], "storage": "F32", "parallelism": "single GPU",
                   "graph_chunk": chunk},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
