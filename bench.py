"""Benchmark of the CSD propagation hot path on one MI355X.

Headline workload: a Gaussian Schell-model source, N = 128 samples per axis (2^28 CSD elements),
complex64, pitch 20 um, sigma_S = 0.1 mm, sigma_g = 0.05 mm, lambda = 632.8 nm, Fresnel z = 0.5 m.
One step is the forward path of Algorithm 1 plus the observables: build W0 -> Fresnel propagation ->
S -> mu(P1, .). Inputs are synthetic and the source is built on the GPU. The timed region starts
with everything resident in HBM.

It prints ONE JSON line. `value` = N^4 / (time per step) in CSD elements/s. `roofline` covers the
propagation operator: algorithmic bytes (2 sweeps x read + write = 32 B/element in complex64)
divided by the summed duration of its kernel launches, measured with HIP events on the stream the
kernels run on. `cpu_baseline` times the FP64 oracle on the host for one step of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(msg: str) -> None:
    """Progress on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the c128 / far-field / adjoint / copy detail")
    ap.add_argument("--no-big", action="store_true", help="skip the N=256 complex64 workload (34 GB)")
    ap.add_argument("--plan", default="default",
                    help="pass schedule for N=128 complex64: 'default' (the library's built-in plan), 'auto' "
                         "(autotune), or "
                         "'fused,slab_chunk,col_chunk[,coop_cols,coop_lookahead]'")
    ap.add_argument("--pmc-sample", nargs="?", const="propagate", default=None,
                    choices=["propagate", "batch", "padded", "source", "n256"],
                    help="run one untimed invocation for a counter run and exit: 'propagate' (build, in-place "
                         "propagation, then a 2 GiB runtime copy of known size for calibration), 'batch' "
                         "(the 64-pair observables batch, then the 16-wavelength sum at z = 0.5 m on the FFT grid of "
                         "500 nm), 'padded' (N = 200 complex64 in place, padded to "
                         "N_z = 512, then unpadded) or 'source' (build + propagation, then the one-call source "
                         "propagation, five times each) or 'n256' (the N = 256 GSM complex64 build and one in-place "
                         "propagation under the plan of the timed N = 256 leg, 0,512,64, then a 2 GiB runtime copy "
                         "for calibration)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="rocprofv3 FETCH/WRITE summary for the current kernels (optional)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="no GPU: from the counter_collection.csv files of two rocprofv3 runs of "
                         "'--pmc-sample propagate' (FETCH_SIZE, then WRITE_SIZE) with the same --plan, write the "
                         "calibrated HBM bytes of one propagation to --traffic and exit")
    ap.add_argument("--traffic-workload", default="gsm128_fresnel_c64", choices=["gsm128_fresnel_c64", "gsm256_fresnel_c64"],
                    help="workload name recorded by --write-traffic ('gsm256_fresnel_c64' for '--pmc-sample n256', "
                         "with --plan 0,512,64 and --traffic profiles/traffic_gsm256.json)")
    return ap.parse_args()


def timed_steps(fn, steps, warmup, marks):
    """Run `fn(record)` warmup + steps times; `record(name)` drops a HIP event on the current stream.
    Returns (total ms over the timed steps, {segment: mean ms})."""
    import torch

    for _ in range(warmup):
        fn(lambda name: None)
    torch.cuda.synchronize()
    ev = []

    def record(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        ev[-1].append((name, e))

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        ev.append([])
        record("begin")
        fn(record)
    stop.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    total = start.elapsed_time(stop)
    seg = {}
    for step in ev:
        for (a, ea), (b, eb) in zip(step[:-1], step[1:]):
            seg.setdefault(b, []).append(ea.elapsed_time(eb))
        seg.setdefault("step", []).append(step[0][1].elapsed_time(step[-1][1]))
    mean = {k: sum(v) / len(v) for k, v in seg.items()}
    median = {k: sorted(v)[len(v) // 2] if len(v) % 2 else 0.5 * (sorted(v)[len(v) // 2 - 1] + sorted(v)[len(v) // 2])
              for k, v in seg.items()}
    return total, wall, mean, median


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.plan, args.traffic, args.traffic_workload)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; run it with --gpus 1 "
              "(multi-GPU sharding of the CSD propagation is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2203_02734_amd as wolf
    import wolf_inputs as WI

    wolf.load()
    torch.cuda.set_device(0)
    wl = WI.gsm128()
    n, p, lam, z = wl.n, wl.pitch_m, wl.wavelength_m, wl.z_m
    elems = n ** 4
    ip, jp = wl.probe

    w = torch.empty((n, n, n, n), dtype=torch.complex64, device="cuda")
    wb = torch.empty_like(w)
    # Pass schedule: the library's built-in plan, its autotuner (untimed, part of the set-up), or a given one.
    if args.plan == "auto":
        plan, _ = wolf.autotune(n, torch.complex64, reps=3, work=wb)
    elif args.plan != "default":
        vals = [int(x) for x in args.plan.split(",")]
        wolf.set_plan(n, torch.complex64, *vals)   # fused, slab_chunk, col_chunk[, coop_cols, coop_lookahead]
    plan = wolf.get_plan(n, torch.complex64)
    del wb
    torch.cuda.empty_cache()
    if args.pmc_sample == "propagate":
        wolf.build_source(wl.source, n, p, out=w)
        wolf.propagate_fresnel(w, p, lam, z, out=w)
        cal = torch.empty_like(w)
        cal.copy_(w)  # calibration: 2 GiB read + 2 GiB write by the runtime's copy kernel
        torch.cuda.synchronize()
        print("pmc sample done", flush=True)
        return
    if args.pmc_sample == "source":
        # Build + in-place propagation five times, then the source and its propagation in one call
        # (wolf_propagate_source) five times.
        for _ in range(5):
            wolf.build_source(wl.source, n, p, out=w)
            wolf.propagate_fresnel(w, p, lam, z, out=w)
        for _ in range(5):
            wolf.propagate_source(wl.source, n, p, lam, z, out=w)
        torch.cuda.synchronize()
        print("pmc sample done", flush=True)
        return
    if args.pmc_sample == "padded":
        del w
        torch.cuda.empty_cache()
        n2, p2, z2, w2 = padded_source(wolf)
        for nz in (512, 200):
            wolf.propagate_padded(w2, p2, wolf_lam(), z2, nz, out=w2)
        torch.cuda.synchronize()
        print("pmc sample done", flush=True)
        return
    if args.pmc_sample == "n256":
        del w
        torch.cuda.empty_cache()
        wl2 = WI.gsm256()[0]
        n2, p2 = wl2.n, wl2.pitch_m
        wolf.set_plan(n2, torch.complex64, *N256_PLAN)
        w2 = wolf.build_source(wl2.source, n2, p2, torch.complex64)
        wolf.propagate_fresnel(w2, p2, wl2.wavelength_m, wl2.z_m, out=w2)
        cal = torch.empty(1 << 28, dtype=torch.complex64, device="cuda")
        cal.copy_(w2.view(-1)[: 1 << 28])  # calibration: 2 GiB read + 2 GiB write by the runtime's copy kernel
        torch.cuda.synchronize()
        print("pmc sample done", flush=True)
        return
    if args.pmc_sample == "batch":
        pairs = WI.polychromatic_pairs()
        wolf.build_source(wl.source, n, p, out=w)
        wolf.propagate_batch(w, p, pairs["wavelength"], pairs["z"], pairs["weight"], ip=ip, jp=jp)
        sel = pairs["z"] == 0.5
        wolf.propagate_polychromatic(w, p, pairs["wavelength"][sel], pairs["z"][sel], pairs["weight"][sel],
                                     500e-9 * 0.5 / (n * p), ip=ip, jp=jp)
        torch.cuda.synchronize()
        print("pmc sample done", flush=True)
        return

    # The step rebuilds W0 each time, so it propagates in place (w_in == w_out): each pass then
    # reads and writes the same lines, which HBM serves faster than a read stream plus a separate
    # write stream.
    def step(record):
        wolf.build_source(wl.source, n, p, out=w)
        record("build")
        wolf.propagate_fresnel(w, p, lam, z, out=w)
        record("propagate")
        wolf.spectral_density(w)
        wolf.degree_of_coherence(w, ip, jp)
        record("observables")

    log("timed steps")
    total_ms, wall_ms, seg, seg_median = timed_steps(step, args.steps, args.warmup, None)
    ms_per_step = total_ms / args.steps
    prop_ms = seg["propagate"]
    bytes_prop = 32.0 * elems            # algorithmic: 2 sweeps x (read + write) x 8 B
    achieved = bytes_prop / (prop_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            if (tr.get("kernels_sha") == kernels_sha() and tr.get("workload") == "gsm128_fresnel_c64"
                    and tr.get("plan") == plan):
                traffic = tr.get("propagate_bytes_per_launch")
        except Exception:
            traffic = None

    detail = {"plan_c64": plan, "build_ms": round(seg["build"], 4), "propagate_ms": round(prop_ms, 4),
              "observables_ms": round(seg["observables"], 4),
              "median_ms_per_step": round(seg_median["step"], 4),
              "median_propagate_ms": round(seg_median["propagate"], 4),
              "propagate_elems_per_s": elems / (prop_ms * 1e-3),
              "wall_ms_timed_region": round(wall_ms, 3)}
    # The complex64 result of the last timed step, kept on the host for its error against the FP64 oracle.
    torch.cuda.synchronize()
    w_last = w.cpu()
    log("full mu, ceilings")
    detail.update(mu_full(wolf, w, ip, jp))
    detail.update(ceilings(wolf, w))       # overwrites w (the write-only pass fills it with zeros)
    del w
    torch.cuda.empty_cache()

    if not args.no_extras:
        log("extras")
        detail.update(extras(wolf, wl, args))
        log("batch and fit")
        detail.update(batch_and_fit(wolf, args))
        log("direct check")
        detail.update(direct_check(wolf))
        log("padded")
        detail.update(padded_check(wolf))
    if not args.no_big:
        log("N = 256")
        detail.update(big(wolf, args))

    result = {
        "metric": "CSD elems/s propagated, N=128 c64 vs c128 at rel err<=1e-5; % HBM peak",
        "value": elems / (ms_per_step * 1e-3),
        "unit": "elems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "gsm128_fresnel: GSM source N=128 (2^28 CSD elements) complex64, pitch 20 um, "
                               "sigma_S 0.1 mm, sigma_g 0.05 mm, lambda 632.8 nm, Fresnel z 0.5 m; step = "
                               "build W0 + propagate in place + S + mu(P1)",
                   "n": n, "elements": elems, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "wolf_propagate_fresnel (all its passes), 32 B/element algorithmic"},
        "detail": detail,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"], wb_ref = cpu_baseline(wl)
        detail["c64_rel_l2_vs_fp64_oracle"] = rel_l2_slabs(w_last, wb_ref)
        detail["c64_rel_l2_vs_fp64_oracle_source"] = "the oracle's W_B of the cpu_baseline step (full 4D, FP64)"
        del wb_ref
        log("cpu baseline N = 64")
        detail["cpu_baseline_n64"] = cpu_baseline_n64()
    else:
        detail["c64_rel_l2_vs_fp64_oracle"] = rel_l2_separable(w_last, wl)
        detail["c64_rel_l2_vs_fp64_oracle_source"] = "the oracle's separable FP64 form of W_B (GSM source)"
    print(json.dumps(result), flush=True)


def _time(fn, reps):
    """Mean ms of `reps` calls of fn on the current stream (HIP events), after two warm-up calls."""
    import torch

    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def ceilings(wolf, w):
    """Measured memory ceilings on the same 2 GiB array (hand-written streaming kernels, see
    wolf_memory_ceiling): in-place read + write (the pattern of every in-place pass), write only, read
    only; each the better of plain and nontemporal accesses. The propagation passes are compared with
    the first."""
    nbytes = w.numel() * w.element_size()
    out = {}
    for mode, tag, moved in ((0, "rmw", 2), (1, "write", 1), (2, "read", 1)):
        plain = moved * nbytes / (_time(lambda: wolf.memory_ceiling(w, mode), 10) * 1e-3) / 1e9
        nt = moved * nbytes / (_time(lambda: wolf.memory_ceiling(w, mode + 3), 10) * 1e-3) / 1e9
        out[f"ceiling_{tag}_GBps"] = round(max(plain, nt), 1)
        out[f"ceiling_{tag}_plain_GBps"] = round(plain, 1)
        out[f"ceiling_{tag}_nontemporal_GBps"] = round(nt, 1)
    return out


def mu_full(wolf, w, ip, jp):
    """The full N^4 degree of coherence (Algorithm 5 at every P1) of the propagated W_B of the step.
    It writes every mu entry (8 B) and reads W only where both S exceed the floor, so the bytes it moves
    are 8 + 8 f B/element, f the fraction of (p1, p2) pairs above the floor."""
    import torch

    n = w.shape[0]
    elems = float(n) ** 4
    o = torch.empty_like(w)
    floor = 1e-12
    t = _time(lambda: wolf.degree_of_coherence(w, -1, -1, floor, out=o), 5)
    s = wolf.spectral_density(w).double()
    f = float((s > floor * s.max()).double().mean()) ** 2
    moved = (8.0 + 8.0 * f) * elems
    del o
    return {"c64_mu_full_ms": round(t, 4), "c64_mu_full_pairs_read_fraction": round(f, 4),
            "c64_mu_full_moved_GBps": round(moved / (t * 1e-3) / 1e9, 1),
            "c64_mu_full_note": "propagated W_B of the step, floor 1e-12; bytes = 8 B write + 8 B read per pair above the floor"}


def rel_l2_slabs(w_dev_host, wb_ref):
    """Relative L2 distance of the complex64 result from the FP64 oracle, over all N^4 entries, one slab
    row at a time."""
    import numpy as np

    num = den = 0.0
    for i in range(wb_ref.shape[0]):
        a = w_dev_host[i].numpy().astype(np.complex128)
        b = wb_ref[i]
        num += float(np.sum(np.abs(a - b) ** 2))
        den += float(np.sum(np.abs(b) ** 2))
    return math.sqrt(num / den)


def rel_l2_separable(w_dev_host, wl):
    """The same distance against the oracle's separable FP64 form of W_B (GSM source)."""
    import numpy as np

    import oracle as O

    n, p, lam, z = wl.n, wl.pitch_m, wl.wavelength_m, wl.z_m
    sp = wl.source
    bx, by = O.propagate_separable(O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "x"),
                                   O.gsm_axis_factor(n, p, sp.sigma_s_m, sp.sigma_g_m, "y"), n, p, lam, z)
    num = den = 0.0
    for i in range(n):
        a = w_dev_host[i].numpy().astype(np.complex128)
        b = bx[i][None, :, None] * by[:, None, :]
        num += float(np.sum(np.abs(a - b) ** 2))
        den += float(np.sum(np.abs(b) ** 2))
    return math.sqrt(num / den)


def plan_dict(text: str) -> dict:
    """The plan of '--plan f,s,c[,coop_cols,lookahead]' in the form get_plan returns."""
    v = [int(x) for x in text.split(",")] + [0, 1][len(text.split(",")) - 3:]
    return {"fused_slab": v[0], "slab_chunk": v[1], "col_chunk": v[2], "coop_cols": v[3], "coop_lookahead": v[4]}


def write_traffic(fetch_csv: str, write_csv: str, plan_text: str, out_path: str,
                  workload: str = "gsm128_fresnel_c64") -> None:
    """Calibrated HBM bytes of the one propagation of '--pmc-sample propagate' (or 'n256'): the FETCH_SIZE and WRITE_SIZE
    values (KiB per dispatch) of the operator's dispatches (after the source build, before the copy), each
    scaled by what the same counter reads for the runtime's 2 GiB copy (2 GiB read and 2 GiB written)."""
    import csv

    def read(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]

    out = {}
    for tag, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        seq = read(path, counter)
        i0 = max(i for i, (k, _) in enumerate(seq) if "k_build_source" in k)
        i1 = min(i for i, (k, _) in enumerate(seq) if "copyBuffer" in k and i > i0)
        factor = float(2 << 30) / (seq[i1][1] * 1024.0)
        out[tag] = sum(v for _, v in seq[i0 + 1:i1]) * 1024.0 * factor
        out[tag + "_factor"] = round(factor, 4)
        out[tag + "_dispatches"] = i1 - i0 - 1
    rec = {"workload": workload, "plan": plan_dict(plan_text), "kernels_sha": kernels_sha(),
           "propagate_bytes_per_launch": int(out["fetch"] + out["write"]), "fetch_bytes": int(out["fetch"]),
           "write_bytes": int(out["write"]), "fetch_factor": out["fetch_factor"],
           "write_factor": out["write_factor"], "dispatches": out["fetch_dispatches"]}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def kernels_sha() -> str:
    """Hash of the sources that the propagation operator's kernels are compiled from: the traffic
    figure in profiles/traffic.json is used only while it matches."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_02734_amd", "csrc")
    for f in ("wolf_device.hpp", "wolf_internal.hpp", "wolf_fft.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def extras(wolf, wl, args):
    """complex128 speedup, far field, adjoint ratio and a copy-kernel ceiling (same N=128 source); the
    relative L2 error of the complex64 result against the complex128 one, here and on the N = 64 top-hat
    source with a thin lens (f = 0.2 m, Fresnel z = 0.2 m)."""
    import torch

    import wolf_inputs as WI

    n, p, lam, z = wl.n, wl.pitch_m, wl.wavelength_m, wl.z_m
    elems = n ** 4
    out = {}
    reps = max(3, min(args.steps, 10))

    def time_op(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    w = wolf.build_source(wl.source, n, p, torch.complex64)
    o = torch.empty_like(w)
    t64 = time_op(lambda: wolf.propagate_fresnel(w, p, lam, z, out=o))
    kept64 = o.clone()  # the complex64 Fresnel result, compared with complex128 below
    tff = time_op(lambda: wolf.propagate_farfield(w, p, lam, z, out=o))
    tadj = time_op(lambda: wolf.propagate_adjoint(w, p, lam, z, out=o))
    out["extras_mode"] = "out of place (w_in != w_out)"
    out["c64_fresnel_ms"] = round(t64, 4)
    out["c64_farfield_ms"] = round(tff, 4)
    out["c64_adjoint_ms"] = round(tadj, 4)
    out["adjoint_over_forward"] = round(tadj / t64, 3)
    # Two-stage imaging (lens plane at 0.4 m, f = 0.2 m, image at 0.4 m, circular pupil), in place:
    # two operator launches, the lens phase and pupil folded into the second one.
    pb = lam * 0.4 / (n * p)
    timg = time_op(lambda: wolf.image_through_lens(o, p, lam, 0.4, 0.2, 0.4, wolf.GEO_CIRCLE, 0.3 * n * pb, out=o))
    out["c64_imaging_ms"] = round(timg, 4)
    out["c64_imaging_achieved_GBps"] = round(2 * 32.0 * elems / (timg * 1e-3) / 1e9, 1)
    del w, o
    torch.cuda.empty_cache()
    w = wolf.build_source(wl.source, n, p, torch.complex128)
    o = torch.empty_like(w)
    out["plan_c128"] = wolf.autotune(n, torch.complex128, reps=2, work=o)[0]
    t128 = time_op(lambda: wolf.propagate_fresnel(w, p, lam, z, out=o))
    out["c128_fresnel_ms"] = round(t128, 4)
    out["c128_propagate_elems_per_s"] = elems / (t128 * 1e-3)
    out["c128_achieved_GBps"] = round(64.0 * elems / (t128 * 1e-3) / 1e9, 1)
    out["c64_speedup_over_c128"] = round(t128 / t64, 3)
    out["c64_rel_l2_vs_c128"] = float(torch.linalg.vector_norm(kept64.to(torch.complex128) - o) /
                                      torch.linalg.vector_norm(o))
    del w, o, kept64
    torch.cuda.empty_cache()
    t = WI.tophat_lens64()
    r = {}
    for dt in (torch.complex64, torch.complex128):
        r[dt] = wolf.propagate_fresnel(wolf.build_source(t.source, t.n, t.pitch_m, dt), t.pitch_m, t.wavelength_m,
                                       t.z_m)[0]
    out["tophat_lens64_c64_rel_l2_vs_c128"] = float(
        torch.linalg.vector_norm(r[torch.complex64].to(torch.complex128) - r[torch.complex128]) /
        torch.linalg.vector_norm(r[torch.complex128]))
    # The same N = 64 workload's step (build with the lens phase + propagation), complex64.
    w64 = torch.empty((t.n,) * 4, dtype=torch.complex64, device="cuda")
    t64s = time_op(lambda: wolf.propagate_fresnel(wolf.build_source(t.source, t.n, t.pitch_m, out=w64), t.pitch_m,
                                                  t.wavelength_m, t.z_m, out=w64))
    out["tophat_lens64_c64_step_ms"] = round(t64s, 4)
    out["tophat_lens64_c64_elems_per_s"] = t.n ** 4 / (t64s * 1e-3)
    # The same steps through wolf_propagate_source: the half-buffer slab pass (the built-in schedule at
    # N = 64 and 128) forms the source where it would load W0 (bit-identical result), so W0 is never
    # written and read back.
    t64f = time_op(lambda: wolf.propagate_source(t.source, t.n, t.pitch_m, t.wavelength_m, t.z_m, out=w64))
    out["tophat_lens64_c64_source_step_ms"] = round(t64f, 4)
    del w64
    w = torch.empty((n,) * 4, dtype=torch.complex64, device="cuda")
    ip, jp = wl.probe

    def source_step():
        wolf.propagate_source(wl.source, n, p, lam, z, out=w)
        wolf.spectral_density(w)
        wolf.degree_of_coherence(w, ip, jp)

    tsrc = time_op(source_step)
    out["c64_source_step_ms"] = round(tsrc, 4)
    out["c64_source_step_elems_per_s"] = elems / (tsrc * 1e-3)
    del w
    torch.cuda.empty_cache()
    w = torch.empty((n,) * 4, dtype=torch.complex128, device="cuda")
    out["c128_source_propagate_ms"] = round(time_op(lambda: wolf.propagate_source(
        wl.source, n, p, lam, z, dtype=torch.complex128, out=w)), 4)
    del w
    torch.cuda.empty_cache()
    return out


def batch_and_fit(wolf, args):
    """The polychromatic batch (N=128 c64, 16 lambda x 4 z, Fresnel and far field, one recorded graph
    each; S and mu only, no propagated N^4 output) and one fit step
    (N=64 c64 custom map: forward and adjoint timed separately)."""
    import math

    import numpy as np
    import torch

    import wolf_inputs as WI
    from paper_2203_02734_amd.autograd import propagated_spectral_density

    out = {}
    wl = WI.gsm128()
    n, p = wl.n, wl.pitch_m
    pairs = WI.polychromatic_pairs()
    w0 = wolf.build_source(wl.source, n, p, torch.complex64)
    work = torch.empty(wolf.batch_work_bytes(n, torch.complex64), dtype=torch.uint8, device="cuda")
    k = len(pairs["z"])
    for tag, ff in (("batch64", False), ("batch64_farfield", True)):
        run = lambda: wolf.propagate_batch(w0, p, pairs["wavelength"], pairs["z"], pairs["weight"], farfield=ff,
                                           ip=wl.probe[0], jp=wl.probe[1], work=work)
        for _ in range(2):  # the first call records the group's graph
            run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        reps = 10
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / reps
        out[f"{tag}_ms"] = round(t, 3)
        out[f"{tag}_pairs_per_s"] = round(k / (t * 1e-3), 1)
    # Fresnel: two contractions over the first point shared by the 64 pairs, 8 real flops per complex
    # multiply-add, 64 pairs x N^4 multiply-adds each.
    out["batch64_contraction_TFLOPs"] = round(2 * 8 * k * n ** 4 / (out["batch64_ms"] * 1e-3) / 1e12, 2)
    # Polychromatic sum on a common grid (the FFT grid of 500 nm): the 16 wavelengths at z = 0.5 m, and all
    # 64 pairs, S and mu(P1, .) of the weighted sum.
    pwork = torch.empty(wolf.polychromatic_work_bytes(n, torch.complex64), dtype=torch.uint8, device="cuda")
    dxc = 500e-9 * 0.5 / (n * p)
    for tag, sel in (("poly16", pairs["z"] == 0.5), ("poly64", pairs["z"] > 0)):
        args3 = (pairs["wavelength"][sel], pairs["z"][sel], pairs["weight"][sel])
        run = lambda: wolf.propagate_polychromatic(w0, p, *args3, dxc, ip=wl.probe[0], jp=wl.probe[1], work=pwork)
        for _ in range(2):
            run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            run()
        b.record()
        torch.cuda.synchronize()
        out[f"{tag}_common_grid_ms"] = round(a.elapsed_time(b) / 10, 3)
    del pwork
    del w0, work
    torch.cuda.empty_cache()
    # The same 64-pair Fresnel batch in complex128 (vector-FMA contractions).
    w0 = wolf.build_source(wl.source, n, p, torch.complex128)
    work = torch.empty(wolf.batch_work_bytes(n, torch.complex128), dtype=torch.uint8, device="cuda")
    run = lambda: wolf.propagate_batch(w0, p, pairs["wavelength"], pairs["z"], pairs["weight"], ip=wl.probe[0],
                                       jp=wl.probe[1], work=work)
    run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    run()
    b.record()
    torch.cuda.synchronize()
    out["batch64_c128_ms"] = round(a.elapsed_time(b), 3)
    del w0, work
    torch.cuda.empty_cache()

    fw, tw = WI.fit_map64(), WI.fit_target64()
    n, p, lam, z = fw.n, fw.pitch_m, fw.wavelength_m, fw.z_m
    im = torch.tensor(fw.source.intensity_map, dtype=torch.float32, device="cuda", requires_grad=True)
    sg = torch.tensor(fw.source.sigma_g_m, dtype=torch.float64, requires_grad=True)
    target = wolf.spectral_density(wolf.propagate_fresnel(wolf.build_source(tw.source, n, p), p, lam, z)[0])
    fwd_ms, bwd_ms = [], []
    for it in range(6):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        s = propagated_spectral_density(im, sg, p, lam, z)
        loss = torch.sum((s - target) ** 2)
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        if it >= 2:
            fwd_ms.append(e0.elapsed_time(e1))
            bwd_ms.append(e1.elapsed_time(e2))
        im.grad = None
        sg.grad = None
    f, g = sum(fwd_ms) / len(fwd_ms), sum(bwd_ms) / len(bwd_ms)
    out["fit64_forward_ms"] = round(f, 4)
    out["fit64_backward_ms"] = round(g, 4)
    out["fit64_backward_over_forward"] = round(g / f, 3)
    return out


def direct_check(wolf):
    """Exact-kernel direct sum (the validity check of the Fresnel approximation), N = 64 GSM source at
    z = 20 mm: two dense complex products of size N^2 = 4096 (8 N^6 real flops each)."""
    import torch

    import wolf_inputs as WI

    out = {}
    n, p, z = 64, 20e-6, 0.02
    src = WI.gsm_small()[0].source
    flops = 2 * 8.0 * float(n * n) ** 3
    for dt, tag in ((torch.complex128, "c128"), (torch.complex64, "c64")):
        w = wolf.build_source(src, n, p, dt)
        o = torch.empty_like(w)
        work = torch.empty(int(wolf.load().wolf_direct_work_bytes(n, 1 if dt == torch.complex128 else 0)),
                           dtype=torch.uint8, device="cuda")
        wolf.propagate_direct(w, p, wolf_lam(), z, out=o, work=work)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            wolf.propagate_direct(w, p, wolf_lam(), z, out=o, work=work)
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / 3
        out[f"direct64_{tag}_ms"] = round(t, 3)
        out[f"direct64_{tag}_TFLOPs"] = round(flops / (t * 1e-3) / 1e12, 2)
        del w, o, work
    w = wolf.build_source(src, n, p, torch.complex128)
    out["fresnel_validity_n64_z20mm"] = wolf.fresnel_validity(w, p, wolf_lam(), z)
    del w
    torch.cuda.empty_cache()
    return out


def padded_source(wolf):
    """The N = 200 GSM source of the padded workload (complex64, 12.8 GB), with its pitch and distance."""
    import types

    import torch

    import wolf_inputs as WI

    n, p, z = 200, 20e-6, 0.5
    src = types.SimpleNamespace(model=WI.MODEL_GSM, amplitude=1.0, sigma_s_m=0.1e-3, sigma_g_m=0.05e-3,
                                geometry=WI.GEO_NONE, geo_r0_m=0.0, geo_r1_m=0.0, intensity_map=None, mask=None,
                                lens_focal_m=0.0, wavelength_m=0.0)
    return n, p, z, wolf.build_source(src, n, p, torch.complex64)


def padded_check(wolf):
    """The paper's example size: N = 200 (not a power of two), GSM source, Fresnel z = 0.5 m, complex64,
    in place (1.6e9 elements, 12.8 GB). Padded to N_z = 512 (Secs. 5.1, 5.2): four zero-padded FFT
    passes. Unpadded (N_z = 200, Secs. 5.3, 5.4): four 20 x 10 mixed-radix FFT passes. Both move 64 B
    per element (the operator needs 32 B/element). For comparison the dense passes, which any other
    N_z takes (here N_z = 210), with a 12.8 GB work array, 32 N real flops per element."""
    import torch

    n, p, z, w = padded_source(wolf)
    work = torch.empty_like(w)
    elems = float(n) ** 4
    out = {}
    for nz, tag in ((512, "padded200_512"), (200, "fft200"), (210, "dense200_210")):
        for _ in range(1 if nz == 210 else 2):
            wolf.propagate_padded(w, p, wolf_lam(), z, nz, out=w, work=work)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        reps = 2 if nz == 210 else 3
        for _ in range(reps):
            wolf.propagate_padded(w, p, wolf_lam(), z, nz, out=w, work=work)
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / reps
        out[f"{tag}_c64_ms"] = round(t, 2)
        out[f"{tag}_elems_per_s"] = elems / (t * 1e-3)
        if nz != 210:
            out[f"{tag}_moved_GBps"] = round(64.0 * elems / (t * 1e-3) / 1e9, 1)
            out[f"{tag}_algorithmic_GBps"] = round(32.0 * elems / (t * 1e-3) / 1e9, 1)
        else:
            out[f"{tag}_TFLOPs"] = round(32.0 * n * elems / (t * 1e-3) / 1e12, 2)
    del w, work
    torch.cuda.empty_cache()
    return out


def wolf_lam():
    import wolf_inputs as WI
    return WI.LAMBDA_HENE


# The N = 256 complex64 plan (row pass, i2 and j1 passes over chunks of 512 slabs, 64-column first-point chunks):
# the autotuner picks 64 or 128 columns from run to run, within 1 % of each other. The timed leg and the counter
# sample both run under this one, so that the recorded traffic applies.
N256_PLAN = (0, 512, 64)


def big(wolf, args):
    import torch

    import wolf_inputs as WI

    wl = WI.gsm256()[0]
    n, p, lam, z = wl.n, wl.pitch_m, wl.wavelength_m, wl.z_m
    wolf.set_plan(n, torch.complex64, *N256_PLAN)
    plan = wolf.get_plan(n, torch.complex64)
    w = wolf.build_source(wl.source, n, p, torch.complex64)
    for _ in range(1):
        wolf.propagate_fresnel(w, p, lam, z, out=w)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    reps = 3
    for _ in range(reps):
        wolf.propagate_fresnel(w, p, lam, z, out=w)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / reps
    del w
    torch.cuda.empty_cache()
    ach = 32.0 * n ** 4 / (t * 1e-3) / 1e9
    traffic = None
    path = os.path.join(ROOT, "profiles", "traffic_gsm256.json")
    if os.path.exists(path):
        try:
            tr = json.load(open(path))
            if (tr.get("kernels_sha") == kernels_sha() and tr.get("workload") == "gsm256_fresnel_c64"
                    and tr.get("plan") == plan):
                traffic = tr.get("propagate_bytes_per_launch")
        except Exception:
            traffic = None
    return {"n256_plan": plan, "n256_c64_fresnel_ms": round(t, 3), "n256_elems_per_s": n ** 4 / (t * 1e-3),
            "n256_roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                              "kernel": "wolf_propagate_fresnel at N = 256 GSM complex64 in place, 32 B/element "
                                        "algorithmic (2^32 elements)"}}


def cpu_baseline(wl):
    """The FP64 oracle, as it stands, for one full step of the same workload on the host cores."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_info

        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    n, p, lam, z = wl.n, wl.pitch_m, wl.wavelength_m, wl.z_m
    t0 = time.perf_counter()
    w = O.build_source(wl.source, n, p)
    wb, _ = O.propagate(w, n, p, lam, z)
    del w
    O.spectral_density(wb)
    O.degree_of_coherence(wb, *wl.probe)
    t = time.perf_counter() - t0
    return ({"value": n ** 4 / t, "unit": "elems/s", "cores": cores, "kind": "oracle",
             "sample": f"one full step of the same workload (N={n}, build + FP64 propagate + S + mu), {t:.1f} s"}, wb)


def cpu_baseline_n64():
    """The oracle's FP64 Fresnel propagation alone at N = 64 (the GSM source of the headline workload on
    a 64-point grid), on the host cores."""
    import oracle as O
    import wolf_inputs as WI

    wl = WI.gsm128()
    n, p, lam, z = 64, wl.pitch_m, wl.wavelength_m, wl.z_m
    w = O.build_source(wl.source, n, p)
    t0 = time.perf_counter()
    O.propagate(w, n, p, lam, z)
    t = time.perf_counter() - t0
    return {"value": n ** 4 / t, "unit": "elems/s", "sample": f"one FP64 Fresnel propagation at N=64, {t:.2f} s"}


if __name__ == "__main__":
    main()
