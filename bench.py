"""Benchmark of the MEM imaging hot path on one MI355X.

One step = one projected-CG iteration over the whole hot path: direction
update and projection, forward model of the direction (separable DFT on
matrix cores), chi^2 line-search scalars, the FP64 line search, image and
residual update, adjoint gradient (separable DFT), entropy term and the
Polak-Ribiere update.  Each step does one forward and one adjoint pass over
every (visibility, pixel) pair, so the headline value is
    vis.pixel evaluations / s = sum_c Z_c N^2 * steps / time.
Inputs are resident in HBM before the timed region.

Prints one JSON line (see the keys below).  The CPU baseline is the FP64
oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vis·pixel evals/sec (fwd+adjoint ∇Φ); CG iters/sec, mixed vs FP32 at stated err"
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0, "fp16x3": 2500.0}   # TFLOP/s, dense MFMA
KERNEL_SRC = "paper_1703_02920_amd/csrc/k_dft.hip"
# DFT kernel functions per precision: (forward, adjoint)
KERNELS = {"fp32": ("k_forward_p", "k_adjoint_w"), "fp64": ("k_forward_p", "k_adjoint"),
           "bf16x3": ("k_forward_h16m", "k_adjoint_h16s"), "fp16x3": ("k_forward_h16m", "k_adjoint_h16s")}


def kernel_hash(kernel: str) -> str:
    """Hash of the DFT source up to the launch code, with every other kernel's
    definition and all comments removed: it changes when the code of this
    kernel or of a device helper it may use changes."""
    import re
    with open(os.path.join(ROOT, KERNEL_SRC)) as f:
        src = f.read()
    cut = src.find("hipError_t fwd_dispatch")
    if cut > 0:
        src = src[:cut]
    src = re.sub(r"[ \t]*//[^\n]*", "", src)
    src = re.sub(r"\n\s*\n", "\n", src)
    # a kernel definition runs from its template line to the closing brace at
    # column 0
    pat = re.compile(r"^(?:template <[^\n]*>\n)?__global__ [^\n]*? void (k_\w+)\(.*?^}\n", re.S | re.M)
    if kernel not in {m.group(1) for m in pat.finditer(src)}:
        raise ValueError(f"no kernel {kernel} in {KERNEL_SRC}")
    kept = pat.sub(lambda m: m.group(0) if m.group(1) == kernel else "", src)
    return hashlib.sha256(kept.encode()).hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 counters for the current
    kernel source (null when the kernel changed since the counters)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("kernel_hash") != kernel_hash(kernel):
        return None
    return ent.get("bytes_per_launch")


# The paper's own timings (Sec. 4.1 timing table, abstract, conclusions):
# one Tesla K80 die against one thread of a Xeon E5-2640 v2 at 2.0 GHz, the
# FFT-gridded model with an exact direct-sum gradient, real ALMA data.
PAPER_CONTEXT = {
    "hardware": "one Tesla K80 GK210B die vs one thread of an Intel Xeon E5-2640 v2 (2.0 GHz)",
    "speedup_range_abstract": "1,000x - 5,000x over the sequential version",
    "largest_single_data_set": "2.1 min (GPU) vs 2.5 days (CPU), HD142527 CO(6-5), 107,494 visibilities, 1024^2",
    "per_iteration_minutes_cpu_gpu_speedup": {
        "CO(6-5) 1024^2": [131, 0.08, 1638], "CO(6-5) 2048^2": [349, 0.11, 3173],
        "CO(6-5) 4096^2": [360, 0.13, 2769], "HL Tau SPW0 1024^2": [2645, 0.60, 4408],
        "HL Tau SPW0 2048^2": [10339, 2.39, 4326], "HL Tau SPW0 4096^2": [55009, 9.86, 5579]},
    "note": "context only: other hardware, another forward model (gridded) and real data",
}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(ds, target_s: float = 12.0, single_s: float = 4.0):
    """FP64 oracle on a bounded sample: the forward model at a subset of the
    visibilities (all pixels) and the adjoint at a subset of the pixels (all
    visibilities).  One vis.pixel evaluation = one forward term + one adjoint
    term, so the rate is (forward pairs + adjoint pairs) / 2 / time.  Timed on
    every host thread OpenMP uses, then on one thread (the paper's speedups
    are against a single CPU thread)."""
    import numpy as np

    import oracle
    ch = ds.channels[0]
    n = ds.n
    A = oracle.beam(n, ds.cell, ch.fwhm)
    img = np.full((n, n), ds.prior_m)
    coef = (ch.w.astype(np.float64) * ch.vis.astype(np.complex128))
    rng = np.random.default_rng(0)

    def run(n_vis, n_pix):
        vi = np.sort(rng.choice(ch.nvis, size=n_vis, replace=False))
        px = np.sort(rng.choice(n * n, size=n_pix, replace=False))
        t0 = time.perf_counter()
        oracle.forward_sel(n, ds.cell, vi, ch.u, ch.v, A, img)
        oracle.adjoint(n, ds.cell, ch.u, ch.v, A, coef, pix=px)
        dt = time.perf_counter() - t0
        return (n_vis * n * n + ch.nvis * n_pix) / 2.0, dt

    def sizes(rate, seconds):
        pairs_goal = rate * seconds * 2.0
        return (int(min(ch.nvis, max(4, pairs_goal / 2.0 / (n * n)))),
                int(min(n * n, max(4, pairs_goal / 2.0 / ch.nvis))))

    def timed(seconds):
        # calibrate on a tiny sample, then on one of ~1 s (the tiny one
        # underestimates the rate), then size the real one
        p0, t0 = run(min(4, ch.nvis), 4)
        p1, t1 = run(*sizes(p0 / max(t0, 1e-6), min(1.0, seconds / 4)))
        n_vis, n_pix = sizes(p1 / max(t1, 1e-6), seconds)
        pairs, dt = run(n_vis, n_pix)
        return pairs / dt, n_vis, n_pix, dt

    threads = oracle.num_threads()
    rate, n_vis, n_pix, dt = timed(target_s)
    oracle.set_threads(1)
    try:
        rate1, n_vis1, n_pix1, dt1 = timed(single_s)
    finally:
        oracle.set_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    return {"value": rate, "unit": "vis·pixel evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 direct sums: forward at {n_vis} of {ch.nvis} visibilities x {n * n} pixels "
                      f"+ adjoint at {n_pix} of {n * n} pixels x {ch.nvis} visibilities; {dt:.1f} s on "
                      f"{threads} threads",
            "seconds": dt,
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(), "host_cpus_usable": affinity,
            "single_thread": {"value": rate1, "unit": "vis·pixel evals/s", "cores": 1,
                              "sample": f"forward at {n_vis1} visibilities + adjoint at {n_pix1} pixels; "
                                        f"{dt1:.1f} s"},
            "paper_context": PAPER_CONTEXT}


MFMA_KINDS = {"fp32": (0, "v_mfma_f32_16x16x4_f32"), "fp64": (1, "v_mfma_f64_16x16x4_f64"),
              "bf16": (2, "v_mfma_f32_16x16x32_bf16"), "fp16": (3, "v_mfma_f32_16x16x32_f16"),
              "bf16_32x32": (4, "v_mfma_f32_32x32x16_bf16"), "fp16_32x32": (5, "v_mfma_f32_32x32x16_f16")}
SPEC_PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0, "bf16_32x32": 2500.0,
             "fp16_32x32": 2500.0}


def mfma_peak(kinds=None, target_ms=20.0):
    """Measured matrix-core rate per instruction form (libmfma_peak.so built
    from mfma_peak.hip): 1,024 workgroups of four waves issuing independent
    matrix instructions; best of 5 launches of ~target_ms."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "libmfma_peak.so"))
    lib.mfma_peak.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    out = {}
    blocks = 1024
    flops = {0: 2048.0 * 8, 1: 2048.0 * 8, 2: 16384.0 * 8, 3: 16384.0 * 8, 4: 32768.0 * 4, 5: 32768.0 * 4}
    for name in (kinds or MFMA_KINDS):
        kind, inst = MFMA_KINDS[name]
        iters = int(target_ms * 1e-3 * SPEC_PEAK[name] * 1e12 / (4 * blocks * flops[kind]))
        tf, ms = ctypes.c_double(), ctypes.c_double()
        code = lib.mfma_peak(kind, blocks, max(iters, 1), 5, ctypes.byref(tf), ctypes.byref(ms))
        if code != 0:
            raise RuntimeError(f"mfma_peak({name}) failed: {code}")
        out[name] = {"instruction": inst, "tflops": tf.value, "spec_tflops": SPEC_PEAK[name],
                     "frac_of_spec": tf.value / SPEC_PEAK[name], "ms": ms.value, "iters": iters}
    return out


# matrix-instruction form of each split-precision DFT kernel on 128-row
# forward blocks and 256-pixel adjoint tiles (the c2-c5 workloads)
SPLIT_FORMS = {"bf16x3": {"forward": "bf16_32x32", "adjoint": "bf16"},
               "fp16x3": {"forward": "fp16_32x32", "adjoint": "fp16"}}


def mixed_measured(prec, kern, flops_per_launch):
    """Issued 3-product rate of each split DFT kernel over the measured rate
    of the matrix-instruction form it uses."""
    try:
        forms = SPLIT_FORMS[prec]
        pk = mfma_peak(sorted(set(forms.values())))
    except (OSError, RuntimeError, KeyError):
        return None
    return {k: {"frac": 3 * flops_per_launch / (v / 1e3) / 1e12 / pk[forms[k]]["tflops"],
                "measured_peak": pk[forms[k]]["tflops"], "instruction": pk[forms[k]]["instruction"]}
            for k, v in kern.items() if k in forms}


def run_steps(ctx, steps, warmup, graph):
    """cg_init, warm-up steps, then `steps` timed CG iterations; returns
    (ms for the timed region, wall seconds, per-kernel average ms)."""
    import torch
    I = ctx.image()
    scal = ctx.scalars()
    ctx.cg_init(I, init_to_floor=True)
    for _ in range(warmup):
        ctx.cg_step(I, scal)
    if graph:
        ctx.cg_run(I, 1, graph=True)
    torch.cuda.synchronize()
    ctx.timing(not graph)
    ctx.timing_read(0, reset=True)
    ctx.timing_read(1, reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(ctx.stream)
    if graph:
        ctx.cg_run(I, steps, graph=True)
    else:
        for _ in range(steps):
            ctx.cg_step(I, scal)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    kern = {}
    for which, name in ((0, "forward"), (1, "adjoint")):
        tot, cnt = ctx.timing_read(which)
        if cnt:
            kern[name] = tot / cnt
    ctx.timing(False)
    ctx.check()
    return ms, t_wall, kern


def eval_error(ds, ctx, ref):
    """Relative error of V^m, chi^2, Phi and grad Phi of `ctx` against the
    FP64 context `ref` (the FP64 path that the full-size parity tests hold to
    the oracle at 1e-12) at the P1 and P3 evaluation images (same inputs,
    FP32-rounded images)."""
    import numpy as np
    import torch
    from paper_1703_02920_amd import synth
    out = {}
    for which in ("P1", "P3"):
        x = synth.eval_images(ds, which).astype(np.float32)
        I = torch.tensor(x, dtype=ctx.dtype, device=ctx.device)
        Ir = torch.tensor(x.astype(np.float64), dtype=torch.float64, device=ref.device)
        V, Vr = ctx.forward(I).clone(), ref.forward(Ir).clone()
        s, g = ctx.phi_and_grad(I)
        sr, gr = ref.phi_and_grad(Ir)
        torch.cuda.synchronize()

        def rel(a, b):
            dt = torch.complex128 if a.is_complex() else torch.float64
            a, b = a.to(dt), b.to(dt)
            return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

        out[which] = {"V": rel(V, Vr),
                      "chi2": abs(float(s[:, 1].sum()) - float(sr[:, 1].sum())) / abs(float(sr[:, 1].sum())),
                      "phi": abs(float(s[:, 0].sum()) - float(sr[:, 0].sum())) / abs(float(sr[:, 0].sum())),
                      "grad": rel(g, gr)}
    return out


def _median_eval_ms(ctx, img, reps=20, warmup=3):
    """Median ms of one Phi + grad evaluation and the average forward and
    adjoint launch times (HIP events on the context's stream)."""
    import numpy as np
    import torch
    scal, grad = ctx.scalars(), torch.empty_like(img)
    for _ in range(warmup):
        ctx.phi_and_grad(img, grad, scal)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(0, reset=True)
    ctx.timing_read(1, reset=True)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.phi_and_grad(img, grad, scal)
        e1.record(ctx.stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    (fm, fc), (am, ac) = ctx.timing_read(0), ctx.timing_read(1)
    ctx.timing(False)
    ctx.check()
    return float(np.median(ts)), fm / max(fc, 1), am / max(ac, 1)


def grid_error(configs, oversamples, prec="fp32"):
    """The gridded model of Alg. 1 against the exact DFT model on the same
    workload and image (P2 = the sky, P3 = M + U[0, 1)): relative error of
    V^m, chi^2 and grad Phi -- with the gridded model's own gradient and with
    the exact-DFT gradient at the gridded residuals -- and the time of one
    Phi + grad evaluation (with forward / adjoint launch times) of each."""
    import numpy as np
    import torch
    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context

    def rel(a, b):
        return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))

    rows = []
    for c in configs:
        ds = synth.make_config(c)
        ex = Context.from_dataset(ds, prec)
        imgs = {w: torch.tensor(synth.eval_images(ds, w), dtype=ex.dtype, device=ex.device) for w in ("P2", "P3")}
        ref = {}
        for w, img in imgs.items():
            V = ex.forward(img).clone()
            sc, g = ex.phi_and_grad(img)
            ref[w] = (V, sc.clone(), g.clone())
        t_ex = _median_eval_ms(ex, imgs["P3"])
        ex.close()
        for s in oversamples:
            L = s * ds.n
            if L > 8192 or L & (L - 1):
                continue
            for grad in ("adjoint", "dft"):
                ctx = Context.from_dataset(ds, prec, forward="gridded", oversample=s, grad=grad)
                for w, img in imgs.items():
                    V = ctx.forward(img)
                    sc, g = ctx.phi_and_grad(img)
                    Vr, scr, gr = ref[w]
                    row = {"config": f"c{c}", "precision": prec, "oversample": s, "grid": L, "grad": grad,
                           "image": w, "rel_err_V": rel(V, Vr),
                           "rel_err_chi2": abs(float(sc[:, 1].sum() - scr[:, 1].sum())) / float(scr[:, 1].sum()),
                           "rel_err_grad": rel(g, gr)}
                    if w == "P3":
                        t = _median_eval_ms(ctx, img)
                        row.update({"ms_eval": t[0], "ms_forward": t[1], "ms_adjoint": t[2],
                                    "ms_eval_exact": t_ex[0], "ms_forward_exact": t_ex[1],
                                    "ms_adjoint_exact": t_ex[2]})
                    rows.append(row)
                    print(json.dumps(row), flush=True)
                ctx.close()
    return rows


def grid_cg(c, oversamples, prec="fp32", iters=None):
    """T graph-replayed CG iterations with the exact model and with the
    gridded model (each gradient choice); every final image is scored with
    the exact objective: Phi_exact(I_T) and chi^2_exact(I_T) relative to the
    exact run's, the image's relative difference from the exact run's, and
    iterations/s."""
    import torch
    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context
    ds = synth.make_config(c)
    T = iters or ds.cg_iters
    ex = Context.from_dataset(ds, prec)
    runs = [("dft", 1, "adjoint")] + [("gridded", s, g) for s in oversamples for g in ("adjoint", "dft")
                                      if s * ds.n <= 8192]
    out, base = [], None
    for fwd, s, g in runs:
        ctx = ex if fwd == "dft" else Context.from_dataset(ds, prec, forward=fwd, oversample=s, grad=g)
        I = ctx.image()
        ctx.cg_init(I, init_to_floor=True)
        ctx.cg_run(I, 1, graph=True)
        ctx.cg_init(I, init_to_floor=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.cg_run(I, T, graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ctx.check()
        ms = e0.elapsed_time(e1)
        sc, _ = ex.phi_and_grad(I)
        phi, chi2 = float(sc[:, 0].sum()), float(sc[:, 1].sum())
        row = {"config": f"c{c}", "precision": prec, "forward": fwd, "oversample": s if fwd != "dft" else None,
               "grad": g if fwd != "dft" else None, "iters": T, "ms": ms, "cg_iters_per_s": T / (ms / 1e3),
               "phi_exact_T": phi, "chi2_exact_T": chi2}
        if base is None:
            base = (phi, chi2, I.clone())
        else:
            row["rel_phi_exact_vs_exact_run"] = (phi - base[0]) / abs(base[0])
            row["rel_chi2_exact_vs_exact_run"] = (chi2 - base[1]) / abs(base[1])
            row["rel_image_diff_vs_exact_run"] = float(torch.linalg.vector_norm((I - base[2]).double())
                                                       / torch.linalg.vector_norm(base[2].double()))
        out.append(row)
        print(json.dumps(row), flush=True)
        if ctx is not ex:
            ctx.close()
    ex.close()
    return out


def eval_sweep(configs, precs, reps=20, warmup=3, mode=None):
    """M1 per configuration and precision: median time of one Phi + grad Phi
    evaluation (forward, chi^2, adjoint, entropy, combine) at the P3 image,
    timed with events on the context's stream.  mode "shared" fits the first
    P3 plane to every channel (one image, Eq. chi2-multi); the DFT work per
    channel is the same as in cube mode."""
    import numpy as np
    import torch
    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context
    rows = []
    for c in configs:
        ds = synth.make_config(c)
        img_np = synth.eval_images(ds, "P3")
        md = mode or ("shared" if ds.shared else "cube")
        if md == "shared":
            img_np = img_np[:1]
        for prec in precs:
            if prec == "fp64" and ds.n > 512:
                continue
            ctx = Context.from_dataset(ds, prec, mode=md)
            img = torch.tensor(img_np, dtype=ctx.dtype, device=ctx.device)
            ms, fwd_ms, adj_ms = _median_eval_ms(ctx, img, reps=reps, warmup=warmup)
            ctx.close()
            rows.append({"config": f"c{c}", "mode": md, "precision": prec, "ms_per_eval": ms,
                         "ms_forward": fwd_ms, "ms_adjoint": adj_ms,
                         "forward_tflops": 4.0 * ds.pairs / (fwd_ms / 1e3) / 1e12,
                         "adjoint_tflops": 4.0 * ds.pairs / (adj_ms / 1e3) / 1e12,
                         "vis_pixel_evals_per_s": ds.pairs / (ms / 1e3),
                         "algorithmic_tflops": 8.0 * ds.pairs / (ms / 1e3) / 1e12,
                         "frac_of_peak": 8.0 * ds.pairs / (ms / 1e3) / 1e12 / PEAK[prec]})
            print(json.dumps(rows[-1]), flush=True)
    return rows


SCHED_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16)


def schedule_sweep(configs, precs, reps=10):
    """The work-list sizes the library's makespan model picks at finalize
    against the measured best of the same candidate sizes: for each
    candidate m (the model's candidates: 256 m forward workgroups, 256 m
    adjoint split-K workgroups -- 512 m for the 128-tile split adjoint) the
    forward and adjoint launch times of a Phi + grad evaluation at P3, then
    the model's own choice.  Reported per direction: the model's time over
    the best candidate's."""
    import torch
    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context
    rows = []
    for c in configs:
        ds = synth.make_config(c)
        img_np = synth.eval_images(ds, "P3")
        md = "shared" if ds.shared else "cube"
        if md == "shared":
            img_np = img_np[:1]
        for prec in precs:
            def run(env):
                old = {k: os.environ.get(k) for k in ("UVMEM_FWD_WGS", "UVMEM_ADJ_WGS")}
                os.environ.update(env)
                try:
                    ctx = Context.from_dataset(ds, prec, mode=md)
                finally:
                    for k, v in old.items():
                        if v is None:
                            os.environ.pop(k, None)
                        else:
                            os.environ[k] = v
                img = torch.tensor(img_np, dtype=ctx.dtype, device=ctx.device)
                ev, fwd, adj = _median_eval_ms(ctx, img, reps=reps)
                info = ctx.info()
                ctx.close()
                return {"ms_eval": ev, "ms_forward": fwd, "ms_adjoint": adj, "fwd_wgs": info["n_fwd_wgs"],
                        "adj_wgs": info["n_adj_items"], "adj_tile": info["adj_tile"]}
            model = run({})
            slots = 512 if prec in ("bf16x3", "fp16x3") and model["adj_tile"] == 128 else 256
            cands = {}
            for m in SCHED_CANDIDATES:
                cands[m] = run({"UVMEM_FWD_WGS": str(256 * m), "UVMEM_ADJ_WGS": str(slots * m)})
            best_f = min(cands.values(), key=lambda r: r["ms_forward"])
            best_a = min(cands.values(), key=lambda r: r["ms_adjoint"])
            row = {"config": f"c{c}", "precision": prec, "model": model,
                   "candidates": {str(m): {k: v for k, v in r.items() if k != "adj_tile"} for m, r in cands.items()},
                   "forward_model_over_best": model["ms_forward"] / best_f["ms_forward"],
                   "adjoint_model_over_best": model["ms_adjoint"] / best_a["ms_adjoint"],
                   "best_forward_wgs": best_f["fwd_wgs"], "best_adjoint_wgs": best_a["adj_wgs"]}
            rows.append(row)
            print(json.dumps(row), flush=True)
    return rows


def centred_region(n, frac):
    """Boolean n x n mask of the centred square of side frac * n."""
    import numpy as np
    m = np.zeros((n, n), bool)
    h = int(round(frac * n / 2))
    m[n // 2 - h:n // 2 + h, n // 2 - h:n // 2 + h] = True
    return m


def cg_compare(c, precs, iters=None, mode=None, region=None, quiet=False):
    """M2: T graph-replayed projected-CG iterations from I = M in each
    precision; iterations/s, and the relative error of Phi_T and of the final
    image against the FP64 trajectory (the FP64 forward and adjoint are held
    to 1e-12 of the oracle at these sizes by the full-size parity tests)."""
    import numpy as np
    import torch
    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context
    ds = synth.make_config(c)
    T = iters or ds.cg_iters
    res = {}
    ref = None
    reg = centred_region(ds.n, region) if region else None
    for prec in ["fp64"] + [p for p in precs if p != "fp64"]:
        ctx = Context.from_dataset(ds, prec, mode=mode, region=reg)
        I = ctx.image()
        ctx.cg_init(I, init_to_floor=True)
        ctx.cg_run(I, 1, graph=True)          # capture (and one iteration)
        ctx.cg_init(I, init_to_floor=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        hist = ctx.cg_run(I, T, graph=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ctx.check()
        ms = e0.elapsed_time(e1)
        phi = hist[-1, :, 0].double().sum().item()
        img = I.double().cpu().numpy()
        row = {"config": f"c{c}", "mode": ctx.mode, "region_side": region, "precision": prec, "iters": T, "ms": ms, "cg_iters_per_s": T / (ms / 1e3),
               "vis_pixel_evals_per_s": ds.pairs * T / (ms / 1e3), "phi_T": phi}
        if prec == "fp64":
            ref = (phi, img)
        else:
            row["rel_err_phi_T_vs_fp64"] = abs(phi - ref[0]) / abs(ref[0])
            row["rel_err_image_T_vs_fp64"] = float(np.linalg.norm(img - ref[1]) / np.linalg.norm(ref[1]))
        res[prec] = row
        print(json.dumps(row), file=sys.stderr if quiet else sys.stdout, flush=True)
        ctx.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=5, help="workload configuration (1..6)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3", "fp16x3"])
    ap.add_argument("--graph", action="store_true", help="replay the step as a HIP graph")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP64-referenced errors and the split-precision companion runs")
    ap.add_argument("--no-cg", action="store_true",
                    help="skip the full CG trajectories (FP64 reference, FP32, bf16x3, fp16x3)")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,fp16x3",
                    help="precisions of --eval-sweep")
    ap.add_argument("--eval-sweep", default="", metavar="CONFIGS",
                    help="only time single Phi + grad evaluations on these configurations (e.g. 1,2,3,4,5)")
    ap.add_argument("--cg-compare", type=int, default=0, metavar="CONFIG",
                    help="only run the configuration's CG iterations in every precision vs FP64")
    ap.add_argument("--mode", default=None, choices=["cube", "shared"],
                    help="image model of --eval-sweep and --cg-compare: an image per channel, or one image "
                         "fitted to every channel (default: shared for the mosaic workload, cube otherwise)")
    ap.add_argument("--grid-error", default="", metavar="CONFIGS",
                    help="only compare the gridded model (Alg. 1) with the exact DFT on these configurations")
    ap.add_argument("--grid-cg", type=int, default=0, metavar="CONFIG",
                    help="only run CG with the exact and the gridded models and score the images exactly")
    ap.add_argument("--oversample", default="1,2,4", help="gridded-model oversampling factors")
    ap.add_argument("--region", type=float, default=0.0,
                    help="--cg-compare with a focus-of-attention region: centred square of this side fraction")
    ap.add_argument("--schedule-sweep", default="", metavar="CONFIGS",
                    help="only compare the finalize-time schedule choice with the measured best candidate")
    ap.add_argument("--mfma-peak", action="store_true",
                    help="only measure the matrix-core rate of each instruction form used (microbenchmark)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (no multi-GPU path); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.eval_sweep:
        eval_sweep([int(x) for x in args.eval_sweep.split(",")], args.precisions.split(","), mode=args.mode)
        return
    if args.grid_error:
        grid_error([int(x) for x in args.grid_error.split(",")], [int(x) for x in args.oversample.split(",")])
        return
    if args.grid_cg:
        grid_cg(args.grid_cg, [int(x) for x in args.oversample.split(",")])
        return
    if args.cg_compare:
        cg_compare(args.cg_compare, ["fp32", "bf16x3", "fp16x3"], mode=args.mode, region=args.region or None)
        return
    if args.schedule_sweep:
        schedule_sweep([int(x) for x in args.schedule_sweep.split(",")], ["fp32", "bf16x3"])
        return
    if args.mfma_peak:
        for k, v in mfma_peak().items():
            print(json.dumps({"form": k, **v}), flush=True)
        return
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)
        return

    from paper_1703_02920_amd import synth
    from paper_1703_02920_amd.uvmem import Context

    torch.cuda.set_device(0)
    print(f"bench: generating workload c{args.config}", file=sys.stderr, flush=True)
    ds = synth.make_config(args.config)
    ctx = Context.from_dataset(ds, args.precision)
    print(f"bench: {ds.description}; {args.precision} CG steps", file=sys.stderr, flush=True)
    ms, t_wall, kern = run_steps(ctx, args.steps, args.warmup, args.graph)
    pairs = ds.pairs
    value = pairs * args.steps / (ms / 1e3)
    flops_per_launch = 4.0 * pairs          # complex twiddle x real pixel (fwd) / Re(complex x complex) (adj)
    roof = None
    if kern:
        dom = max(kern, key=kern.get)
        achieved = flops_per_launch / (kern[dom] / 1e3) / 1e12
        workload = f"c{args.config}-{args.precision}"
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.precision], "unit": "TFLOP/s",
                "frac": achieved / PEAK[args.precision],
                "traffic": traffic_from_profiles(KERNELS[args.precision][0 if dom == "forward" else 1],
                                                 workload),
                "kernel": KERNELS[args.precision][0 if dom == "forward" else 1], "direction": dom,
                "kernel_ms": kern[dom], "flops_per_launch": flops_per_launch,
                "other_kernel_ms": {k: v for k, v in kern.items() if k != dom}}
    if roof is not None:
        try:
            pk = mfma_peak([{"fp32": "fp32", "fp64": "fp64", "bf16x3": "bf16", "fp16x3": "fp16"}[args.precision]])
            pk = next(iter(pk.values()))
            roof["measured_peak"] = pk["tflops"]
            roof["frac_of_measured_peak"] = roof["achieved"] / pk["tflops"]
            roof["measured_peak_instruction"] = pk["instruction"]
        except (OSError, RuntimeError) as exc:
            roof["measured_peak"] = None
            print(f"bench: no matrix-core microbenchmark ({exc})", file=sys.stderr, flush=True)
    # errors against the FP64 path (held to the oracle at 1e-12 at this size
    # by the full-size parity tests), and the split-precision companions
    errors, mixed, cg = None, None, None
    if not args.no_mixed and args.precision != "fp64":
        print("bench: FP64 reference evaluations", file=sys.stderr, flush=True)
        ref = Context.from_dataset(ds, "fp64")
        errors = eval_error(ds, ctx, ref)
        if args.precision == "fp32":
            mixed = {}
            for mp in ("bf16x3", "fp16x3"):
                print(f"bench: split-precision ({mp}) CG steps", file=sys.stderr, flush=True)
                mctx = Context.from_dataset(ds, mp)
                mms, _, mkern = run_steps(mctx, args.steps, args.warmup, args.graph)
                mixed[mp] = {"value": pairs * args.steps / (mms / 1e3),
                             "ms_per_step": mms / args.steps, "cg_iters_per_s": args.steps / (mms / 1e3),
                             "kernel_ms": mkern,
                             "mfma_frac_16bit_algorithmic": {k: flops_per_launch / (v / 1e3) / 1e12 / PEAK[mp]
                                                             for k, v in mkern.items()},
                             "mfma_frac_3_product_issued": {k: 3 * flops_per_launch / (v / 1e3) / 1e12 / PEAK[mp]
                                                            for k, v in mkern.items()},
                             "mfma_frac_3_product_of_measured_peak": mixed_measured(mp, mkern, flops_per_launch),
                             "rel_err_vs_fp64": eval_error(ds, mctx, ref)}
                mctx.close()
        ref.close()
    if not args.no_cg and args.precision == "fp32":
        print(f"bench: {ds.cg_iters}-iteration CG trajectories, FP64 reference and each precision",
              file=sys.stderr, flush=True)
        ctx.close()
        cg = cg_compare(args.config, ["fp32", "bf16x3", "fp16x3"], quiet=True)
    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(ds)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vis·pixel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3", "fp16x3": "fp16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": ds.description + "; one projected-CG iteration per step",
                   "n": ds.n, "channels": ds.n_chan, "visibilities": ds.total_vis,
                   "pairs_per_pass": pairs, "precision": args.precision,
                   "graph": bool(args.graph), "parallelism": "single GPU"},
        "cg_iters_per_s": args.steps / (ms / 1e3),
        "wall_s": t_wall,
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_err_vs_fp64": errors,
        "mixed": mixed,
        "cg_trajectories": cg,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
