#!/usr/bin/env python3
"""Throughput benchmark of the Gauss-polynomial bilateral filter on one MI355X.

Headline (`value`): GP forward in Mpix/s on the 1024x1024 synthetic image
(Voronoi, 200 cells, noise 10) over the spatial sweep sigma_s in {2, 5, 10, 20},
sigma_r 30, degree 20.  One step = the four forwards; value = pixels filtered
per second over the timed steps, inputs resident in HBM.

Also reported under "modes": Mpix/s per sigma_s, the direct filter of eq. (1)
per sigma_s, the 16-MP forward (4096x4096, sigma_s 10, sigma_r 20), the
batched and forward+backward modes, and max abs errors against the FP64
oracle and the direct filter.  `roofline` is for the kernel with the largest
share of the timed region, from per-launch HIP events on the stream the
library launches on.  `cpu_baseline` times the FP64 oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s of Gauss-poly bilateral (fwd, fwd+bwd, batched) vs direct; max abs err"
SWEEP = (2.0, 5.0, 10.0, 20.0)
SIGMA_R = 30.0
DEGREE = 20
HBM_PEAK_GBS = 8000.0


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="comma list of sections to run (headline always runs)")
    return ap.parse_args()


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps  # ms per call


# MI355X's published FP32 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 (packed
# FP32, two lanes' worth per instruction) x FMA (2 flops) x 2.4 GHz.  This
# build issues no packed FP32 instructions, so the rate its kernels can reach
# is half of it, the unpacked figure (one FMA per lane per clock).
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6


def step_model(kernel, C, band, fir_radii, n_iir, n_calls, HW):
    """Algorithmic HBM bytes and FP32 flops of one step of the sweep for one
    kernel: every kernel of a forward covers the whole image; fir_radii lists
    the FIR radii of the step, n_iir counts its recursive forwards."""
    rec = 32 * C  # 2 directions x 2 second-order sections x (2 input + 2 feedback taps) x 2 flops
    per = {
        "k_stats": (4 * n_calls, 0),
        "k_fir": ((4 + 4) * len(fir_radii), sum(4 * (2 * r + 1) * C for r in fir_radii)),
        "k_vband_agg": ((4 + 32 * C / band) * n_iir, rec * n_iir),
        "k_vresolve": (2 * 32 * C / band * n_iir, 0),
        "k_vband": ((4 + 4 * C + 32 * C / band) * n_iir, rec * n_iir),
        "k_hrow": ((4 * C + 4 + 4) * n_iir, rec * n_iir),
        "k_direct": (8 * n_calls, 0),
    }.get(kernel)
    if per is None:
        return None, None
    return per[0] * HW, per[1] * HW


def launch_ids(stage, bf, H, W, C, fir_radii):
    """(kernel instantiation, grid threads) of every launch of `stage` in one
    step, as the counter files name them (the launch shapes the library
    chooses, restated here)."""
    if stage == "k_fir":
        return [(f"k_fir<{r}, false>", ((W + fir_tx(r) - 1) // fir_tx(r)) * ((H + fir_ty(r) - 1) // fir_ty(r)) * 256)
                for r in fir_radii]
    sh = bf.iir_shape(H, W, C - 2)
    B, G, L, T, Gr = sh["band_rows"], sh["col_groups"], sh["row_chunk"], sh["row_threads"], sh["row_groups"]
    # stack pitch: the width rounded up to 4 plus the row passes' reach
    # (16 + 2 columns at most), rounded up to 32
    P = (((W + 3) // 4 * 4 + 16 + 2 + 31) // 32) * 32
    nb = (H + B - 1) // B
    cg = (W + 63) // 64
    # 32-row bands in 2..8 channel groups run as k_vbandg (the groups of a
    # band in one workgroup), with the same thread count; the end states come
    # from k_vagg (32-row bands: 2 or 4 interleaved groups, 256 threads for
    # one band (4 groups) or two (2 groups); 64-row bands: 4 groups, one band)
    vb = "k_vbandg" if B == 32 and 2 <= G <= 8 else "k_vband"
    ga = 2 if B == 32 and 2 * cg * nb >= 2048 and C <= 24 else 4
    agg = (f"k_vagg<{B}, {ga}, {4 // ga}>", (cg * nb if ga == 4 else (cg * nb + 1) // 2) * 256)
    return {
        "k_hrow": [(f"k_hrow2<{L}, false>", H * T * Gr)],
        "k_vband": [(f"{vb}<{B}, false, false>", ((P + 63) // 64) * nb * G * 64)],
        "k_vband_agg": [agg],
        "k_vresolve": [("k_vresolve", cg * 64 * C * 2)],
        "k_stats": [("k_stats", min(H, 256) * 256)],
    }.get(stage, [])


def fir_tx(r):
    """Columns of the FIR output tile for radius r (forward without saved terms)."""
    return 224 if r <= 16 else 64


def fir_ty(r):
    """Rows of the FIR output tile for radius r (forward without saved terms)."""
    return 8 if r <= 16 else (32 if r == 17 else 16)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU (one image, or one batch, per device); "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)
    only = set(filter(None, args.only.split(",")))

    def want(name):
        return not only or name in only

    import numpy as np
    import torch

    import paper_1505_00077_amd as bf
    import synthimg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, Wm = args.steps, args.warmup
    C = DEGREE + 2
    modes = {}

    # ---------------- headline: 1024^2 sweep ----------------
    log("generating 1024x1024 image")
    img = torch.from_numpy(synthimg.mid_1024()).to(dev)
    H, W = img.shape
    outs = {ss: torch.empty_like(img) for ss in SWEEP}
    # AUTO mode: FIR/IIR crossover measured on this device (cached per device)
    from paper_1505_00077_amd import autotune
    t0 = time.time()
    crossover = autotune.ensure(DEGREE, log=log)
    log(f"crossover table {crossover} ({time.time() - t0:.1f} s)")
    wss = {ss: bf.workspace(H, W, DEGREE, ss, "auto") for ss in SWEEP}
    plan = {ss: bf.resolve_spatial(ss, shape=(H, W)) for ss in SWEEP}
    band = bf.iir_shape(H, W, DEGREE)["band_rows"]

    def step():
        for ss in SWEEP:
            bf.gp_forward(img, ss, SIGMA_R, DEGREE, out=outs[ss], ws=wss[ss])

    log(f"headline: {K} steps of the sigma_s sweep {SWEEP} ({plan})")
    for _ in range(Wm):
        step()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(K):
        step()
    e.record()
    torch.cuda.synchronize()
    ms_step = s.elapsed_time(e) / K
    px_step = len(SWEEP) * H * W
    value = px_step / (ms_step * 1e-3) / 1e6
    for ss in SWEEP:
        if bf.status(wss[ss]) != bf.BF_OK:
            raise RuntimeError(f"device status not OK at sigma_s={ss}")
    # the same K steps again with a HIP event pair around every kernel launch
    # (recorded by the library on the stream it launches on); the events
    # themselves slow the step, so the headline above is taken without them
    bf.profile_enable(True)
    s.record()
    for _ in range(K):
        step()
    e.record()
    torch.cuda.synchronize()
    stage_t = bf.profile_collect(with_threads=True)
    stage = {k: v[:2] for k, v in stage_t.items()}
    bf.profile_enable(False)
    ms_step_profiled = s.elapsed_time(e) / K

    # dominant kernel of the step, against the roofline that binds it: the
    # higher of its algorithmic HBM-byte and FP32-flop fractions
    kname, (kcount, kms) = max(stage.items(), key=lambda kv: kv[1][1])
    avg_ms = kms / kcount
    fir_radii = [bf.fir_radius(ss) for ss in SWEEP if plan[ss] == "fir"]
    n_iir = sum(1 for ss in SWEEP if plan[ss] == "iir")
    bytes_step, flops_step = step_model(kname, C, band, fir_radii, n_iir, len(SWEEP), H * W)
    per_launch = K / kcount  # launches of this kernel per step, inverted
    gbs = bytes_step * per_launch / (avg_ms * 1e-3) / 1e9 if bytes_step else None
    tflops = flops_step * per_launch / (avg_ms * 1e-3) / 1e12 if flops_step else None
    f_hbm = gbs / HBM_PEAK_GBS if gbs else 0.0
    f_alu = tflops / FP32_PEAK_TFLOPS if tflops else 0.0
    # measured HBM traffic of the same kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    # calibrated by a device copy), valid only for the sources it was taken with
    from paper_1505_00077_amd import profiling
    traffic = profiling.traffic_for(os.path.join(ROOT, "profiles", "traffic_counters.json"),
                                    launch_ids(kname, bf, H, W, C, fir_radii))
    common = {"kernel": kname, "traffic": (traffic / (avg_ms * 1e-3) / 1e9) if traffic else None,
              "traffic_bytes_per_launch": traffic,
              "algorithmic_bytes_per_launch": bytes_step * per_launch if bytes_step else None,
              "algorithmic_fp32_flops_per_launch": flops_step * per_launch if flops_step else None,
              "avg_launch_ms": avg_ms, "launches": kcount, "share_of_profiled_step": kms / (ms_step_profiled * K),
              "hbm_frac": f_hbm, "fp32_frac": f_alu,
              "fp32_unpacked_peak": FP32_UNPACKED_PEAK_TFLOPS,
              "fp32_unpacked_frac": tflops / FP32_UNPACKED_PEAK_TFLOPS if tflops else 0.0}
    if f_alu > f_hbm:
        roofline = {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": f_alu, **common}
    else:
        roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": f_hbm, **common}
    modes["stages_ms_per_step"] = {k: v[1] / K for k, v in sorted(stage.items())}
    modes["profiled_ms_per_step"] = ms_step_profiled

    # ---------------- per-sigma_s forward and direct ----------------
    if want("sweep"):
        per = {}
        for ss in SWEEP:
            ms = timed(lambda: bf.gp_forward(img, ss, SIGMA_R, DEGREE, out=outs[ss], ws=wss[ss]), K, Wm, torch)
            per[str(ss)] = {"plan": plan[ss], "ms": ms, "mpix_s": H * W / (ms * 1e-3) / 1e6}
            log(f"gp sigma_s={ss}: {ms:.3f} ms")
        # the two spatial modes are different filters: their difference on the
        # sweep image wherever both exist (the FIR tile reaches radius 24)
        fvi = {}
        for ss in SWEEP:
            if bf.fir_radius(ss) <= bf.FIR_MAX_RADIUS:
                a = bf.gp_forward(img, ss, SIGMA_R, DEGREE, spatial="fir")
                b = bf.gp_forward(img, ss, SIGMA_R, DEGREE, spatial="iir")
                fvi[str(ss)] = float((a - b).abs().max())
        per["fir_vs_iir_max_abs"] = fvi
        modes["gp_forward_1024_per_sigma_s"] = per
        dper = {}
        dout = torch.empty_like(img)
        for ss in SWEEP:
            n = max(1, min(K, 5))
            ms = timed(lambda: bf.direct_forward(img, ss, SIGMA_R, out=dout), n, 1, torch)
            dper[str(ss)] = {"window": bf.fir_radius(ss), "ms": ms, "mpix_s": H * W / (ms * 1e-3) / 1e6}
            log(f"direct sigma_s={ss}: {ms:.3f} ms")
            # agreement of the GP output with the direct filter (reported, not gated)
            d = (outs[ss] - dout).abs()
            dper[str(ss)]["gp_vs_direct_max_abs"] = float(d.max())
            dper[str(ss)]["gp_vs_direct_mse_db"] = float(10 * torch.log10((d.double() ** 2).mean()))
        modes["direct_1024_per_sigma_s"] = dper

    # ---------------- 16 MP forward ----------------
    if want("large"):
        log("generating 4096x4096 image")
        big = torch.from_numpy(synthimg.large_4096()).to(dev)
        bws = bf.workspace(4096, 4096, DEGREE, 10.0, "auto")
        bout = torch.empty_like(big)
        ms = timed(lambda: bf.gp_forward(big, 10.0, 20.0, DEGREE, out=bout, ws=bws), K, Wm, torch)
        bf.profile_enable(True)  # a second pass with per-launch events
        timed(lambda: bf.gp_forward(big, 10.0, 20.0, DEGREE, out=bout, ws=bws), K, 0, torch)
        bstage = bf.profile_collect()
        bf.profile_enable(False)
        if bf.status(bws) != bf.BF_OK:
            raise RuntimeError("device status not OK on the 16-MP image")
        mp = 4096 * 4096
        kn, (kc, kt) = max(bstage.items(), key=lambda kv: kv[1][1])
        # average per launch
        kb, _ = step_model(kn, C, bf.iir_shape(4096, 4096, DEGREE)["band_rows"], [], 1, 1, 1)
        model_bytes = (12 + 8 * C) * mp
        modes["gp_forward_4096"] = {
            "plan": bf.resolve_spatial(10.0, shape=(4096, 4096)), "ms": ms, "mpix_s": mp / (ms * 1e-3) / 1e6,
            "iir_shape": bf.iir_shape(4096, 4096, DEGREE),
            "model_bytes_per_px": 12 + 8 * C,
            "model_frac_of_hbm_peak": model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "stages_ms_per_call": {k: v[1] / v[0] for k, v in sorted(bstage.items())},
            "dominant_kernel": kn, "dominant_kernel_gbs": (kb * mp / (kt / kc * 1e-3) / 1e9) if kb else None,
        }
        log(f"16MP: {ms:.3f} ms")
        del big, bws, bout


    batch_samples, batch = [], []
    # ---------------- batched: a graph of grouped per-stage launches ----------------
    if want("batched"):
        log("generating the 64-image batch")
        batch = synthimg.batched_64()
        bimgs = [torch.from_numpy(b[0]).to(dev) for b in batch]
        bss = [b[1] for b in batch]
        bsr = [b[2] for b in batch]
        npx = sum(x.numel() for x in bimgs)
        # the plan's launch shape (band height, channel groups of its recursive
        # images) is the tuner's choice for this batch, cached by composition
        from paper_1505_00077_amd import autotune
        plan_b, plan_shape = autotune.plan_batch(bimgs, bss, bsr, DEGREE, log=log)
        plan_b.run()
        torch.cuda.synchronize()
        graph = plan_b.graph()
        ms_graph = timed(graph.replay, K, Wm, torch)
        souts = [torch.empty_like(x) for x in bimgs]
        swss = [bf.workspace(x.shape[0], x.shape[1], DEGREE, s) for x, s in zip(bimgs, bss)]
        # the batch descriptors hold float32 sigmas; the sequential calls use the same values
        bss32 = [float(np.float32(v)) for v in bss]
        bsr32 = [float(np.float32(v)) for v in bsr]

        def seq():
            for x, o, w, s_, r_ in zip(bimgs, souts, swss, bss32, bsr32):
                bf.gp_forward(x, s_, r_, DEGREE, out=o, ws=w)

        ms_seq = timed(seq, K, Wm, torch)
        bf.profile_enable(True)  # per-stage durations of the batched launches (eager, with events)
        timed(plan_b.run, K, 0, torch)
        bstages = {k: v[1] / K for k, v in sorted(bf.profile_collect().items())}
        bf.profile_enable(False)
        # the same single calls made under the plan's launch shape give the
        # plan's bits (with their own default shapes they differ by rounding,
        # which ill-conditioned images, small sigma_r at N 20, amplify)
        worst_default = max(float((a - b).abs().max()) for a, b in zip(plan_b.outs, souts))
        try:
            bf.set_iir_tuning(*plan_shape)
            swss = [bf.workspace(x.shape[0], x.shape[1], DEGREE, s) for x, s in zip(bimgs, bss)]
            seq()
            torch.cuda.synchronize()
        finally:
            bf.set_iir_tuning(0, 0, 0)
        worst = max(float((a - b).abs().max()) for a, b in zip(plan_b.outs, souts))
        # sampled outputs (image corner and centre) for the oracle leg, and the
        # degree rule's verdict per image (eqs. (4)-(5) at N 20)
        batch_samples = []
        for i, (b, o) in enumerate(zip(batch, plan_b.outs)):
            Hb, Wb = b[0].shape
            pts = [(0, 0), (Hb // 2, Wb // 2)]
            vals = [float(o[y, x]) for y, x in pts]
            xmax = float(np.max(np.abs(b[0].astype(np.float64) - b[0].astype(np.float64).mean()))) / b[2]
            try:
                rule = bf.degree_for(xmax, 1e-3)
            except bf.BfError:
                rule = None
            batch_samples.append({"image": i, "shape": [Hb, Wb], "sigma_s": b[1], "sigma_r": b[2],
                                  "plan": bf.resolve_spatial(b[1], shape=(Hb, Wb)), "xmax": xmax,
                                  "rule_N_eps_1e-3": rule, "points": pts, "gpu": vals})
        modes["batched_64"] = {"images": len(bimgs), "megapixels": npx / 1e6, "ms_graph": ms_graph,
                               "mpix_s_graph": npx / (ms_graph * 1e-3) / 1e6, "ms_sequential": ms_seq,
                               "mpix_s_sequential": npx / (ms_seq * 1e-3) / 1e6,
                               "plan_shape": {"band_rows": plan_shape[0], "col_groups": plan_shape[1],
                                              "row_groups": plan_shape[2]},
                               "max_abs_diff_vs_sequential": worst,
                               "sequential_shapes": "timed with each image's own default launch shape; the "
                                                    "difference is taken against single calls under the plan's "
                                                    "shape (bit-identical when 0)",
                               "max_abs_diff_vs_sequential_default_shapes": worst_default,
                               "stages_ms": bstages,
                               "plans": {m: sum(1 for x, s_ in zip(bimgs, bss)
                                                if bf.resolve_spatial(s_, shape=x.shape) == m) for m in ("fir", "iir")}}
        log(f"batched: graph {ms_graph:.3f} ms, sequential {ms_seq:.3f} ms")
        del plan_b, graph, bimgs, souts, swss

    # ---------------- forward + backward: 16 x 512^2, sigma_r 25 ----------------
    # sigma_s 4 (the gradient workload; FIR, radius 12) and sigma_s 10 (past the
    # FIR radius limit: the recursive mode, whose backward differentiates
    # Deriche's recursion exactly)
    if want("fwdbwd"):
        imgs_np, tgt_np = synthimg.grad_batch()
        gimgs = torch.from_numpy(imgs_np).to(dev)
        tgt = torch.from_numpy(tgt_np).to(dev)
        B_, H_, W_ = gimgs.shape
        sr_g = 25.0
        saved = torch.empty(B_, 16 * H_ * W_, dtype=torch.uint8, device=dev)
        fout = torch.empty_like(gimgs)
        gout = torch.empty_like(gimgs)
        gimg = torch.empty_like(gimgs)
        gls = torch.zeros(B_, dtype=torch.float64, device=dev)
        glr = torch.zeros(B_, dtype=torch.float64, device=dev)
        stream = bf._stream(dev)
        npx = B_ * H_ * W_
        for key, ss_g, mode in (("fwd_bwd_16x512", 4.0, "fir"), ("fwd_bwd_16x512_sigma_s10_iir", 10.0, "iir")):
            fws = bf.workspace(H_, W_, DEGREE, ss_g, mode)
            bws = bf.backward_workspace(H_, W_, DEGREE, ss_g, mode)
            flags = bf._flags(mode)
            # the stacked calls: every stage one launch over the 16 images
            sfws = torch.empty(bf.bf_gp_forward_stacked_workspace_bytes(B_, H_, W_, DEGREE, ss_g, flags),
                               dtype=torch.uint8, device=dev)
            sbws = torch.empty(bf.bf_gp_backward_stacked_workspace_bytes(B_, H_, W_, DEGREE, ss_g, flags),
                               dtype=torch.uint8, device=dev)

            def fwd_bwd():
                bf._check(bf.bf_gp_forward_stacked(gimgs.data_ptr(), fout.data_ptr(), B_, H_, W_, W_, H_ * W_, ss_g,
                                                   sr_g, DEGREE, flags, saved.data_ptr(), sfws.data_ptr(),
                                                   sfws.numel(), stream), "stacked forward")
                torch.sub(fout, tgt, out=gout)
                bf._check(bf.bf_gp_backward_stacked(gimgs.data_ptr(), gout.data_ptr(), saved.data_ptr(), B_, H_, W_,
                                                    W_, H_ * W_, ss_g, sr_g, DEGREE, flags, gimg.data_ptr(),
                                                    gls.data_ptr(), glr.data_ptr(), sbws.data_ptr(), sbws.numel(),
                                                    stream), "stacked backward")

            def fwd_only():
                bf._check(bf.bf_gp_forward_stacked(gimgs.data_ptr(), fout.data_ptr(), B_, H_, W_, W_, H_ * W_, ss_g,
                                                   sr_g, DEGREE, flags, None, sfws.data_ptr(), sfws.numel(), stream),
                          "stacked forward")

            # the same work as 16 single-image calls of each pass
            def fwd_bwd_single():
                for i in range(B_):
                    bf.gp_forward(gimgs[i], ss_g, sr_g, DEGREE, spatial=mode, out=fout[i], ws=fws, saved=saved[i])
                    torch.sub(fout[i], tgt, out=gout[i])
                    bf._check(bf.bf_gp_backward(gimgs[i].data_ptr(), gout[i].data_ptr(), saved[i].data_ptr(), H_,
                                                W_, W_, ss_g, sr_g, DEGREE, flags, gimg[i].data_ptr(),
                                                gls[i:].data_ptr(), glr[i:].data_ptr(), bws.data_ptr(), bws.numel(),
                                                stream), "backward")

            ms_single = timed(fwd_bwd_single, K, Wm, torch)
            ms_fb = timed(fwd_bwd, K, Wm, torch)
            ms_f = timed(fwd_only, K, Wm, torch)
            modes[key] = {"ms": ms_fb, "mpix_s": npx / (ms_fb * 1e-3) / 1e6, "fwd_only_ms": ms_f,
                          "fwd_only_mpix_s": npx / (ms_f * 1e-3) / 1e6, "ms_single_image_calls": ms_single,
                          "plan": mode, "sigma_s": ss_g, "launches": "stacked (one per stage over the 16 images)",
                          "grad_log_sigma_s_sum": float(gls.sum()), "grad_log_sigma_r_sum": float(glr.sum())}
            log(f"fwd+bwd {mode} sigma_s {ss_g}: {ms_fb:.3f} ms stacked (fwd only {ms_f:.3f} ms), "
                f"{ms_single:.3f} ms as single-image calls")
            del fws, bws, sfws, sbws

    # ---------------- joint (cross) filter: 1024^2, guide and data images ----------------
    if want("joint"):
        guide = torch.from_numpy(synthimg.mid_1024()).to(dev)
        jdata = torch.from_numpy(synthimg.voronoi_image(1024, 1024, 300, seed=12)).to(dev)
        jout = torch.empty_like(guide)
        jres = {}
        for ss_j in (2.0, 10.0):
            jws = bf.joint_workspace(1024, 1024, DEGREE, ss_j)
            ms_j = timed(lambda: bf.gp_joint_forward(guide, jdata, ss_j, SIGMA_R, DEGREE, out=jout, ws=jws), K, Wm,
                         torch)
            jres[str(ss_j)] = {"ms": ms_j, "mpix_s": guide.numel() / (ms_j * 1e-3) / 1e6, "plan": "iir",
                               "channels": 2 * (DEGREE + 1)}
            del jws
        modes["joint_1024"] = jres
        log("joint 1024^2: " + ", ".join(f"sigma_s {k} {v['ms']:.3f} ms" for k, v in jres.items()))

    # ---------------- video: 64 frames of 512^2 (16.8 M voxels) ----------------
    if want("video"):
        frames = torch.from_numpy(np.stack([synthimg.voronoi_image(512, 512, 200, seed=700 + t)
                                            for t in range(64)])).to(dev).contiguous()
        vout = torch.empty_like(frames)
        vws = bf.volume_workspace(64, 512, 512, DEGREE, 10.0, 3.0)
        ms_v = timed(lambda: bf.gp_volume_forward(frames, 10.0, 3.0, SIGMA_R, DEGREE, out=vout, ws=vws), K, Wm, torch)
        modes["video_64x512x512"] = {"ms": ms_v, "mvox_s": frames.numel() / (ms_v * 1e-3) / 1e6, "plan": "iir",
                                     "sigma_s": 10.0, "sigma_t": 3.0, "sigma_r": SIGMA_R}
        log(f"video 64x512x512: {ms_v:.3f} ms")
        del frames, vout, vws

    # ---------------- box spatial kernel: running sums, O(1) in the radius ----------------
    # the 1024^2 sweep image at the headline's sigma_s, and the 16-MP image; the
    # two passes move 4 + 4C (column pass) and 4C + 8 (row pass) bytes per
    # pixel, so the per-kernel rates are against HBM
    if want("box"):
        mid = torch.from_numpy(synthimg.mid_1024()).to(dev)
        xout = torch.empty_like(mid)
        xres = {}
        for ss_b in SWEEP:
            xws = bf.workspace(1024, 1024, DEGREE, ss_b, "box")
            ms_b = timed(lambda: bf.gp_forward(mid, ss_b, SIGMA_R, DEGREE, spatial="box", out=xout, ws=xws), K, Wm,
                         torch)
            xres[str(ss_b)] = {"ms": ms_b, "mpix_s": mid.numel() / (ms_b * 1e-3) / 1e6,
                               "radius": bf.fir_radius(ss_b)}
            del xws
        big = torch.from_numpy(synthimg.large_4096()).to(dev)
        bout = torch.empty_like(big)
        xws = bf.workspace(4096, 4096, DEGREE, 10.0, "box")
        ms_b = timed(lambda: bf.gp_forward(big, 10.0, 20.0, DEGREE, spatial="box", out=bout, ws=xws), K, Wm, torch)
        bf.profile_enable(True)
        timed(lambda: bf.gp_forward(big, 10.0, 20.0, DEGREE, spatial="box", out=bout, ws=xws), K, 0, torch)
        xstage = bf.profile_collect()
        bf.profile_enable(False)
        if bf.status(xws) != bf.BF_OK:
            raise RuntimeError("device status not OK on the 16-MP box run")
        mp = 4096 * 4096
        per_px = {"k_boxcol": 4 + 4 * C, "k_boxrow": 4 * C + 8, "k_stats": 4}
        kern = {}
        for k, (kc, kt) in sorted(xstage.items()):
            avg = kt / kc
            kern[k] = {"ms_per_call": avg,
                       "algorithmic_gbs": per_px[k] * mp / (avg * 1e-3) / 1e9 if k in per_px else None}
        modes["box_1024_per_sigma_s"] = xres
        modes["box_4096"] = {"ms": ms_b, "mpix_s": mp / (ms_b * 1e-3) / 1e6, "sigma_s": 10.0, "sigma_r": 20.0,
                             "model_bytes_per_px": 12 + 8 * C,
                             "model_frac_of_hbm_peak": (12 + 8 * C) * mp / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "kernels": kern}
        log("box 1024^2: " + ", ".join(f"sigma_s {k} {v['ms']:.3f} ms" for k, v in xres.items()) +
            f"; 16MP {ms_b:.3f} ms")
        del mid, xout, big, bout, xws

    # ---------------- degree study: error surface against the direct filter ----------------
    # GP in the FIR mode (window ceil(3 sigma_s), the direct filter's) against
    # eq. (1) computed directly on the GPU, max abs error over a 512^2 image,
    # beside the degree rule's choice for a weight tolerance of 1e-3
    if want("degree"):
        dimg_np = synthimg.voronoi_image(512, 512, 100, seed=9)
        dimg = torch.from_numpy(dimg_np).to(dev)
        study = []
        for ss_d in (2.0, 5.0):
            for sr_d in (10.0, 20.0, 30.0, 50.0):
                ref_d = bf.direct_forward(dimg, ss_d, sr_d)
                xmax = float(np.max(np.abs(dimg_np.astype(np.float64) - dimg_np.mean()))) / sr_d
                row = {"sigma_s": ss_d, "sigma_r": sr_d, "xmax": xmax, "max_abs_err": {}}
                try:
                    row["rule_N_eps_1e-3"] = bf.degree_for(xmax, 1e-3)
                except bf.BfError:
                    row["rule_N_eps_1e-3"] = None
                for Nd in (4, 8, 12, 16, 20, 24, 32, 40, 64):
                    got = bf.gp_forward(dimg, ss_d, sr_d, Nd, spatial="fir")
                    row["max_abs_err"][str(Nd)] = float((got - ref_d).abs().max())
                study.append(row)
        modes["degree_study_512"] = study
        log("degree study: " + "; ".join(f"ss {r['sigma_s']} sr {r['sigma_r']}: N20 {r['max_abs_err']['20']:.3g} "
                                          f"rule {r['rule_N_eps_1e-3']}" for r in study))

    # ---------------- copy calibration for the traffic counters ----------------
    if want("calib"):
        # a plain device-to-device copy of 256 MiB: its FETCH_SIZE / WRITE_SIZE
        # counters give the scale between counter readings and bytes moved
        nbytes = 256 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        ms = timed(lambda: dst.copy_(src), max(1, K // 2), 1, torch)
        modes["copy_calibration"] = {"bytes_each_way": nbytes, "ms": ms,
                                     "gbs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}
        del src, dst

    # ---------------- the FP64 oracle: CPU baseline, then accuracy ----------------
    # The only part of the benchmark that runs the oracle.  It is timed on one
    # step of the sweep (the CPU baseline); its outputs then give the GPU's
    # errors on the images the headline times, and it is run on the small
    # case and on sampled pixels of every image of the batch.
    cpu = None
    if not args.no_cpu:
        import oracle
        crop = synthimg.mid_1024().astype(np.float64)
        log("timing the FP64 oracle on one step of the sweep (the whole 1024x1024 image per sigma_s)")
        refs = {}
        t0 = time.perf_counter()
        for ss in SWEEP:
            k, _ = oracle.spatial_table(plan[ss], ss, *crop.shape)
            refs[ss] = oracle.gp_alg1(crop, SIGMA_R, DEGREE, k)
        dt = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        model = None
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), None)
        except OSError:
            pass
        cpu = {"value": len(SWEEP) * crop.size / dt / 1e6, "unit": "Mpix/s", "cores": cores, "kind": "oracle",
               "sample": "one step: the 1024x1024 image at each sigma_s of the sweep, same spatial mode, "
                         "FP64 Algorithm 1 (C, OpenMP)", "seconds": dt, "cpu_model": model}
        # the whole headline images against the oracle (the GPU outputs of the
        # last timed step, in the mode AUTO took under the tuned table)
        errs = {str(ss): float(np.max(np.abs(outs[ss].cpu().numpy().astype(np.float64) - refs[ss]))) for ss in SWEEP}
        modes["max_abs_err_vs_oracle_1024"] = errs
        if "gp_forward_1024_per_sigma_s" in modes:
            for ss in SWEEP:
                modes["gp_forward_1024_per_sigma_s"][str(ss)]["max_abs_err_vs_oracle"] = errs[str(ss)]
        log("max |gpu - oracle| on the 1024^2 sweep: " + ", ".join(f"sigma_s {k} {v:.2e}" for k, v in errs.items()))
        del refs
        # ---------------- accuracy on the small configuration ----------------
        if want("accuracy"):
            small = synthimg.small_256()
            f64 = small.astype(np.float64)
            ref_direct = oracle.direct_gauss(f64, 3.0, SIGMA_R)
            acc = {}
            for mode in ("fir", "iir", "box"):
                got = bf.gp_forward(torch.from_numpy(small).to(dev), 3.0, SIGMA_R, DEGREE, spatial=mode, check=True)
                g = got.cpu().numpy().astype(np.float64)
                k, _ = oracle.spatial_table(mode, 3.0, *small.shape)
                ref = oracle.gp_alg1(f64, SIGMA_R, DEGREE, k)
                # the box mode's own direct filter is eq. (1) with the box kernel
                rd = oracle.direct(f64, SIGMA_R, k) if mode == "box" else ref_direct
                acc[mode] = {"max_abs_err_vs_oracle": float(np.max(np.abs(g - ref))),
                             "max_abs_err_vs_direct": float(np.max(np.abs(g - rd))),
                             "mse_db_vs_direct": oracle.mse_db(g, rd)}
            gd = bf.direct_forward(torch.from_numpy(small).to(dev), 3.0, SIGMA_R).cpu().numpy().astype(np.float64)
            acc["direct"] = {"max_abs_err_vs_oracle": float(np.max(np.abs(gd - ref_direct)))}
            modes["accuracy_256_sigma_s3"] = acc

        # sampled pixels of every image of the batch (centre: the whole
        # image's FP64 mean; neighbourhood: the window, or 15 sigma_s of the
        # recursive kernel, beyond which its weights are below 1e-9 of the peak)
        if batch_samples:
            log("oracle on sampled pixels of the 64-image batch")
            per_img = []
            for rec, b in zip(batch_samples, batch):
                f = b[0].astype(np.float64)
                s32, r32 = float(np.float32(b[1])), float(np.float32(b[2]))
                tc = float(f.mean())
                reach = bf.fir_radius(s32) if rec["plan"] == "fir" else int(np.ceil(15 * s32))
                errs_i = []
                for (y, x), g in zip(rec["points"], rec["gpu"]):
                    y0, y1 = max(0, y - reach), min(f.shape[0], y + reach + 1)
                    x0, x1 = max(0, x - reach), min(f.shape[1], x + reach + 1)
                    c = f[y0:y1, x0:x1] - tc
                    if rec["plan"] == "fir":
                        kt = oracle.gauss_table(s32, bf.fir_radius(s32))
                    else:
                        kt = oracle.deriche_table(s32, max(1, max(c.shape) - 1))
                    ref = oracle.gp_alg1(c, r32, DEGREE, kt, oracle.CENTER_NONE)[y - y0, x - x0] + tc
                    errs_i.append(abs(g - ref))
                per_img.append({"image": rec["image"], "shape": rec["shape"], "plan": rec["plan"],
                                "sigma_s": rec["sigma_s"], "sigma_r": rec["sigma_r"], "xmax": rec["xmax"],
                                "rule_N_eps_1e-3": rec["rule_N_eps_1e-3"], "max_abs_err_vs_oracle": max(errs_i)})
            modes["batched_64"]["per_image_sampled"] = per_img
            modes["batched_64"]["sampled_max_abs_err_vs_oracle"] = max(p_["max_abs_err_vs_oracle"] for p_ in per_img)
            modes["batched_64"]["images_within_1e-3"] = sum(1 for p_ in per_img if p_["max_abs_err_vs_oracle"] <= 1e-3)
            modes["batched_64"]["images_the_rule_accepts_at_N20"] = sum(
                1 for p_ in per_img if p_["rule_N_eps_1e-3"] is not None and p_["rule_N_eps_1e-3"] <= DEGREE)

    # HBM fractions of the 16-MP runs: the two-pass model (12 + 8C B/px) against
    # the peak and against the measured copy rate, and the on-chip floor
    # (12 B/px: image reads and output write only) against the peak
    cal = modes.get("copy_calibration")
    for key in ("gp_forward_4096", "box_4096"):
        m = modes.get(key)
        if m:
            px = 4096 * 4096
            m["model_gbs"] = m["model_bytes_per_px"] * px / (m["ms"] * 1e-3) / 1e9
            m["onchip_floor_frac_of_hbm_peak"] = 12 * px / (m["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
            if cal:
                m["model_frac_of_copy_bw"] = m["model_gbs"] / cal["gbs_read_plus_write"]

    line = {
        "metric": METRIC, "value": value, "unit": "Mpix/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gp_forward 1024x1024 voronoi-200+noise10, sigma_s sweep {2,5,10,20}, sigma_r 30, "
                               "N 20 (one step = the four forwards)",
                   "global_batch": 1, "image": [H, W], "plan": {str(k): v for k, v in plan.items()},
                   "fir_crossover_table": crossover, "iir_shape": bf.iir_shape(H, W, DEGREE),
                   "recombination": "f64", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": modes,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
