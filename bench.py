#!/usr/bin/env python3
"""SPDHG epoch benchmark on one MI355X.

Workload (one step = one SPDHG epoch of Algorithm 2): mMR-shaped span-11 cylinder,
image 344 x 344 x 127 voxels at 2.08 mm, sinogram 344 radial x 252 angles x 837 planes
(72,557,856 bins, FP32); seeded brain-like ellipsoid phantom, randoms + scatter at 30 % of
the trues, 1e8 expected counts; TV prior beta = 2e-3 with non-negativity; 21 subsets of
equidistant angles; SPDHG+ (balanced sampling, preconditioned step sizes); an epoch is
42 iterations.  Inputs are generated on the GPU (analytic line integrals) and resident in
HBM before the timed region.

Prints one JSON line with epochs/s, the live roofline of the dominant kernel (HIP events
around each launch inside the timed region) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "mMR-size SPDHG epochs/s, proj+backproj GB/s; time to 1e-3 rel objective"
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE counters, valid only
# for the kernel sources they were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mmr_tv21.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1808_07150_amd", "csrc", f)
                  for f in ("kernels.hip", "geom.hpp", "spdhg.hip")]
COPY_BYTES = 256 << 20

# Workloads (one step = one epoch of Algorithm 2): mMR geometry, brain phantom, randoms +
# scatter at 30 % of the trues, SPDHG+ (balanced sampling, preconditioned steps).
# Algorithmic bytes per voxel of one prior launch: TV reads x, 3 duals, z, T and writes x,
# 3 duals, z (44 B); dTV also reads the 3-component field xi (56 B); a TGV launch is
# block n-1 (23 arrays) or block n (28 arrays), drawn equally often (102 B on average).
WORKLOADS = {
    "mmr-tv21": dict(m=21, prior="tv", counts=1e8, alpha=2e-3, alpha1=0.0, prior_bpv=44,
                     label="mMR 344x344x127 / 344x252x837 span-11, TV beta=2e-3 + nonneg, "
                           "21 subsets, SPDHG+ (balanced, preconditioned), 1e8 counts"),
    "mmr-tgv252": dict(m=252, prior="tgv", counts=3e7, alpha=2e-3, alpha1=1e-3, prior_bpv=102,
                       label="mMR 344x344x127 / 344x252x837 span-11, TGV alpha0=2e-3 "
                             "alpha1=1e-3 + nonneg, 252 single-angle subsets, SPDHG+, 3e7 counts"),
    "mmr-dtv252": dict(m=252, prior="dtv", counts=3e7, alpha=2e-3, alpha1=0.0, prior_bpv=56,
                       label="mMR 344x344x127 / 344x252x837 span-11, dTV beta=2e-3 eta=1e-2 "
                             "(MR-like side image) + nonneg, 252 single-angle subsets, "
                             "SPDHG+, 3e7 counts"),
    "mmr-span1-tv21": dict(m=21, prior="tv", counts=1e8, alpha=2e-3, alpha1=0.0, prior_bpv=44,
                           geometry="span1",
                           label="mMR span-1 344x344x127 / 344x252x4084 (64 rings, ring "
                                 "differences up to 60: 121 segments, 354M bins), TV "
                                 "beta=2e-3 + nonneg, 21 subsets, SPDHG+ (balanced, "
                                 "preconditioned), 1e8 counts"),
    "mmr-scanner-tv21": dict(m=21, prior="tv", counts=1e8, alpha=2e-3, alpha1=0.0, prior_bpv=44,
                             geometry="scanner",
                             label="mMR closer scanner model: span-11 data 344x252x837 as sums "
                                   "of the 4084 ring-pair planes (64 rings, ring differences up "
                                   "to 60), non-arc-corrected radial bins and s-dependent "
                                   "slopes on a 328 mm ring, detector gaps (1 in 9), image "
                                   "344x344x127, TV beta=2e-3 + nonneg, 21 subsets, SPDHG+, 1e8 "
                                   "counts"),
}
HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (256 CUs at 2.4 GHz, packed FP32 FMA); the kernels
# are built without packed-FP32 instructions, whose own ceiling is half of it (78.6)
ALU_PEAK_TFLOPS = 157.3
ALU_UNPACKED_TFLOPS = 78.6
SEED = 18080200


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind):
    """HBM bytes per launch of kernel kind `kind` from the counter summary, or None when
    the summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_digest() or f"{kind}_bytes_per_launch" not in kv:
        return None
    return float(kv[f"{kind}_bytes_per_launch"])


def copy_calibration(torch, dev):
    """A plain copy kernel of known size (COPY_BYTES read, COPY_BYTES written), launched
    4 times: the scale for the HBM byte counters."""
    src = torch.rand(COPY_BYTES // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(4):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def cpu_baseline(g, d_host, wl, seed):
    """The FP64 oracle (oracle/) on a bounded sample of the same workload: one data
    iteration (subset 0: forward, KL-dual prox, backprojection) and one iteration of each
    prior block at full mMR size, run by the oracle's own Algorithm 2 loop, scaled to the
    expected iterations of an epoch."""
    import numpy as np
    from oracle import spdhg as S
    m, prior = wl["m"], wl["prior"]

    class _Steps(S.Problem):  # the oracle problem without its (full-size) step setup
        def _setup_steps(self):
            self.sigma = [np.full(b.shape, 1e-3) for b in self.sub_b]
            self.prior_sigma = [0.1] * self.n_prior
            self.norms = [None] * self.n
            self.T = np.full(self.image_shape(), 1e-3)

    prob = _Steps(g, d_host["b"], d_host["r"], d_host["mult"], n_subsets=m, prior=prior,
                  alpha=wl["alpha"], alpha1=wl["alpha1"], sampling="balanced", precond=True,
                  side=d_host.get("side"))
    x0 = np.full(prob.image_shape(), 0.5)
    st = prob.new_state(x0)
    t0 = time.perf_counter()
    S.spdhg(prob, 1, seed, state=st, blocks=[0])
    t_data = time.perf_counter() - t0
    t_prior = []
    for j in range(prob.n_prior):
        t0 = time.perf_counter()
        S.spdhg(prob, 1, seed, state=st, blocks=[m + j])
        t_prior.append(time.perf_counter() - t0)
    ipe = prob.iters_per_epoch()
    per_epoch = t_data * ipe * sum(prob.p[:m]) + sum(
        t * ipe * prob.p[m + j] for j, t in enumerate(t_prior))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    prior_txt = " + ".join(f"{t:.1f} s" for t in t_prior)
    return {"value": 1.0 / per_epoch, "unit": "epochs/s", "cores": threads, "kind": "oracle",
            "sample": f"1 data iteration (subset 0: {t_data:.1f} s) + 1 iteration of each "
                      f"prior block ({prior_txt}) at full mMR size, FP64, scaled to "
                      f"{ipe * sum(prob.p[:m]):.0f} + {ipe * sum(prob.p[m:]):.0f} "
                      f"iterations/epoch"}


def reference_minimum(P, torch, g, d, wl, seed, ref_epochs=200, pdhg_iters=2000, split=0):
    """Psi* of the relative objective (Section 4): the paper computes it with thousands of
    deterministic PDHG iterations (Algorithm 1).  Here: spdhg_pdhg_iterate on a context
    with one data block (weights 1/2, 1/2) for pdhg_iters iterations, with its duality gap
    (box [0, U], U = 2 max x) as the certificate Psi(x_pdhg) - Psi_min <= gap; TGV, for
    which PDHG is not built and the box gap is infinite, uses ref_epochs epochs of SPDHG.
    With more than 21 subsets SPDHG's late phase is slow (single-angle subsets plateau well
    above the PDHG value, in the FP64 oracle too), so 200 epochs of SPDHG on 21 subsets of
    the same problem are added.  All are upper bounds of the minimum; Psi* is the smallest.
    Returns (psi0, psi_star, info)."""
    dev = d["b"].device
    prm = P.cparams(wl["m"], wl["prior"], "balanced", True, alpha=wl["alpha"],
                    alpha1=wl["alpha1"], seed=seed)
    x = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
    ref = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x, side=d.get("side"))
    if split:
        ref.set_tuning(split)
    psi0 = float(ref.objective()[0].item())
    t0 = time.time()
    ref.epoch(ref_epochs)
    psi_spdhg = float(ref.objective()[0].item())
    ref.close()
    info = {"spdhg_epochs": ref_epochs, "psi_spdhg": psi_spdhg,
            "spdhg_s": round(time.time() - t0, 1)}
    psi_star = psi_spdhg
    if wl["m"] > 21:
        t0 = time.time()
        x.zero_()
        p21 = P.cparams(21, wl["prior"], "balanced", True, alpha=wl["alpha"],
                        alpha1=wl["alpha1"], seed=seed)
        r21 = P.Reconstruction(g, p21, d["b"], d["r"], d["mult"], x, side=d.get("side"))
        r21.epoch(200)
        psi_21 = float(r21.objective()[0].item())
        r21.close()
        info.update({"spdhg21_epochs": 200, "psi_spdhg21": psi_21,
                     "spdhg21_s": round(time.time() - t0, 1)})
        psi_star = min(psi_star, psi_21)
    if wl["prior"] != "tgv" and pdhg_iters > 0:
        t0 = time.time()
        x.zero_()
        pp = P.cparams(1, wl["prior"], "balanced", True, alpha=wl["alpha"], seed=seed)
        pd = P.Reconstruction(g, pp, d["b"], d["r"], d["mult"], x, side=d.get("side"))
        done, trail = 0, []
        while done < pdhg_iters:
            n = min(250, pdhg_iters - done)
            pd.pdhg_iterate(n)
            done += n
            trail.append((done, float(pd.objective()[0].item())))
        psi_pdhg = trail[-1][1]
        U = 2.0 * float(x.max().item())
        gap = pd.gap(U).cpu().numpy()
        pd.close()
        info.update({"pdhg_iters": pdhg_iters, "psi_pdhg": psi_pdhg,
                     "pdhg_gap": [float(v) for v in gap], "pdhg_gap_U": U,
                     "pdhg_s": round(time.time() - t0, 1)})
        psi_star = min(psi_star, psi_pdhg)
        rng_ = psi0 - psi_star
        info["gap_over_range"] = float(gap[0]) / rng_
        # the objective over the last PDHG iterations, relative to the range: how much the
        # reference still moves (the box gap is a loose certificate)
        info["pdhg_tail"] = [(k, (v - psi_star) / rng_) for k, v in trail[-4:]]
        info["spdhg_over_pdhg"] = (psi_spdhg - psi_pdhg) / rng_
    srcs = [f"{ref_epochs} epochs of SPDHG"]
    if "psi_spdhg21" in info:
        srcs.append("200 epochs of SPDHG on 21 subsets")
        info["spdhg_over_best"] = (psi_spdhg - psi_star) / (psi0 - psi_star)
    if "psi_pdhg" in info:
        srcs.append(f"{pdhg_iters} iterations of PDHG (Algorithm 1)")
    info["psi_star_from"] = "min(" + ", ".join(srcs) + ")" if len(srcs) > 1 else srcs[0]
    log(f"reference minimum: {info}")
    return psi0, psi_star, info


def time_to_target(P, torch, g, d, prm, psi0, psi_star, ref_info, target=1e-3, max_epochs=60,
                   split=0):
    """Iteration time until the relative objective (Psi(x^k) - Psi*) / (Psi(x^0) - Psi*)
    (Section 4) first falls to `target`, from x^0 = 0, with the objective evaluated off the
    clock at every quarter epoch (Psi* from reference_minimum).  `split` (if not 0) fixes
    the ray-bundle split."""
    dev = d["b"].device
    x2 = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
    rec = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x2, side=d.get("side"))
    if split:
        rec.set_tuning(split)
    ipe = rec.iters_per_epoch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ms, done, rel = 0.0, 0, float("nan")
    for q in range(4 * max_epochs):
        n = ipe * (q + 1) // 4 - ipe * q // 4
        ev0.record()
        rec.iterate(n)
        ev1.record()
        torch.cuda.synchronize()
        t_ms += ev0.elapsed_time(ev1)
        done += n
        psi = float(rec.objective()[0].item())
        rel = (psi - psi_star) / (psi0 - psi_star)
        if rel <= target:
            break
    rec.close()
    return {"target_rel_objective": target, "seconds": round(t_ms * 1e-3, 4),
            "epochs": round(done / ipe, 2), "reached": bool(rel <= target),
            "rel_objective": rel, "psi0": psi0, "psi_star": psi_star,
            "reference": ref_info,
            "snapshots": "every quarter epoch, objective off the clock"}


def full_operator_rates(P, torch, g, d, nnz, reps=3):
    """spdhg_project / spdhg_backproject over the full sinogram (all angles, caller
    layouts, mult applied): time per call (HIP events, operator workspace allocated
    beforehand) and (image bytes + sinogram bytes) / time, with taps/s (one tap = one
    nonzero of A)."""
    dev = d["b"].device
    ws = P.op_workspace(g, dev)
    x = torch.rand(g.image_shape, device=dev)
    y = torch.empty(g.sino_shape, device=dev)
    xb = torch.empty_like(x)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, call in (("project", lambda: P.spdhg_project(g, 1, -1, d["mult"], x, y, ws=ws)),
                       ("backproject",
                        lambda: P.spdhg_backproject(g, 1, -1, d["mult"], y, xb, ws=ws))):
        call()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            call()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        # image 4 nv + sinogram 4 n_bins (+ mult 4 n_bins)
        nbytes = 4 * g.n_vox + 8 * g.n_bins
        out[name] = {"ms": round(ms, 3), "GBs": round(nbytes / (ms * 1e6), 1),
                     "gtaps_s": round(nnz / (ms * 1e6), 1)}
    return out


def batch_leg(P, torch, steps=3, n_problems=64, seed=18080500):
    """Batched reconstructions: n_problems independent problems of mixed shapes (2-D
    slices 128^2 / 256^2 / 344^2 and mMR slabs 344x344x16 / 32 with segments 0, +-1),
    subset counts 8..64, TV or no prior, 1e5..1e7 counts (beta = 0.1 sqrt(1e5 / counts)),
    advanced together on worker streams / in one HIP graph per batch epoch.  Ray-bundle
    splits come from the autotuner (one timing per shape class)."""
    import numpy as np
    import synth
    from paper_1808_07150_amd import tuning
    from synth.phantom import brain_problem_torch
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [("slice", 128), ("slice", 256), ("slice", 344), ("slab", 16), ("slab", 32)]
    dev = torch.device("cuda:0")
    recs, xs, keep = [], [], []
    t0 = time.time()
    for j in range(n_problems):
        kind, n = shapes[j % len(shapes)]
        g = synth.slice_2d(n) if kind == "slice" else synth.slab(n)
        m = int(min(rng.integers(8, 65), g.n_ang))
        prior = "tv" if rng.random() < 0.5 else "none"
        counts = float(10 ** rng.uniform(5, 7))
        # generated with torch on the host (host Poisson sampler), then copied to the GPU
        dh = brain_problem_torch(g, seed + j, counts, torch.device("cpu"), host_poisson=True)
        d = {k: dh[k].to(dev) for k in ("b", "r", "mult")}
        x = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
        prm = P.cparams(m, prior, "balanced", True, alpha=0.1 * (1e5 / counts) ** 0.5,
                        seed=seed + j)
        recs.append(P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x))
        xs.append(x)
        keep.append(d)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    cache = tuning.autotune(recs)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"problems": n_problems, "epochs": steps, "inputs_s": round(t_gen, 1),
           "tuned_shape_classes": len(cache)}
    # one solo epoch of every problem after the other, then batched epochs
    for mode in ("sequential", "streams", "graph"):
        P.batch_epoch(recs, 1, n_streams=4, graph=(mode == "graph"))  # warm-up
        torch.cuda.synchronize()
        ev0.record()
        if mode == "sequential":
            for _ in range(steps):
                for r in recs:
                    r.epoch(1)
        else:
            P.batch_epoch(recs, steps, n_streams=4, graph=(mode == "graph"))
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        out[f"{mode}_problem_epochs_per_s"] = round(n_problems * steps / (ms * 1e-3), 2)
    for r in recs:
        r.close()
    return out


def run_to_target(P, torch, g, d, prm, x0, psi0, psi_star, target=1e-3, max_epochs=60,
                  split=0):
    """Iteration time (HIP events) from x0 until (Psi - Psi*) / (Psi0 - Psi*) <= target,
    objective off the clock every quarter epoch; returns (seconds, epochs, reached).
    `split` (if not 0) fixes the ray-bundle split."""
    x = x0.clone()
    rec = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x, side=d.get("side"))
    if split:
        rec.set_tuning(split)
    ipe = rec.iters_per_epoch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ms, done = 0.0, 0
    psi = float(rec.objective()[0].item())
    rel = (psi - psi_star) / (psi0 - psi_star)
    q = 0
    while rel > target and q < 4 * max_epochs:
        n = ipe * (q + 1) // 4 - ipe * q // 4
        ev0.record()
        rec.iterate(n)
        ev1.record()
        torch.cuda.synchronize()
        t_ms += ev0.elapsed_time(ev1)
        done += n
        q += 1
        rel = (float(rec.objective()[0].item()) - psi_star) / (psi0 - psi_star)
    rec.close()
    return t_ms * 1e-3, done / ipe, bool(rel <= target)


def sweep_leg(P, torch, g, d, wl, seed, split, psi0, psi_star, ref_info, kind, values):
    """Time to 1e-3 relative objective from x^0 = 0 on the same data for each value of a
    step or sampling parameter, with Psi(x^0) and Psi* shared (the reference minimum of
    the headline measurement).  kind "gamma": the step-size balance of Theorem 2 (S_i =
    gamma rho / A_i 1, T_i = rho p_i / (gamma A_i^T 1); the paper runs gamma = 1 and leaves
    its tuning open, Discussion); kind "p_prior": a constant tuned sampling (Discussion) in
    which the prior block is drawn with probability p_prior and each of the m data blocks
    with (1 - p_prior) / m (balanced sampling is p_prior = 1/2)."""
    m = wl["m"]
    dev = d["b"].device
    rows = []
    for v in values:
        kw = dict(alpha=wl["alpha"], alpha1=wl["alpha1"], seed=seed)
        if kind == "gamma":
            prm = P.cparams(m, wl["prior"], "balanced", True, gamma=v, **kw)
        else:
            prm = P.cparams(m, wl["prior"], "custom", True, p_prior=v, **kw)
        zero = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
        t, ep, ok = run_to_target(P, torch, g, d, prm, zero, psi0, psi_star, split=split)
        rows.append({kind: v, "seconds": round(t, 4), "epochs": round(ep, 2), "reached": ok})
        log(f"{kind} {v}: {t:.4f} s, {ep:.2f} epochs to 1e-3")
    return {"target_rel_objective": 1e-3, "psi_star_from": ref_info.get("psi_star_from"),
            "rows": rows}


def state_precision_leg(P, torch, g, d, wl, seed, split, epochs, psi0, psi_star, ref_info):
    """The primal state's precision: the same SPDHG run from x^0 = 0 with the plain FP32
    x and z and with the compensated state (FP32 pairs, primal step in FP64), relative
    objective against the shared Psi* at a few epoch counts, and how far the iterate still
    moves between them (relative L2 change and the voxels that changed at all)."""
    dev = d["b"].device
    marks = [e for e in (5, 10, 20, 40, 80, 120, 160, 200, 300, 400) if e <= epochs]
    runs = {}
    for comp in (False, True):
        prm = P.cparams(wl["m"], wl["prior"], "balanced", True, alpha=wl["alpha"],
                        alpha1=wl["alpha1"], seed=seed, compensated=comp)
        x = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
        rec = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x, side=d.get("side"))
        if split:
            rec.set_tuning(split)
        rows, done, prev = [], 0, None
        for e in marks:
            rec.epoch(e - done)
            done = e
            psi = float(rec.objective()[0].item())
            row = {"epochs": e, "rel_objective": (psi - psi_star) / (psi0 - psi_star)}
            if prev is not None:
                row["x_change"] = float((x - prev).norm() / x.norm())
                row["voxels_changed"] = int((x != prev).sum())
            rows.append(row)
            prev = x.clone()
        rec.close()
        runs["compensated" if comp else "plain"] = rows
        log(f"state precision ({'compensated' if comp else 'plain'}): " +
            ", ".join(f"{r['epochs']}: {r['rel_objective']:.4e}" for r in rows))
    diff = max(abs(a["rel_objective"] - b["rel_objective"])
               for a, b in zip(runs["plain"], runs["compensated"]))
    return {"psi_star_from": ref_info.get("psi_star_from"), "runs": runs,
            "max_rel_objective_difference": diff}


def warm_start_leg(P, torch, n_train=200, n_test=20, train_passes=12, seed=18080400):
    """Warm start (not part of the paper): a 3-level 3-D conv encoder-decoder (16/32/64
    channels, BF16 MFMA kernels) trained to map the normalised backprojection to the TV MAP
    solution of plain SPDHG (100 epochs) on seeded brain phantoms at 172x172x127 (sinogram
    172 x 126 x 837) whose head, brain and ventricle shapes vary per seed; on held-out
    seeds, time to 1e-3 relative objective (cold-start denominator, Psi* from 200 epochs)
    with and without the warm start.  The warm path's time includes everything from the
    data: the normalised backprojection (A^T b) / (A^T 1) (two backprojections and the
    division, in the library), the input scale, the network and the layout changes."""
    import numpy as np
    import synth
    from paper_1808_07150_amd import warmstart as W
    from synth.phantom import brain_problem_torch
    dev = torch.device("cuda:0")
    g = synth.warmstart_geometry()
    shape = W.padded_shape(g)
    prm = P.cparams(21, "tv", "balanced", True, alpha=2e-3, seed=seed)
    samples = []
    t0 = time.time()
    for j in range(n_train + n_test):
        d = brain_problem_torch(g, seed + j, 3e7, dev, host_poisson=True, vary=True)
        nbp = W.normalised_backprojection(g, d)
        x = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
        rec = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x)
        psi0 = float(rec.objective()[0].item())
        rec.epoch(100 if j < n_train else 200)
        torch.cuda.synchronize()
        psi_ref = float(rec.objective()[0].item())
        rec.close()
        samples.append(dict(d=d if j >= n_train else None, nbp=nbp, target=x.clone(), psi0=psi0,
                            psi_ref=psi_ref, scale=W.input_scale(nbp)))
        if (j + 1) % 10 == 0:
            log(f"warm start: {j + 1} of {n_train + n_test} samples in {time.time() - t0:.1f} s")
    t_data = time.time() - t0
    log(f"warm start: {n_train + n_test} samples and targets in {t_data:.1f} s")
    net = W.WarmStartNet(shape, dev, seed=seed)
    t0 = time.time()
    losses = []
    rng = np.random.Generator(np.random.PCG64(seed))
    for ep in range(train_passes):
        lr = 1e-3 * (0.5 ** (ep * 3 // max(train_passes, 1)))  # halved at each third
        tot = 0.0
        for j in rng.permutation(n_train):
            s_ = samples[j]
            tot += net.train_step(W.to_net(s_["nbp"], shape), W.to_net(s_["target"], shape),
                                  s_["scale"], lr=lr)
        losses.append(tot / n_train)
        log(f"warm start: pass {ep + 1} of {train_passes}, mean loss {losses[-1]:.4g}")
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"warm start: {train_passes} passes over {n_train} samples in {t_train:.1f} s; "
        f"loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = []
    for s_ in samples[n_train:]:
        zero = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
        tc, ec, okc = run_to_target(P, torch, g, s_["d"], prm, zero, s_["psi0"], s_["psi_ref"])
        # the whole warm path from the data (one host read: the input scale)
        stats = torch.empty(3, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nbp = W.normalised_backprojection(g, s_["d"], stats)
        scale = float(stats[2].item())  # count / sum over the support: 1 / mean
        out = net.forward(W.to_net(nbp, shape), scale)
        xw = W.from_net(out, g).clamp_(min=0.0)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t1
        tw, ew, okw = run_to_target(P, torch, g, s_["d"], prm, xw, s_["psi0"], s_["psi_ref"])
        rel_init = None
        res.append(dict(cold_s=round(tc, 4), cold_epochs=ec, cold_reached=okc,
                        warm_s=round(tw + t_inf, 4), warm_epochs=ew, warm_reached=okw,
                        warm_input_and_inference_s=round(t_inf, 5)))
    cold = float(np.mean([r_["cold_s"] for r_ in res]))
    warm = float(np.mean([r_["warm_s"] for r_ in res]))
    return {"geometry": "172x172x127 at 4.16x4.16x2.08 mm, sinogram 172x126x837",
            "train_samples": n_train, "test_samples": n_test, "train_passes": train_passes,
            "targets": "SPDHG+ TV beta=2e-3, 21 subsets, 100 epochs from zero",
            "psi_star": "200 epochs", "data_s": round(t_data, 1), "train_s": round(t_train, 1),
            "loss_first_last": [losses[0], losses[-1]], "per_test": res,
            "mean_cold_s": round(cold, 4), "mean_warm_s": round(warm, 4),
            "speedup": round(cold / warm, 3) if warm > 0 else None}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    # an epoch draws its data / prior iterations at random (half of each on average; a
    # data iteration costs about four prior ones), so the rate of a short window varies by
    # a few percent: 40 epochs keep the spread near 2%
    ap.add_argument("--steps", type=int, default=40, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=2, help="untimed epochs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="mmr-tv21",
                    help="mmr-tv21: the headline workload; mmr-tgv252 / mmr-dtv252: 252 "
                         "single-angle subsets with TGV or directional TV at 3e7 counts")
    ap.add_argument("--inputs", choices=("phantom", "random"), default="phantom",
                    help="phantom: the brain-phantom workload; random: i.i.d. inputs of the "
                         "same shapes (the kernels' memory accesses do not depend on values)")
    ap.add_argument("--warm-start", action="store_true",
                    help="also train the warm-start network and measure its time to target "
                         "(several minutes)")
    ap.add_argument("--ws-train", type=int, default=200, help="warm start: training phantoms")
    ap.add_argument("--ws-test", type=int, default=20, help="warm start: held-out phantoms")
    ap.add_argument("--ws-passes", type=int, default=12, help="warm start: training passes")
    ap.add_argument("--gamma-sweep", action="store_true",
                    help="also measure the time to 1e-3 for step balances gamma = 0.25 .. 32 "
                         "(the headline value stays at the paper's gamma = 1)")
    ap.add_argument("--p-sweep", action="store_true",
                    help="also measure the time to 1e-3 for a tuned constant sampling: prior "
                         "block probability p_prior = 0.1 .. 0.8 (balanced is 0.5)")
    ap.add_argument("--batch", action="store_true",
                    help="also measure batched reconstructions (64 mixed problems, inputs "
                         "generated on the host)")
    ap.add_argument("--fwd-split", type=int, default=0,
                    help="wavefronts per ray bundle of the subset projection (1, 2, 4, 8, or 20 / "
                         "40 for the plane-split variant); 0 = autotune")
    ap.add_argument("--pdhg-iters", type=int, default=2000,
                    help="deterministic PDHG iterations for the reference minimum Psi* "
                         "(Section 4 uses thousands)")
    ap.add_argument("--no-time-to-target", action="store_true",
                    help="skip the time-to-1e-3-relative-objective measurement")
    ap.add_argument("--state-precision", type=int, default=0, metavar="EPOCHS",
                    help="compare the plain and the compensated primal state over this many "
                         "epochs (relative objective against the reference minimum)")
    ap.add_argument("--compensated", action="store_true",
                    help="time the compensated primal step (FP32 pairs for x and z, the step "
                         "in FP64) instead of the plain FP32 state")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="launch a copy kernel of known size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the single-GPU kernels are the subject of this "
              "benchmark and no multi-GPU path is built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1808_07150_amd as P
    import synth
    from synth.phantom import brain_problem_torch

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(torch, dev)
    wl = WORKLOADS[args.workload]
    g = {"span1": synth.mmr_span1, "scanner": synth.mmr_scanner}.get(wl.get("geometry"),
                                                                      synth.mmr)()
    m = wl["m"]
    t0 = time.time()
    if args.inputs == "phantom":
        d = brain_problem_torch(g, SEED, wl["counts"], dev, with_side=wl["prior"] == "dtv",
                                gaps=wl.get("geometry") == "scanner")
    else:
        torch.manual_seed(SEED)
        mean = wl["counts"] / g.n_bins
        d = {"mult": torch.rand(g.sino_shape, device=dev) * 0.4 + 0.8,
             "b": torch.poisson(torch.full(g.sino_shape, mean, device=dev)),
             "r": torch.full(g.sino_shape, 0.3 * mean, device=dev)}
        if wl["prior"] == "dtv":
            d["side"] = torch.rand(g.image_shape, device=dev)
    torch.cuda.synchronize()
    log(f"inputs generated in {time.time() - t0:.1f} s (total counts {float(d['b'].sum()):.3e})")
    x = torch.zeros(g.image_shape, dtype=torch.float32, device=dev)
    prm = P.cparams(m, wl["prior"], "balanced", True, alpha=wl["alpha"], alpha1=wl["alpha1"],
                    seed=SEED, compensated=args.compensated)
    t0 = time.time()
    rec = P.Reconstruction(g, prm, d["b"], d["r"], d["mult"], x, side=d.get("side"))
    torch.cuda.synchronize()
    log(f"init (step sizes) {time.time() - t0:.2f} s; {rec.iters_per_epoch} iterations/epoch")
    if args.fwd_split:
        rec.set_tuning(args.fwd_split)
        split = args.fwd_split
        log(f"ray-bundle split fixed at {split}")
    else:
        split, split_ms = rec.autotune()
        log(f"autotuned ray-bundle split: {split} wavefronts ({split_ms:.3f} ms per subset "
            f"projection); gather tiling {rec.tuning()[1]}")
    obj = rec.objective()
    psi0 = float(obj[0].item())

    for _ in range(args.warmup):
        rec.epoch(1)
    torch.cuda.synchronize()
    # Every leg below runs the same epochs: the state saved here is restored before each
    # (its iteration counter fixes the random draws), so they do the same work.  First,
    # untimed, every kernel kind under events, which names the dominant kernel and gives
    # the others' launch times; the timed epochs then carry events around the dominant
    # kernel only (each event pair costs the stream a few microseconds).
    snap = rec.save_state()
    rec.set_profiling(True)
    rec.epoch(args.steps)
    prof = rec.profile()
    rec.set_profiling(False)
    dom = max(prof, key=lambda k: prof[k][0])
    rec.load_state(snap)
    rec.set_profiling(True, kinds=(dom,))
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    rec.epoch(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof_timed = rec.profile()
    rec.set_profiling(False)
    # the same iterations as the untimed pass, so the same launches of the dominant kind
    assert prof_timed[dom][1] == prof[dom][1], (prof_timed, prof)
    prof[dom] = prof_timed[dom]  # the dominant kernel's launch times of the timed region
    psi = float(rec.objective()[0].item())
    x_timed = x.clone()
    # the same epochs without per-launch events: plain launches and HIP-graph epochs, each
    # checked bitwise against the image of the timed epochs
    alt = {}
    for mode in ("eager", "graph"):
        if mode == "graph":
            rec.epoch_graph(1)  # builds and instantiates the persistent graph (untimed)
        rec.load_state(snap)
        torch.cuda.synchronize()
        ev0.record(stream)
        if mode == "eager":
            rec.epoch(args.steps)
        else:
            rec.epoch_graph(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        alt[f"{mode}_epochs_per_s"] = round(args.steps / (ev0.elapsed_time(ev1) * 1e-3), 3)
        alt[f"{mode}_same_image"] = bool(torch.equal(x, x_timed))
        # TGV's lazy w step is settled at every graph epoch's end but only at the end of
        # the eager call, so there the two differ by rounding
        alt[f"{mode}_max_rel_diff"] = float((x - x_timed).abs().max() / x_timed.abs().max())
    del snap, x_timed
    log(f"without per-kernel events: {alt}")
    log(f"{args.steps} epochs in {ms:.1f} ms (events around {dom} only); objective "
        f"{psi0:.6e} -> {psi:.6e}")
    log("kernels: " + ", ".join(f"{k} {v[0]:.1f} ms / {v[1]}" for k, v in prof.items())
        + f" ({dom}: timed region; others: the same epochs in the untimed pass)")

    nv = g.n_vox
    n_i = P.subset_bins(g, m, 0)
    nnz = P.spdhg_nnz(g, m, 0)
    nnz_full = P.spdhg_nnz(g, 1, -1)
    # algorithmic bytes per launch (FP32, compulsory traffic, no re-reads)
    bytes_fwd = 4 * nv + 28 * n_i          # x; y b r mult sigma in, y d out
    bytes_bwd = 20 * nv + 4 * n_i          # d in; z x T in, z x out
    bytes_prior = wl["prior_bpv"] * nv     # see WORKLOADS
    if args.compensated:                   # low parts of x and z in and out
        bytes_bwd += 16 * nv
        bytes_prior += 16 * nv
    flops_fwd = 2.0 * nnz + 20.0 * n_i     # one FMA per nonzero + the prox per bin
    flops_bwd = 2.0 * nnz + 6.0 * nv
    # launches of the timed epochs (the untimed pass ran the same iterations)
    n_fwd, n_prior = prof["fwd"][1], prof["prior"][1]
    epoch_bytes = (n_fwd * (bytes_fwd + bytes_bwd) + n_prior * bytes_prior) / args.steps
    kinds = {
        "fwd": dict(bound="alu", work=flops_fwd, unit="TFLOP/s", peak=ALU_PEAK_TFLOPS,
                    name="fwd_wave (projection + KL-dual prox)"),
        "bwd": dict(bound="alu", work=flops_bwd, unit="TFLOP/s", peak=ALU_PEAK_TFLOPS,
                    name="bwd_strip partial + iter (gather backprojection + primal epilogue)"),
        "prior": dict(bound="hbm", work=bytes_prior, unit="GB/s", peak=HBM_PEAK_GBS,
                      name={"tv": "tv_wave (TV dual + adjoint + primal epilogue)",
                            "dtv": "tv_wave (dTV dual + adjoint + primal epilogue)",
                            "tgv": "tgv1_wave / tgv2_wave (TGV duals + adjoints + primal "
                                   "epilogue of u and w)"}[wl["prior"]]),
    }
    avg_ms = prof[dom][0] / max(prof[dom][1], 1)
    kd = kinds[dom]
    scale = 1e-12 if kd["unit"] == "TFLOP/s" else 1e-9
    achieved = kd["work"] * scale / (avg_ms * 1e-3)
    per_kernel = {}
    for k, (tot, n) in prof.items():
        if n:
            a = tot / n
            per_kernel[k] = {"avg_ms": round(a, 4), "launches": n,
                             "algorithmic_GBs": round((dict(fwd=bytes_fwd, bwd=bytes_bwd,
                                                            prior=bytes_prior)[k]) / (a * 1e6), 1)}
    roofline = {"bound": kd["bound"], "achieved": round(achieved, 3), "peak": kd["peak"],
                "unit": kd["unit"], "frac": round(achieved / kd["peak"], 4),
                "frac_of_unpacked_fp32": round(achieved / ALU_UNPACKED_TFLOPS, 4)
                if kd["unit"] == "TFLOP/s" else None,
                "traffic": (measured_traffic(dom) if args.workload == "mmr-tv21"
                            and not args.compensated else None),
                "kernel": kd["name"], "avg_ms": round(avg_ms, 4)}
    epochs_per_s = args.steps / (ms * 1e-3)
    pb_ms = sum(prof[k][0] / max(prof[k][1], 1) for k in ("fwd", "bwd"))
    out = {
        "metric": METRIC, "value": round(epochs_per_s, 3), "unit": "epochs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["label"], "iters_per_epoch": rec.iters_per_epoch,
                   "fwd_split": split,
                   "nnz_per_subset": nnz,
                   "primal_state": "FP32 pairs, FP64 step" if args.compensated else "FP32"},
        "epoch_hbm": {"algorithmic_GB": round(epoch_bytes / 1e9, 2),
                      "achieved_GBs": round(epoch_bytes / (ms / args.steps * 1e6), 1),
                      "frac": round(epoch_bytes / (ms / args.steps * 1e6) / HBM_PEAK_GBS, 4)},
        "subset_step": {"ms": round(pb_ms, 3),
                        "algorithmic_GBs": round((bytes_fwd + bytes_bwd) / (pb_ms * 1e6), 1),
                        "gtaps_s": round(2 * nnz / (pb_ms * 1e6), 1),
                        "what": "fused subset projection + KL-dual prox and gather "
                                "backprojection + primal epilogue of one data iteration"},
        "proj_backproj": full_operator_rates(P, torch, g, d, nnz_full),
        "kernels": per_kernel,
        "roofline": roofline,
        "iterations": {"data": n_fwd, "prior": n_prior},  # of the timed epochs
        "objective": {"initial": psi0, "after": psi},
        "unprofiled": alt,
    }
    if not args.no_time_to_target:
        t0 = time.time()
        rec.close()
        psi0_ref, psi_star, ref_info = reference_minimum(
            P, torch, g, d, wl, SEED, ref_epochs=200 if m <= 21 else 40,
            pdhg_iters=args.pdhg_iters, split=split)
        out["time_to_target"] = time_to_target(P, torch, g, d, prm, psi0_ref, psi_star,
                                               ref_info, split=split)
        log(f"time to 1e-3 relative objective: {out['time_to_target']['seconds']} s "
            f"({out['time_to_target']['epochs']} epochs; measured in {time.time() - t0:.1f} s)")
    if args.gamma_sweep or args.p_sweep or args.state_precision:
        if args.no_time_to_target:
            psi0_ref, psi_star, ref_info = reference_minimum(
                P, torch, g, d, wl, SEED, ref_epochs=200 if m <= 21 else 40,
                pdhg_iters=args.pdhg_iters, split=split)
        if args.gamma_sweep:
            out["gamma_sweep"] = sweep_leg(P, torch, g, d, wl, SEED, split, psi0_ref, psi_star,
                                           ref_info, "gamma",
                                           (0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0))
        if args.p_sweep:
            out["p_prior_sweep"] = sweep_leg(P, torch, g, d, wl, SEED, split, psi0_ref,
                                             psi_star, ref_info, "p_prior",
                                             (0.1, 0.2, 0.35, 0.5, 0.65, 0.8))
        if args.state_precision:
            out["state_precision"] = state_precision_leg(P, torch, g, d, wl, SEED, split,
                                                         args.state_precision, psi0_ref,
                                                         psi_star, ref_info)
    if args.warm_start:
        t0 = time.time()
        out["warm_start"] = warm_start_leg(P, torch, n_train=args.ws_train, n_test=args.ws_test,
                                           train_passes=args.ws_passes)
        log(f"warm start: {out['warm_start']['mean_cold_s']} s cold vs "
            f"{out['warm_start']['mean_warm_s']} s warm ({time.time() - t0:.1f} s)")
    if args.batch:
        t0 = time.time()
        out["batch"] = batch_leg(P, torch)
        log(f"batch: {out['batch']} ({time.time() - t0:.1f} s)")
    if not args.no_cpu_baseline:
        t0 = time.time()
        host = {k: d[k].cpu().numpy() for k in ("b", "r", "mult")}
        if "side" in d:
            host["side"] = d["side"].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(g, host, wl, SEED)
        log(f"cpu baseline {time.time() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
