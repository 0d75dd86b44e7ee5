"""Benchmark of the SORF hot path on one MI355X.

One step = one pass of the whole training + inference path over the QM9-like
workload (20,000 molecules of 3..29 atoms, d = 128, 64 stacks -> D = 8192,
sigma = 4): features Z (sorf_forward), normal equations G += Z^T Z, Zty += Z^T y
(sorf_gram_accumulate, FP32 as the workload states), FP64 ridge solve with 3 refinement steps (sorf_solve),
energies E = Z alpha without forming Z (sorf_predict) and dE/dx for every atom
(sorf_backward). Inputs are synthetic, seeded, and resident in HBM before the
clock starts.

A serving leg follows: a Poisson trace of energy+force requests (D = 16384,
5..300 atoms) served by continuous batching and by one molecule per launch;
p50/p99 latency and atoms/s of both are reported under "serving".

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "bf16_hilo": 2500.0,
                    "fp16_hilo": 2500.0, "fp64": 78.6, "fp32_kahan": 157.3, "split": 2500.0}
# matrix-core work per algorithmic product, in units of one 16-bit product: hi+lo runs
# four fp16/bf16 products; split runs one int8 product (double rate) and three fp16
MFMA_WORK = {"bf16_hilo": 4.0, "fp16_hilo": 4.0, "split": 3.5}
# VALU issue ceiling derived from unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3 T lane-instructions/s (packed FP32, which would double it, is disabled by the library's compile flags)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def valu_slots_per_feature(d: int, T: int, backward: bool = False) -> float:
    """Algorithmic VALU issue slots per atom-feature. Forward: T log2(d)
    butterfly add/subs + T sign flips + 1 phase FMA + 1 accumulate + one
    transcendental (quarter rate = 4 slots). Fused forward+backward: twice the
    transform work, cos and sin, and 2 more FMAs (alpha weighting)."""
    lg = math.log2(d)
    fwd = T * lg + T + 1 + 4 + 1
    if not backward:
        return fwd
    return 2 * (T * lg + T) + 1 + 8 + 3


def dz_slots_per_unit(d: int, T: int) -> float:
    """Algorithmic VALU issue slots per (atom, coordinate column, feature) of
    the derivative features: T log2(d) butterfly add/subs + T sign flips of
    the Jacobian column's transform + 1 FMA of sin(u) times it into the row."""
    return T * math.log2(d) + T + 1


def measured_gram_counters(mode, M, D):
    """HBM bytes and matrix-core busy fraction of one Gram call from the
    committed counter runs (profiles/gram_qm9_like_counters.json: scaled
    FETCH_SIZE + WRITE_SIZE per call, SQ_VALU_MFMA_BUSY_CYCLES per SIMD-cycle),
    valid only for the same mode and size and while the Gram source is
    unchanged since the counters were taken; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gram_qm9_like_counters.json")
    src = os.path.join(ROOT, "paper_2206_01580_amd", "csrc", "sorf_gram.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != h or rec.get("M") != M or rec.get("D") != D \
            or mode not in rec.get("modes", {}):
        return None
    return rec["modes"][mode]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--gram", default="fp32", choices=list(PEAK_MFMA_TFLOPS))
    ap.add_argument("--gram-modes", default="fp32_kahan,bf16,bf16_hilo,fp16_hilo,split",
                    help="other Gram modes timed on the same Z after the step (labelled extras)")
    ap.add_argument("--n-mols", type=int, default=20000)
    ap.add_argument("--n-refine", type=int, default=3)
    ap.add_argument("--lam", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mols", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the Poisson request trace (0 skips the serving leg)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-max-atoms", type=int, default=8192)
    ap.add_argument("--serve-sweep", default="5000,10000,20000,32000",
                    help="extra offered loads (req/s), each a trace of --serve-sweep-requests")
    ap.add_argument("--serve-sweep-requests", type=int, default=4000)
    ap.add_argument("--force-confs", type=int, default=2000,
                    help="conformations of the force-training leg (0 skips it)")
    ap.add_argument("--force-steps", type=int, default=3)
    ap.add_argument("--projection", type=int, default=1,
                    help="run the per-element projection leg (0 skips it)")
    ap.add_argument("--ntransform-study", type=int, default=1,
                    help="run the N_transform study (0 skips it)")
    ap.add_argument("--roundoff-study", type=int, default=1,
                    help="run the FP32 round-off study of dense-W RFF vs SORF phases (0 skips it)")
    ap.add_argument("--representation", type=int, default=1,
                    help="run the FCHL19 representation leg (0 skips it)")
    ap.add_argument("--components", type=int, default=1,
                    help="time the energy+force chain on single configurations (0 skips it)")
    ap.add_argument("--precision-mols", type=int, default=100000,
                    help="molecules of the precision study (0 skips it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (scale reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def serving_leg(args, dev, log, rate, seconds):
    """Energy+force serving on a Poisson trace (D = 16384, sizes log-uniform
    5..300 atoms), same GPU, same resident model and request pool:
    - batched: continuous batching into the library's persistent serving
      kernel (sorf_server_*: batches published through a ring in host-coherent
      memory, no launch per batch), up to 64 requests and --serve-max-atoms
      atoms per batch, --serve-slots batches in flight;
    - plain: one molecule per sorf_predict launch sequence, FIFO, one stream.
    Each request's results are bitwise the same on both paths."""
    import torch

    from paper_2206_01580_amd import serve, sorf, workloads
    tr = workloads.serving_trace(rate_hz=rate, duration_s=seconds)
    J = workloads.device_normal(tr.J_pool_floats, tr.J_seed, 0.1, device=dev)
    pool = serve.RequestPool(tr.x, tr.element, tr.sizes, J, tr.J_off, device=dev)
    model = sorf.Model.from_problem(tr.model)
    alpha = torch.from_numpy(tr.model.alpha).to(dev)
    R = len(tr.sizes)
    cap = max(args.serve_max_atoms, int(tr.sizes.max()))
    exp = serve.GpuExecutor(model, alpha, pool, max_batch_atoms=int(tr.sizes.max()),
                            max_batch_reqs=1, n_slots=1, device=dev)
    h = exp.submit(0, 1)         # load the kernels and touch every buffer once
    while not h.done():
        pass
    exp.results.clear()
    torch.cuda.synchronize()
    log(f"serving: {R} requests, {int(tr.sizes.sum())} atoms, rate {rate:g}/s")
    srv = serve.NativeServer(model, alpha, pool, max_batch_atoms=cap, ring_slots=args.serve_slots,
                             idle_timeout_s=max(30.0, 2 * seconds), device=dev)
    # in-flight request state: the result slots of the ring
    budget = args.serve_slots * srv.slot_bytes()
    try:
        h = srv.submit(0, 1)     # first batch: the kernel's code and the pool pages are warm
        while not h.done():
            pass
        srv.results.clear()
        sb = serve.BatchingScheduler(srv, cap, args.serve_slots, budget,
                                     max_batch_requests=serve.NativeServer.MAX_REQUESTS
                                     ).run(tr.arrival_s, tr.sizes)
    finally:
        state = srv.stop()
    torch.cuda.synchronize()
    log(f"serving: batched done ({len(sb.batches)} batches, kernel exit state {state})")
    sp = serve.PlainRunner(exp).run(tr.arrival_s, tr.sizes)
    torch.cuda.synchronize()
    log("serving: plain done")
    warm = min(1.0, 0.1 * seconds)       # the first second of the trace is warm-up
    b, p = sb.summary(warm, tr.arrival_s), sp.summary(warm, tr.arrival_s)
    del pool, J, exp, srv
    torch.cuda.empty_cache()
    return {
        "workload": (f"Poisson {rate:g} req/s for {seconds:g} s, sizes log-uniform 5..300 atoms, "
                     f"d=128, D=16384, energies + forces (J blocks N x 128 x 3N at random offsets "
                     f"of a {tr.J_pool_floats * 4 >> 20} MiB pool)"),
        "rate_hz": rate, "requests": R, "atoms": int(tr.sizes.sum()), "warmup_s": warm,
        "batched": dict(b, executor="persistent serving kernel (sorf_server)",
                        ring_slots=args.serve_slots, max_batch_atoms=cap,
                        max_batch_requests=serve.NativeServer.MAX_REQUESTS, kernel_exit_state=state),
        "plain": dict(p, executor="sorf_predict per request (4 kernels, 2 offset uploads, "
                                  "2 result copies, 1 event)"),
        "p50_speedup": (p["p50_ms"] / b["p50_ms"]) if b["p50_ms"] else None,
        "p99_speedup": (p["p99_ms"] / b["p99_ms"]) if b["p99_ms"] else None,
        "atoms_per_s_ratio": (b["atoms_per_s"] / p["atoms_per_s"]) if p["atoms_per_s"] else None,
    }


def force_training_leg(args, dev, log):
    """Force-trained normal equations on the differentiation workload (one
    21-atom molecule in 2,000 conformations, d = 128, D = 8192, Jacobians
    d x 63 per atom): features Z, derivative features dZ (3 rows per atom),
    G = Z^T Z + dZ^T dZ and Zty = Z^T E + dZ^T F in the bench's Gram mode, and
    the FP64 solve. Energy and force targets are seeded N(0, 1) (the timing
    does not depend on them)."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    p = workloads.conformations(n_conf=args.force_confs, with_J=False)
    D, A, M = p.n_features, p.n_atoms, p.n_mols
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    n_j = A * p.d * 3 * int(p.mol_sizes()[0])
    J = workloads.device_normal(n_j, p.seed + 1, 0.1, device=dev)
    J_ptr = torch.arange(M + 1, dtype=torch.int64, device=dev) * (n_j // M)
    E_t = workloads.device_normal(M, p.seed + 2, 1.0, device=dev)
    F_t = workloads.device_normal(3 * A, p.seed + 3, 1.0, device=dev)
    Z = torch.empty(M, D, device=dev)
    dZ = torch.empty(3 * A, D, device=dev)
    acc_t = torch.float64 if args.gram in ("fp64", "split") else torch.float32
    G = torch.empty(D, D, device=dev, dtype=acc_t)
    r = torch.empty(D, device=dev, dtype=acc_t)
    ws = sorf.GramWorkspace(dev)
    if args.gram != "fp64":
        ws.get(3 * A, D, args.gram)             # allocate before timing
    solver = sorf.Solver(D, device=dev)
    alpha = torch.empty(D, device=dev, dtype=torch.float64)
    scale_exp = 0
    if args.gram.startswith("fp16"):
        torch.cuda.synchronize()
        sorf.derivative_features(model, batch, J, J_ptr, out=dZ)
        sorf.forward(model, batch, out=Z)
        mx = max(float(Z.abs().max()), float(dZ.abs().max()))
        scale_exp = sorf.fp16_scale_exp(mx)
    phases = ["forward", "dz", "gram", "solve"]
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in phases}
    times = {k: [] for k in phases}

    def step(record):
        def mark(k, i):
            if record:
                ev[k][i].record()
        mark("forward", 0)
        sorf.forward(model, batch, out=Z)
        mark("forward", 1)
        mark("dz", 0)
        sorf.derivative_features(model, batch, J, J_ptr, out=dZ)
        mark("dz", 1)
        G.zero_()
        r.zero_()
        mark("gram", 0)
        sorf.gram_accumulate(Z, G, E_t, r, precision=args.gram, scale_exp=scale_exp, workspace=ws)
        sorf.gram_accumulate(dZ, G, F_t, r, precision=args.gram, scale_exp=scale_exp, workspace=ws)
        mark("gram", 1)
        mark("solve", 0)
        solver(G, r, args.lam, args.n_refine, out=alpha)
        mark("solve", 1)

    step(False)
    torch.cuda.synchronize()
    info = int(solver.info.item())
    log(f"force training: {M} conformations, dZ {3 * A} x {D}, info {info}")
    t0 = time.perf_counter()
    for _ in range(args.force_steps):
        step(True)
        torch.cuda.synchronize()
        for k in phases:
            times[k].append(ev[k][0].elapsed_time(ev[k][1]))
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.force_steps
    med = {k: float(np.median(v)) for k, v in times.items()}
    # inference on the same conformations with the fitted alpha: energies and
    # forces in one sorf_predict call, dE/dx alone (sorf_backward), and the force
    # contraction alone (sorf_forces) on that gradient
    a32 = alpha.float().contiguous()
    pred, fcon = sorf.Predictor(model, dev), sorf.ForceContraction(dev)
    E_p, F_p, F_c = (torch.empty(M, device=dev), torch.empty(3 * A, device=dev),
                     torch.empty(3 * A, device=dev))
    gx = torch.empty((A, p.d), device=dev)

    def infer(e=None):
        for k, fn in enumerate((lambda: pred(batch, a32, J, J_ptr, E=E_p, F=F_p),
                                lambda: sorf.backward(model, batch, a32, out=gx),
                                lambda: fcon(batch.mol_ptr, gx, J, J_ptr, out=F_c))):
            if e is not None:
                e[2 * k].record()
            fn()
            if e is not None:
                e[2 * k + 1].record()

    infer()
    torch.cuda.synchronize()
    inames = ["predict_energy_force", "dE_dx", "forces"]
    itimes = {k: [] for k in inames}
    for _ in range(max(3, args.force_steps)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        infer(e)
        torch.cuda.synchronize()
        for k, nm in enumerate(inames):
            itimes[nm].append(e[2 * k].elapsed_time(e[2 * k + 1]))
    imed = {k: float(np.median(v)) for k, v in itimes.items()}
    f_diff = float((F_c - F_p).abs().max() / F_p.abs().max().clamp_min(1e-30))
    f_bytes = 4.0 * (n_j + A * p.d + 3 * A)                  # J, dE/dx and F, once each
    f_gbs = f_bytes / (imed["forces"] * 1e-3) / 1e9
    units = float(A) * 3 * int(p.mol_sizes()[0]) * D          # (atom, column, feature)
    dz_tops = units * dz_slots_per_unit(p.d, p.n_transforms) / (med["dz"] * 1e-3) / 1e12
    rows = M + 3 * A
    gram_tf = float(rows) * D * (D + 1) / (med["gram"] * 1e-3) / 1e12
    out = {
        "workload": (f"{M} conformations of a 21-atom molecule, d={p.d}, {p.n_stacks} stacks "
                     f"(D={D}), sigma={p.sigma:g}, Jacobians d x 63 per atom N(0, 0.1); "
                     f"(Z, dZ) has {rows} rows; Gram {args.gram}, lambda={args.lam:g}"),
        "ms_per_step": wall_ms, "phase_ms": med, "solve_info": info,
        "dz_rows_per_s": 3.0 * A / (med["dz"] * 1e-3),
        "roofline_dz": {"bound": "alu", "achieved": dz_tops, "peak": PEAK_VALU_TOPS,
                        "unit": "T VALU-slots/s", "frac": dz_tops / PEAK_VALU_TOPS,
                        "traffic": None,
                        "slots_per_unit": dz_slots_per_unit(p.d, p.n_transforms),
                        "units_per_launch": units},
        "gram_tflops": gram_tf,
        "gram_frac": gram_tf / PEAK_MFMA_TFLOPS[args.gram],
        "inference": {
            "phase_ms": imed,
            "conformations_per_s": M / (imed["predict_energy_force"] * 1e-3),
            "forces_call_vs_predict_max_rel_diff": f_diff,
            "roofline_forces": {"bound": "hbm", "achieved": f_gbs, "peak": PEAK_HBM_GBS,
                                "unit": "GB/s", "frac": f_gbs / PEAK_HBM_GBS, "traffic": None,
                                "algorithmic_bytes": f_bytes},
        },
    }
    if not args.no_cpu_baseline:
        from oracle import sorf_oracle as O
        q = workloads.conformations(n_conf=4)
        t1 = time.perf_counter()
        O.derivative_features(q.x, q.element, q.mol_ptr, q.signs, q.bias, q.sigma, q.J, q.J_ptr)
        t_o = time.perf_counter() - t1
        out["cpu_baseline_dz"] = {
            "value": 3.0 * q.n_atoms / t_o, "unit": "dZ rows/s",
            "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"FP64 dense-W oracle, dZ of 4 conformations ({3 * q.n_atoms} rows), {t_o:.2f} s"}
    del Z, dZ, G, r, ws, solver, J, gx, E_p, F_p, F_c, pred, fcon
    torch.cuda.empty_cache()
    return out


def projection_leg(args, p, dev, log):
    """Per-element projection on the QM9-like batch: every atom's 720-entry
    representation (the FCHL19 size for five elements with the energy+force
    parameters; synthetic, drawn on the device) projected to d = 128 with a
    matrix per element, fitted on the GPU from 1000 sampled atoms of that
    element."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    d_rep, d, E = workloads.FCHL19_EF_SIZE, p.d, p.n_elements
    el = torch.from_numpy(p.element).to(dev)
    rho = workloads.device_representations(p.element, E, d_rep, seed=p.seed + 5, device=dev)
    U = torch.empty((E, d_rep, d), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(p.seed + 6)
    fit_ms = []
    for e in range(E):
        rows = np.nonzero(p.element == e)[0]
        rows = np.sort(rng.choice(rows, size=min(len(rows), 1000), replace=False))
        sample = rho.index_select(0, torch.from_numpy(rows).to(dev)).contiguous()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sorf.projection_fit(sample, d, out=U[e])
        e1.record()
        torch.cuda.synchronize()
        fit_ms.append(e0.elapsed_time(e1))
    proj = sorf.Projector(U)
    x = torch.empty((p.n_atoms, d), dtype=torch.float32, device=dev)
    proj(rho, el, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = max(3, args.steps)
    e0.record()
    for _ in range(n):
        proj(rho, el, x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    flop = 2.0 * p.n_atoms * d_rep * d
    tf = flop / (ms * 1e-3) / 1e12
    out = {
        "workload": (f"{p.n_atoms} atoms of the QM9-like batch, representations of {d_rep} entries "
                     f"-> d={d}, {E} elements, projections fitted from 1000 atoms per element"),
        "project_ms": ms, "fit_ms_per_element": fit_ms,
        "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_MFMA_TFLOPS["fp32"],
                     "unit": "TFLOP/s", "frac": tf / PEAK_MFMA_TFLOPS["fp32"], "traffic": None,
                     "algorithmic_bytes": 4.0 * p.n_atoms * (d_rep + d)},
    }
    if not args.no_cpu_baseline:
        from oracle import sorf_oracle as O
        k = min(100000, p.n_atoms)
        rows = np.arange(k)
        rho_h = rho[:k].cpu().numpy()
        Uh = U.cpu().numpy()
        t0 = time.perf_counter()
        O.project(rho_h, p.element[rows], Uh)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": k / t, "unit": "atoms/s", "cores": len(os.sched_getaffinity(0)),
                               "kind": "oracle", "sample": f"FP64 oracle projection of {k} atoms, {t:.2f} s"}
    del rho, x, U, proj
    torch.cuda.empty_cache()
    return out


def ntransform_study(args, p, dev, log):
    """N_transform in {1, 2, 3} on the QM9-like batch (the paper runs T = 2,
    the main step T = 3): forward and dE/dx times at full size, and the
    kernel-approximation error of the features: over 256 carbon atoms,
    ||Zhat Zhat^T - K||_F / ||K||_F against the Gaussian kernel
    K_ij = exp(-|x_i - x_j|^2 / (2 sigma^2)) the estimator approximates,
    using the first N_F features (N_F = 1024 .. 8192). The feature map keeps
    its sqrt(2/N_F) normaliser for each N_F."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    C = p.element_names.index("C")
    rows = np.nonzero(p.element == C)[0][:256]
    xs = p.x[rows].astype(np.float64)
    sq = np.sum((xs[:, None, :] - xs[None, :, :]) ** 2, axis=2)
    K = np.exp(-sq / (2.0 * p.sigma ** 2))
    res = {}
    for T in (1, 2, 3):
        q = workloads.with_transforms(p, T)
        model, batch = sorf.Model.from_problem(q), sorf.Batch.from_problem(q)
        alpha = torch.from_numpy(q.alpha if q.alpha is not None else
                                 np.ones(q.n_features, np.float32)).to(dev)
        Z = torch.empty(q.n_mols, q.n_features, device=dev)
        g = torch.empty(q.n_atoms, q.d, device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        sorf.forward(model, batch, out=Z)
        sorf.backward(model, batch, alpha, out=g)
        torch.cuda.synchronize()
        n = 3
        ev[0].record()
        for _ in range(n):
            sorf.forward(model, batch, out=Z)
        ev[1].record()
        for _ in range(n):
            sorf.backward(model, batch, alpha, out=g)
        ev[2].record()
        torch.cuda.synchronize()
        f_ms, b_ms = ev[0].elapsed_time(ev[1]) / n, ev[1].elapsed_time(ev[2]) / n
        # single-atom molecules of the 256 carbon atoms
        a = workloads.Problem(q.name, q.d, q.n_stacks, T, q.sigma, q.element_names,
                              np.ascontiguousarray(q.x[rows]), np.full(len(rows), C, np.int32),
                              np.arange(len(rows) + 1, dtype=np.int64), q.signs, q.bias)
        Za = sorf.forward(sorf.Model.from_problem(a), sorf.Batch.from_problem(a)).double()
        err = {}
        for nf in (1024, 2048, 4096, 8192):
            Zs = Za[:, :nf] * math.sqrt(q.n_features / nf)
            Kh = (Zs @ Zs.T).cpu().numpy()
            err[str(nf)] = float(np.linalg.norm(Kh - K) / np.linalg.norm(K))
        res[f"T{T}"] = {"forward_ms": f_ms, "backward_ms": b_ms,
                        "forward_atom_features_per_s": q.n_atoms * q.n_features / (f_ms * 1e-3),
                        "kernel_rel_err_by_nf": err}
        del Z, g, model, batch
        torch.cuda.empty_cache()
        log(f"ntransform: T={T} done")
    return {"workload": (f"{p.n_atoms} atoms of the QM9-like batch, D={p.n_features}; kernel error over "
                         f"{len(rows)} carbon atoms against exp(-|dx|^2/(2 sigma^2)), sigma={p.sigma:g}"),
            "by_T": res}


def roundoff_study(args, p, dev, log):
    """FP32 round-off of the phases W x: dense Gaussian W (RFF, entries
    N(0, 1/sigma^2)) against the SORF transform, both in FP32 on the GPU, on
    the x of 256 carbon atoms of the QM9-like batch (d = 128, sigma = 4). RFF
    phases come from the FP32 matrix-core product of sorf_project (W^T as a
    one-element projection); SORF features from sorf_forward on single-atom
    molecules. Errors against FP64 on the host: the RFF phase error itself, and
    for both the feature error |dz| in units of sqrt(2/N_F) (for RFF, cos of the
    FP32 phases taken in FP64, so only the phase round-off counts)."""
    import torch

    from oracle import sorf_oracle as O
    from paper_2206_01580_amd import sorf, workloads
    C = p.element_names.index("C")
    rows = np.nonzero(p.element == C)[0][:256]
    x = np.ascontiguousarray(p.x[rows])
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(p.seed + 7)
    out = {}
    for S in (8, 32, 128):
        D = S * p.d
        W = (rng.standard_normal((D, p.d)) / p.sigma).astype(np.float32)
        b = rng.uniform(0.0, 2.0 * math.pi, D)
        Ut = torch.from_numpy(np.ascontiguousarray(W.T)[None]).to(dev)
        u32 = sorf.project(torch.from_numpy(x).to(dev),
                           torch.zeros(len(rows), dtype=torch.int32, device=dev), Ut)
        u32 = u32.double().cpu().numpy()
        u64 = x64 @ W.astype(np.float64).T
        rff_dz = np.abs(np.cos(u32 + b) - np.cos(u64 + b))
        # SORF: the same atoms as single-atom molecules, D features of the batch's model
        signs = p.signs[C:C + 1, :, :S] if S <= p.n_stacks else None
        if signs is None:
            rs = np.random.default_rng(p.seed + 8 + S)
            signs = (1 - 2 * rs.integers(0, 2, size=(1, p.n_transforms, S, p.d))).astype(np.int8)
        bias = np.ascontiguousarray(b[None].astype(np.float32))
        a = workloads.Problem("roundoff", p.d, S, p.n_transforms, p.sigma, ("C",), x,
                              np.zeros(len(rows), np.int32), np.arange(len(rows) + 1, dtype=np.int64),
                              np.ascontiguousarray(signs), bias)
        Zs = sorf.forward(sorf.Model.from_problem(a), sorf.Batch.from_problem(a)).double().cpu().numpy()
        Zo = O.molecule_features(a.x, a.element, a.mol_ptr, a.signs, a.bias, a.sigma)
        sorf_dz = np.abs(Zs - Zo) / math.sqrt(2.0 / D)
        uo = O.phases(a.x, a.element, a.signs, a.bias, a.sigma)
        out[str(D)] = {
            "rff_phase_err_max": float(np.abs(u32 - u64).max()),
            "rff_phase_err_rms": float(np.sqrt(np.mean((u32 - u64) ** 2))),
            "rff_phase_abs_max": float(np.abs(u64).max()),
            "sorf_phase_abs_max": float(np.abs(uo - a.bias[0].astype(np.float64)).max()),
            "rff_feature_err_max": float(rff_dz.max()), "rff_feature_err_rms": float(np.sqrt(np.mean(rff_dz ** 2))),
            "sorf_feature_err_max": float(sorf_dz.max()),
            "sorf_feature_err_rms": float(np.sqrt(np.mean(sorf_dz ** 2))),
        }
        log(f"roundoff: N_F={D} done")
    return {"workload": (f"x of {len(rows)} carbon atoms of the QM9-like batch (d={p.d}, sigma={p.sigma:g}); "
                         "errors against FP64, feature errors in units of sqrt(2/N_F)"),
            "by_nf": out}


def fchl19_slots(R, mol_ptr, rcut, n2, n3):
    """VALU-slot model of the FCHL19 forward: 8 slots per (neighbour, two-body bin)
    (one exponential at quarter rate = 4, and the square, scale, multiply, add),
    7 per (neighbour pair, three-body bin) (exponential 4, difference, square,
    two FMAs) and 80 per neighbour pair for its geometry (a square root, divisions,
    the power and three cutoff cosines). Returns (slots, neighbours, pairs)."""
    nb = 0
    pairs = 0
    for m in range(len(mol_ptr) - 1):
        X = R[mol_ptr[m]:mol_ptr[m + 1]].astype(np.float64)
        d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
        n = (d < rcut).sum(axis=1) - 1
        nb += int(n.sum())
        pairs += int((n * (n - 1) // 2).sum())
    return 8.0 * nb * n2 + 7.0 * pairs * n3 + 80.0 * pairs, nb, pairs


def fchl19_backward_slots(nb, pairs, n2, n3):
    """VALU-slot model of the FCHL19 backward: 23 slots per (neighbour, two-body
    bin) (logarithm, exponential and reciprocal at quarter rate = 12, and the
    polynomial in the log-distance), 15 per (neighbour pair, three-body bin)
    (exponential 5, the bin's distance and its square, the Gaussian's
    derivative, four FMAs) and 160 per neighbour pair (three square roots,
    reciprocals and sine/cosine pairs, the power, the cosine derivatives, and
    the gather along the pair's direction)."""
    return 23.0 * nb * n2 + 15.0 * pairs * n3 + 160.0 * pairs


# Single configurations of the paper's component timings: atoms, element
# counts (in the order of the representation's bins) and the mean number of
# neighbours within r_cut that the paper gives for each system.
COMPONENT_SYSTEMS = (
    ("aspirin-like", (8, 9, 4), 17.0),                 # H8 C9 O4
    ("brass-cluster-like", (225, 20), 46.0),           # Cu225 Zn20
    ("myoglobin-like", (632, 393, 107, 120, 8), 38.0),  # H C N O S, protein-like shares
)


def component_timing_leg(args, dev, log):
    """Energy + force evaluation of one configuration at a time, component by
    component (Results: component timings of one aspirin, one brass-cluster and
    one myoglobin configuration at N_F = 32768 and r_cut = 6 A). Synthetic
    molecule-like geometries of 21, 245 and 1260 atoms, scaled so that the mean
    number of neighbours within r_cut is the paper's (17, 46, 38); elements in
    the paper's proportions, shuffled. The chain: FCHL19 -> per-element
    projection to d = 128 -> energies -> dE/dx (d = 128, 256 stacks: N_F =
    32768) -> projection transpose -> FCHL19 backward (the forces). Each
    component is timed with HIP events, median of 20 runs after warm-up."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    prm_d = workloads.FCHL19_EF
    prm = sorf.fchl19_params(**prm_d)
    d, S, T = 128, 256, 3
    names = ["fchl19_forward", "project", "energies", "dE_dx", "project_transpose",
             "fchl19_backward"]
    out = {}
    for k, (name, counts, target) in enumerate(COMPONENT_SYSTEMS):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([220601580, 60 + k])))
        n, E = int(sum(counts)), len(counts)
        X = workloads.molecule_geometry(rng, n)
        dist = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
        lo, hi = 0.2, 5.0   # scale of the geometry with the target mean neighbour count
        for _ in range(50):
            mid = 0.5 * (lo + hi)
            if ((dist * mid < prm_d["rcut"]).sum(1) - 1).mean() > target:
                lo = mid
            else:
                hi = mid
        X = (X * 0.5 * (lo + hi)).astype(np.float32)
        nb = (np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)) < prm_d["rcut"]).sum(1) - 1
        el_np = rng.permutation(np.repeat(np.arange(E, dtype=np.int32), counts)).astype(np.int32)
        L = E * prm_d["n2"] + E * (E + 1) // 2 * prm_d["n3"] * 2
        model = sorf.Model.from_arrays(workloads.draw_signs(rng, E, T, S, d),
                                       workloads.draw_bias(rng, E, S * d), 4.0, dev)
        alpha = torch.from_numpy(rng.standard_normal(S * d).astype(np.float32)).to(dev)
        U = torch.from_numpy(workloads.random_projection(220601580 + 70 + k, E, L, d)).to(dev)
        proj, projT = sorf.Projector(U), sorf.Projector(U.transpose(1, 2).contiguous())
        Rt = torch.from_numpy(X).to(dev)
        el = torch.from_numpy(el_np).to(dev)
        ptr = torch.tensor([0, n], dtype=torch.int64, device=dev)
        rho = torch.empty((n, L), device=dev)
        x = torch.empty((n, d), device=dev)
        gx = torch.empty((n, d), device=dev)
        grho = torch.empty((n, L), device=dev)
        dR = torch.empty((n, 3), device=dev)
        Eout = torch.empty(1, device=dev)
        predictor = sorf.Predictor(model, dev)
        bx = sorf.Batch(x, el, ptr)

        def chain(ev=None):
            def mark(i):
                if ev is not None:
                    ev[i].record()
            mark(0)
            sorf.fchl19(Rt, el, ptr, E, prm, out=rho)
            mark(1)
            proj(rho, el, x)
            mark(2)
            predictor(bx, alpha, E=Eout)
            mark(3)
            sorf.backward(model, bx, alpha, out=gx)
            mark(4)
            projT(gx, el, grho)
            mark(5)
            sorf.fchl19_backward(Rt, el, ptr, E, grho, prm, out=dR)
            mark(6)

        for _ in range(3):
            chain()
        torch.cuda.synchronize()
        times = {nm: [] for nm in names}
        for _ in range(20):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            chain(ev)
            torch.cuda.synchronize()
            for i, nm in enumerate(names):
                times[nm].append(ev[i].elapsed_time(ev[i + 1]))
        med = {nm: float(np.median(v)) for nm, v in times.items()}
        total = sum(med.values())
        out[name] = {"atoms": n, "elements": E, "mean_neighbours": float(nb.mean()),
                     "max_neighbours": int(nb.max()), "component_ms": med, "total_ms": total,
                     "fchl19_share": (med["fchl19_forward"] + med["fchl19_backward"]) / total,
                     "sorf_share": (med["energies"] + med["dE_dx"]) / total}
        log(f"components: {name} {total:.3f} ms")
        del rho, x, gx, grho, dR
    torch.cuda.empty_cache()
    return {"workload": ("one configuration at a time: 21, 245 and 1260 atoms (aspirin-, brass- and "
                         "myoglobin-like), FCHL19 energy+force parameters, d=128, 256 stacks "
                         "(N_F=32768), energies and forces"),
            "systems": out}


def representation_leg(args, p, dev, log):
    """FCHL19 on the QM9-like batch (20,000 molecules, 360,149 atoms on synthetic
    molecule-like geometries, five elements, the paper's energy+force parameters,
    720 entries per atom): the representation, its backward pass, and the whole
    energy+force prediction chain of the paper (representation -> projection ->
    energies; dE/dx -> dE/drho through the projection's transpose -> forces)."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    t0 = time.perf_counter()
    R = workloads.host_geometries(p.mol_sizes(), seed=p.seed + 9)
    gen_s = time.perf_counter() - t0
    prm_d = workloads.FCHL19_EF
    prm = sorf.fchl19_params(**prm_d)
    Rt = torch.from_numpy(R).to(dev)
    el = torch.from_numpy(p.element).to(dev)
    ptr = torch.from_numpy(p.mol_ptr).to(dev)
    E, A, d = p.n_elements, p.n_atoms, p.d
    L = workloads.FCHL19_EF_SIZE
    rho = torch.empty((A, L), device=dev)
    dR = torch.empty((A, 3), device=dev)
    g = workloads.device_normal(A * L, p.seed + 10, 1.0, device=dev).view(A, L)
    U = torch.from_numpy(workloads.random_projection(p.seed + 11, E, L, d)).to(dev)
    Ut = U.transpose(1, 2).contiguous()
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    alpha = torch.ones(p.n_features, device=dev)
    predictor = sorf.Predictor(model, dev)
    proj, projT = sorf.Projector(U), sorf.Projector(Ut)
    x = torch.empty((A, d), device=dev)
    Eout = torch.empty(p.n_mols, device=dev)
    gx = torch.empty((A, d), device=dev)
    grho = torch.empty((A, L), device=dev)
    bx = sorf.Batch(x, el, ptr)

    def chain(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        sorf.fchl19(Rt, el, ptr, E, prm, out=rho)
        mark(1)
        proj(rho, el, x)
        mark(2)
        predictor(bx, alpha, E=Eout)
        mark(3)
        sorf.backward(model, bx, alpha, out=gx)
        mark(4)
        projT(gx, el, grho)
        mark(5)
        sorf.fchl19_backward(Rt, el, ptr, E, grho, prm, out=dR)
        mark(6)

    chain()
    sorf.fchl19_backward(Rt, el, ptr, E, g, prm, out=dR)
    torch.cuda.synchronize()
    names = ["fchl19_forward", "project", "energies", "dE_dx", "project_transpose", "fchl19_backward"]
    times = {k: [] for k in names}
    n = 3
    for _ in range(n):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        chain(ev)
        torch.cuda.synchronize()
        for k, nm in enumerate(names):
            times[nm].append(ev[k].elapsed_time(ev[k + 1]))
    med = {k: float(np.median(v)) for k, v in times.items()}
    slots, nb, pairs = fchl19_slots(R, p.mol_ptr, prm_d["rcut"], prm_d["n2"], prm_d["n3"])
    tops = slots / (med["fchl19_forward"] * 1e-3) / 1e12
    slots_b = fchl19_backward_slots(nb, pairs, prm_d["n2"], prm_d["n3"])
    tops_b = slots_b / (med["fchl19_backward"] * 1e-3) / 1e12
    out = {
        "workload": (f"{p.n_mols} QM9-like molecules, {A} atoms on synthetic geometries, {E} elements, "
                     f"FCHL19 energy+force parameters ({L} entries), {nb} neighbour entries, "
                     f"{pairs} neighbour pairs; projection {L} -> {d}, D={p.n_features}"),
        "phase_ms": med,
        "chain_ms": sum(med.values()),
        "atoms_per_s_energy_force": A / (sum(med.values()) * 1e-3),
        "roofline_fchl19_forward": {"bound": "alu", "achieved": tops, "peak": PEAK_VALU_TOPS,
                                    "unit": "T VALU-slots/s", "frac": tops / PEAK_VALU_TOPS,
                                    "traffic": None, "slots_per_launch": slots},
        "roofline_fchl19_backward": {"bound": "alu", "achieved": tops_b, "peak": PEAK_VALU_TOPS,
                                     "unit": "T VALU-slots/s", "frac": tops_b / PEAK_VALU_TOPS,
                                     "traffic": None, "slots_per_launch": slots_b},
        "geometry_gen_s": gen_s,
    }
    if not args.no_cpu_baseline:
        from oracle import fchl19_oracle as F
        k = 40
        a1 = int(p.mol_ptr[k])
        t1 = time.perf_counter()
        F.fchl19(R[:a1].astype(np.float64), p.element[:a1], p.mol_ptr[:k + 1], E, prm_d)
        t = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": a1 / t, "unit": "atoms/s (FCHL19 forward)",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"FP64 oracle FCHL19 of {k} molecules ({a1} atoms), {t:.2f} s"}
    del rho, dR, g, U, Ut, x, gx, grho
    torch.cuda.empty_cache()
    return out


def precision_study(args, dev, log):
    """Gram precision modes on the precision workload (100,000 QM9-like
    molecules, D = 16384, lambda = 1e-8, 3 refinement steps): coefficient and
    energy errors of each mode against the FP64 Gram + FP64 solve (the
    paper's double-precision training), all on the GPU."""
    import torch

    from paper_2206_01580_amd import sorf, workloads
    p = workloads.precision_batch(n_mols=args.precision_mols)
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    D, M = p.n_features, p.n_mols
    y = torch.from_numpy(p.y).to(dev)
    Z = sorf.forward(model, batch)
    solver = sorf.Solver(D, device=dev)
    ws = sorf.GramWorkspace(dev)

    def energies(alpha):
        out = torch.empty(M, dtype=torch.float64, device=dev)
        for r0 in range(0, M, 8192):
            out[r0:r0 + 8192] = Z[r0:r0 + 8192].double() @ alpha
        return out

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    G64 = torch.zeros(D, D, dtype=torch.float64, device=dev)
    r64 = torch.zeros(D, dtype=torch.float64, device=dev)
    t_g = timed(lambda: sorf.gram_accumulate(Z, G64, y, r64, precision="fp64"))
    a_ref = solver(G64, r64, p.lam, args.n_refine).clone()
    torch.cuda.synchronize()
    info_ref = int(solver.info.item())
    del G64, r64
    torch.cuda.empty_cache()
    E_ref = energies(a_ref)
    y64 = y.double()
    rms_ref = float(torch.sqrt(torch.mean(E_ref ** 2)))
    res = {"fp64": {"gram_ms": t_g, "info": info_ref,
                    "fit_rmse": float(torch.sqrt(torch.mean((E_ref - y64) ** 2)))}}
    log(f"precision: reference done (info {info_ref})")
    G = torch.empty(D, D, device=dev)
    r = torch.empty(D, device=dev)
    for mode in ("split", "fp32", "fp32_kahan", "bf16", "fp16", "bf16_hilo", "fp16_hilo"):
        if mode == "split":
            G = torch.zeros(D, D, dtype=torch.float64, device=dev)
            r = torch.zeros(D, dtype=torch.float64, device=dev)
        elif G.dtype != torch.float32:
            G = torch.empty(D, D, device=dev)
            r = torch.empty(D, device=dev)
            torch.cuda.empty_cache()
        G.zero_()
        r.zero_()
        k = sorf.fp16_scale_exp(29 * math.sqrt(2.0 / D)) if mode.startswith("fp16") else 0
        t = timed(lambda: sorf.gram_accumulate(Z, G, y, r, precision=mode, scale_exp=k,
                                               workspace=ws))
        a = solver(G, r, p.lam, args.n_refine)
        torch.cuda.synchronize()
        info = int(solver.info.item())
        E = energies(a)
        dE = E - E_ref
        res[mode] = {
            "gram_ms": t, "gram_tflops": float(M) * D * (D + 1) / (t * 1e-3) / 1e12, "info": info,
            "alpha_rel_err": float(torch.linalg.norm(a - a_ref) / torch.linalg.norm(a_ref)),
            "energy_max_rel_err": float(dE.abs().max()) / rms_ref,
            "energy_rms_rel_err": float(torch.sqrt(torch.mean(dE ** 2))) / rms_ref,
            "fit_rmse": float(torch.sqrt(torch.mean((E - y64) ** 2))),
        }
        log(f"precision: {mode} done")
    del G, r, Z, solver, ws
    torch.cuda.empty_cache()
    return {"workload": f"{M} QM9-like molecules, d=128, 128 stacks (D={D}), sigma=4, "
                        f"lambda={p.lam:g}, {args.n_refine} refinement steps",
            "reference": "FP64 Gram + FP64 Cholesky on the GPU (paper's DP training)",
            "energy_errors_relative_to": "rms of the reference energies", "modes": res}


def cpu_baseline(p, D, n_sample, lam):
    """The FP64 oracle (dense W) on the host cores: per-molecule work (features,
    Gram rows, energies, dE/dx) timed on a sample of molecules and scaled to the
    full batch, plus one full-size FP64 solve. Returns atom-features/s."""
    from oracle import sorf_oracle as O
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(0)
    mols = np.sort(rng.choice(p.n_mols, size=n_sample, replace=False))
    q = p.subset(mols)
    alpha = rng.standard_normal(D)
    t0 = time.perf_counter()
    Z = O.molecule_features(q.x, q.element, q.mol_ptr, q.signs, q.bias, q.sigma)
    G, r = O.gram(Z, q.y)
    O.predict_energies(Z, alpha)
    O.grad_x(q.x, q.element, q.mol_ptr, q.signs, q.bias, q.sigma, alpha)
    t_mol = time.perf_counter() - t0
    # one full-size solve on a well-conditioned SPD matrix of the same size
    A = G + (np.abs(G).max() + 1.0) * np.eye(D)
    t1 = time.perf_counter()
    O.solve(A, r, lam)
    t_solve = time.perf_counter() - t1
    t_step = t_mol * (p.n_mols / n_sample) + t_solve
    af = float(p.n_atoms) * D
    return {"value": af / t_step, "unit": "atom-features/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 dense-W oracle on {n_sample} of {p.n_mols} molecules "
                       f"({q.n_atoms} atoms; features, Gram rows, energies, dE/dx: {t_mol:.2f} s, "
                       f"scaled x{p.n_mols / n_sample:.1f}) + one full D={D} Cholesky solve "
                       f"({t_solve:.2f} s)")}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (the multi-GPU sharding is not implemented); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2206_01580_amd import sorf, workloads

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 18                    # floats
        src = torch.ones(n, device=dev)
        dst = torch.empty(n, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    t_gen = time.perf_counter()
    p = workloads.qm9_batch(n_mols=args.n_mols)
    gen_s = time.perf_counter() - t_gen
    D, A, M = p.n_features, p.n_atoms, p.n_mols
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    y = torch.from_numpy(p.y).to(dev)
    acc_t = torch.float64 if args.gram in ("fp64", "split") else torch.float32
    Z = torch.empty(M, D, device=dev)
    G = torch.empty(D, D, device=dev, dtype=acc_t)
    Zty = torch.empty(D, device=dev, dtype=acc_t)
    gram_ws = sorf.GramWorkspace(dev)
    gram_ws.get(M, D, args.gram) if args.gram != "fp64" else None   # allocate before timing
    solver = sorf.Solver(D, device=dev)
    alpha = torch.empty(D, device=dev, dtype=torch.float64)
    energy_grad = sorf.EnergyGrad(model, dev)
    E = torch.empty(M, device=dev)
    grad = torch.empty(A, p.d, device=dev)
    scale_exp = sorf.fp16_scale_exp(29 * math.sqrt(2.0 / D)) if args.gram.startswith("fp16") else 0
    torch.cuda.synchronize()

    # energies and dE/dx come from one adjoint pass over the features
    phases = ["forward", "gram", "solve", "energy_grad"]
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in phases}
    times = {k: [] for k in phases}

    def step(record: bool):
        def mark(k, i):
            if record:
                ev[k][i].record()
        mark("forward", 0)
        sorf.forward(model, batch, out=Z)
        mark("forward", 1)
        G.zero_()
        Zty.zero_()
        mark("gram", 0)
        sorf.gram_accumulate(Z, G, y, Zty, precision=args.gram, scale_exp=scale_exp,
                             workspace=gram_ws)
        mark("gram", 1)
        mark("solve", 0)
        solver(G, Zty, args.lam, args.n_refine, out=alpha)
        mark("solve", 1)
        a32 = alpha.float()
        mark("energy_grad", 0)
        energy_grad(batch, a32, E=E, grad=grad)
        mark("energy_grad", 1)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    info = int(solver.info.item())

    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        for k in phases:
            times[k].append(ev[k][0].elapsed_time(ev[k][1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    af = float(A) * D
    med = {k: float(np.median(v)) for k, v in times.items()}

    # rooflines of the main kernels from their HIP-event times
    gram_flop = float(M) * D * (D + 1)
    gram_tf = gram_flop / (med["gram"] * 1e-3) / 1e12
    fwd_slots = valu_slots_per_feature(p.d, p.n_transforms) * af
    fwd_tops = fwd_slots / (med["forward"] * 1e-3) / 1e12
    bwd_slots = valu_slots_per_feature(p.d, p.n_transforms, backward=True) * af
    bwd_tops = bwd_slots / (med["energy_grad"] * 1e-3) / 1e12
    chol_flop = D ** 3 / 3.0
    mfma_work = MFMA_WORK.get(args.gram, 1.0)
    rooflines = {
        "gram": {"bound": "mfma", "achieved": gram_tf, "peak": PEAK_MFMA_TFLOPS[args.gram],
                 "unit": "TFLOP/s", "frac": gram_tf / PEAK_MFMA_TFLOPS[args.gram], "traffic": None,
                 "ms": med["gram"], "mode": args.gram, "mfma_executed_tflops": gram_tf * mfma_work,
                 "mfma_utilisation": gram_tf * mfma_work / PEAK_MFMA_TFLOPS[args.gram]},
        "forward": {"bound": "alu", "achieved": fwd_tops, "peak": PEAK_VALU_TOPS,
                    "unit": "T VALU-slots/s", "frac": fwd_tops / PEAK_VALU_TOPS, "traffic": None,
                    "ms": med["forward"]},
        "energy_grad": {"bound": "alu", "achieved": bwd_tops, "peak": PEAK_VALU_TOPS,
                        "unit": "T VALU-slots/s", "frac": bwd_tops / PEAK_VALU_TOPS,
                        "traffic": None, "ms": med["energy_grad"]},
        "solve": {"bound": "mfma", "achieved": chol_flop / (med["solve"] * 1e-3) / 1e12,
                  "peak": PEAK_MFMA_TFLOPS["fp64"], "unit": "TFLOP/s",
                  "frac": chol_flop / (med["solve"] * 1e-3) / 1e12 / PEAK_MFMA_TFLOPS["fp64"],
                  "traffic": None, "ms": med["solve"]},
    }
    # the dominant single kernel launch (the solve phase is ~1000 launches of 9 kernels)
    cnt = measured_gram_counters(args.gram, M, D)
    if cnt is not None:
        rooflines["gram"]["traffic"] = cnt["hbm_bytes"]
        rooflines["gram"]["mfma_busy_counter"] = cnt["mfma_busy"]
        rooflines["gram"]["clock_ghz_counter"] = cnt["clock_ghz"]
    dominant = max(("gram", "forward", "energy_grad"), key=lambda k: med[k])
    roof = {k: v for k, v in rooflines[dominant].items() if k != "ms"}
    roof["kernel"] = dominant

    gram_dtype = {"fp32": "fp32", "fp32_kahan": "fp32 (Kahan block sums)", "fp64": "f64",
                  "bf16": "bf16 x1", "fp16": "fp16 x1", "bf16_hilo": "bf16 hi+lo",
                  "fp16_hilo": "fp16 hi+lo", "split": "int8 head + fp16 tail, f64 G"}[args.gram]
    out = {
        "metric": "SORF atom-features/s fwd+bwd; Gram TFLOP/s; force-request p50/p99 vs plain",
        "value": af / (ms_step * 1e-3),
        "unit": "atom-features/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f32 features / {gram_dtype} Gram / f64 solve",
        "data": "synthetic",
        "config": {"workload": "qm9-like train+infer step: 20000 molecules (3..29 atoms), d=128, "
                               "64 stacks (D=8192), 3 transforms, sigma=4; forward, Gram (" + args.gram +
                               "), FP64 solve, energies and dE/dx (one adjoint pass)",
                   "n_mols": M, "n_atoms": A, "D": D, "gram": args.gram, "lambda": args.lam,
                   "n_refine": args.n_refine},
        "fwd_bwd_atom_features_per_s": af / ((med["forward"] + med["energy_grad"]) * 1e-3),
        "gram_tflops": gram_tf,
        "roofline": roof,
        "phase_ms": med,
        "forward_atom_features_per_s": af / (med["forward"] * 1e-3),
        "rooflines": rooflines,
        "solve_info": info,
        "gen_s": gen_s,
    }
    # other Gram modes on the same Z: labelled extras, not the step's arithmetic
    extra = {}
    for mode in [m.strip() for m in args.gram_modes.split(",") if m.strip()]:
        if mode == args.gram:
            continue
        dt = torch.float64 if mode in ("fp64", "split") else torch.float32
        Gm = G if dt == acc_t else torch.empty(D, D, device=dev, dtype=dt)
        rm = torch.empty(D, device=dev, dtype=dt)
        km = sorf.fp16_scale_exp(29 * math.sqrt(2.0 / D)) if mode.startswith("fp16") else 0
        gram_ws.get(M, D, mode)
        ts = []
        for it in range(4):
            Gm.zero_()
            rm.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sorf.gram_accumulate(Z, Gm, y, rm, precision=mode, scale_exp=km, workspace=gram_ws)
            e1.record()
            torch.cuda.synchronize()
            if it > 0:
                ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        tf = gram_flop / (ms * 1e-3) / 1e12
        work = MFMA_WORK.get(mode, 1.0)
        extra[mode] = {"ms": ms, "algorithmic_tflops": tf, "peak": PEAK_MFMA_TFLOPS[mode],
                       "frac": tf / PEAK_MFMA_TFLOPS[mode], "mfma_executed_tflops": tf * work,
                       "mfma_utilisation": tf * work / PEAK_MFMA_TFLOPS[mode]}
        del Gm, rm
        log(f"gram {mode}: {ms:.2f} ms")
    out["gram_modes"] = extra
    # context for the solve: the vendor FP64 Cholesky (torch.linalg.cholesky_ex,
    # rocSOLVER) on the same G + lambda I, against the factorisation and first
    # solve here (no refinement); median of 3 after one untimed call each
    if G.dtype == torch.float32:
        A64 = G.double()
        A64 = torch.tril(A64) + torch.tril(A64, -1).t()
        A64.diagonal().add_(args.lam)

        def med3(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return float(np.median(ts))
        vendor_ms = med3(lambda: torch.linalg.cholesky_ex(A64))
        ours_ms = med3(lambda: solver(G, Zty, args.lam, 0, out=alpha))
        out["solve_vs_vendor"] = {"torch_cholesky_ex_f64_ms": vendor_ms,
                                  "factor_and_first_solve_ms": ours_ms, "D": D}
        log(f"solve: vendor cholesky {vendor_ms:.2f} ms, ours (no refinement) {ours_ms:.2f} ms")
        del A64
    del Z, G, model, batch, energy_grad, solver, grad, gram_ws
    torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        out["serving"] = serving_leg(args, dev, log, args.serve_rate, args.serve_seconds)
        sweep = [float(r) for r in args.serve_sweep.split(",") if r.strip()]
        out["serving_load_sweep"] = [
            serving_leg(args, dev, log, r, args.serve_sweep_requests / r) for r in sweep]
    if args.force_confs > 0:
        out["force_training"] = force_training_leg(args, dev, log)
    if args.projection:
        log("projection")
        out["projection"] = projection_leg(args, p, dev, log)
    if args.ntransform_study:
        out["ntransform_study"] = ntransform_study(args, p, dev, log)
    if args.roundoff_study:
        out["roundoff_study"] = roundoff_study(args, p, dev, log)
    if args.representation:
        log("representation")
        out["representation"] = representation_leg(args, p, dev, log)
    if args.components:
        log("component timings")
        out["component_timings"] = component_timing_leg(args, dev, log)
    if args.precision_mols > 0:
        out["precision_study"] = precision_study(args, dev, log)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(p, D, args.cpu_sample_mols, args.lam)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
