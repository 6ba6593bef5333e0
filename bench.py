#!/usr/bin/env python3
"""Throughput of the sketched-ANLS (DSANLS) hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one outer iteration of the method (update_U then update_V, Alg. 2
with one node) on synthetic data already resident in HBM.

The default workload measures the metric to a fixed relative objective: the
dense 50000 x 20000 planted rank-128 matrix with 1% noise, k = 128, Gaussian
sketch d = d' = 4096, one prox-CD sweep per update, run as plain FP32 and as
the BF16 form (sketch GEMM in BF16 on the matrix cores, FP32 accumulation).
For each of three data seeds the plain FP32 run takes K iterations
(K = --steps, default 30) and its final relative objective is that seed's
eps*; the BF16 form then runs until its objective is <= eps* (1 + 1e-3).
Every iteration is timed on its own between device synchronisations (the
objective, evaluated after it, is outside the timed region).  value is the
BF16 form's iterations/s over its runs to eps*; the line also carries each
form's iterations and time to eps*, the speed-up, the per-update error of
both forms against the plain FP64 oracle on sampled rows, the roofline of
the BF16 sketch GEMM, and the CPU oracle timed on a bounded sample.

Other workloads (--workload) time K iterations at a fixed count.  W warm-up
iterations run first, then U and V are reset to U^0, V^0.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0,
        "fp32_valu_tflops": 78.6}

WORKLOADS = {
    # the small FP64-checkable case (parity configuration)
    "dense-200x150": dict(kind="dense", m=200, n=150, k=10, d=40, iters=20, solver="pgd",
                          gen="uniform", precision="fp32", alpha=0.1, beta=1.0),
    # plain FP32 on one GPU (the default bench line)
    "dense-20000x10000": dict(kind="dense", m=20000, n=10000, k=64, d=1024, iters=50, solver="prox_cd",
                              gen="planted", noise=0.01, noise_relative=False, precision="fp32", alpha=1.0, beta=0.1),
    # precision form: planted rank-128 + 1% noise, FP32 and BF16 sketch GEMM
    "dense-50000x20000-fp32": dict(kind="dense", m=50000, n=20000, k=128, d=4096, iters=30,
                                   solver="prox_cd", gen="planted", noise=0.01, noise_relative=True,
                                   precision="fp32", alpha=0.1, beta=10.0),
    "dense-50000x20000-bf16": dict(kind="dense", m=50000, n=20000, k=128, d=4096, iters=30,
                                   solver="prox_cd", gen="planted", noise=0.01, noise_relative=True,
                                   precision="bf16", alpha=0.1, beta=10.0),
    # text-shaped CSR row block, subsampling sketch (columns sampled and scaled)
    "sparse-500000x200000": dict(kind="sparse", m=500000, n=200000, k=100, d=2000, iters=30,
                                 solver="prox_cd", nnz=100_000_000, precision="fp32", alpha=0.1, beta=0.1),
    # learned warm start on the same data: pairs from 5 plain to-tolerance
    # runs (sketch seeds 1-5), training, then cold vs warm on sketch seed 6
    "sparse-500000x200000-warm": dict(kind="warm", m=500000, n=200000, k=100, d=2000, iters=10,
                                      solver="prox_cd", nnz=100_000_000, precision="fp32", hidden=256,
                                      pairs=1_000_000, runs=5, run_iters=20, label_tol=1e-6, tol=1e-4,
                                      max_sweeps=200, epochs=20, batch=4096, lr=1e-4, alpha=0.1, beta=0.1),
}
# the further sketch kinds of Sec. 3.4 on the same data shapes
WORKLOADS["dense-20000x10000-count"] = dict(WORKLOADS["dense-20000x10000"], sketch="count")
WORKLOADS["dense-20000x10000-srht"] = dict(WORKLOADS["dense-20000x10000"], sketch="srht")
WORKLOADS["sparse-500000x200000-count"] = dict(WORKLOADS["sparse-500000x200000"], sketch="count")
# synthetic analogues of the paper's rank sweep and solver comparison
# (Sec. 5.3): relative objective and time per iteration
WORKLOADS["sparse-500000x200000-ksweep"] = dict(WORKLOADS["sparse-500000x200000"], kind="ksweep",
                                                ks=(20, 50, 100, 200, 500), iters=10)
WORKLOADS["pgd-vs-cd"] = dict(kind="pgd_vs_cd", iters=20,
                              cases=(dict(name="dense-200x150", m=200, n=150, k=10, d=40, gen="uniform", iters=20,
                                          pgd=dict(alpha=0.1, beta=1.0), prox_cd=dict(alpha=1.0, beta=1.0)),
                                     dict(name="dense-20000x10000", m=20000, n=10000, k=64, d=1024, gen="planted",
                                          noise=0.01, noise_relative=False, iters=50)))
# the paper's proximal weight grid (Sec. 5.2): mu_t = alpha + beta t with
# alpha, beta in {0.1, 1, 10}, the best chosen per data set; here per
# workload, by the relative objective after the workload's iterations
WORKLOADS["mu-grid"] = dict(kind="mu_grid", iters=None, grid=(0.1, 1.0, 10.0),
                            cases=("dense-20000x10000", "sparse-500000x200000", "dense-50000x20000-fp32"))
DEFAULT = "dense-50000x20000"
# the precision form measured to a fixed relative objective (the default)
TO_EPS = {"dense-50000x20000": dict(kind="to_eps", m=50000, n=20000, k=128, d=4096, iters=30,
                                    solver="prox_cd", gen="planted", noise=0.01, noise_relative=True,
                                    seeds=(0, 1, 2), max_factor=3, sample_rows=256, alpha=0.1, beta=10.0)}
WORKLOADS.update(TO_EPS)


def describe(name, w, K=None):
    iters = K if K is not None else w["iters"]
    if "alpha" in w and w["kind"] in ("to_eps", "warm", "sparse", "dense"):
        return _describe(name, w, iters) + f", mu_t = {w['alpha']:g} + {w['beta']:g} t"
    return _describe(name, w, iters)


def _describe(name, w, iters):
    if w["kind"] == "ksweep":
        return (f"CSR {w['m']}x{w['n']}, {w['nnz']:.0e} nnz text-shaped, subsampling d=d'={w['d']}, prox-CD 1 sweep, "
                f"k in {list(w['ks'])}, {iters} iterations each")
    if w["kind"] == "pgd_vs_cd":
        return "PGD vs prox-CD, relative objective per iteration: " + ", ".join(
            f"{c['name']} k={c['k']} d={c['d']} ({c['iters']} iterations)" for c in w["cases"])
    if w["kind"] == "to_eps":
        return (f"dense {w['m']}x{w['n']} planted rank-{w['k']} |N(0,1)| factors + {w['noise']:.0%} noise, "
                f"k={w['k']}, Gaussian sketch d=d'={w['d']}, prox-CD 1 sweep; plain FP32 for {iters} iterations "
                f"sets eps* per data seed, the BF16 sketch-GEMM form runs to eps*(1+1e-3); "
                f"{len(w['seeds'])} data seeds")
    if w["kind"] == "warm":
        return (f"CSR {w['m']}x{w['n']}, {w['nnz']:.0e} nnz text-shaped, k={w['k']}, subsampling d=d'={w['d']}, "
                f"prox-CD to tolerance {w['tol']}, MLP warm start [a_i (d); u_i (k)] -> {w['hidden']} -> k "
                f"trained on {w['pairs']:.0e} pairs from {w['runs']} plain runs, {w['iters']} iterations")
    if w["kind"] == "sparse":
        kind = "count sketch" if w.get("sketch") == "count" else "subsampling sketch"
        return (f"CSR {w['m']}x{w['n']}, {w['nnz']:.0e} nnz, power-law rows (alpha=1.5), Zipf(1.1) "
                f"columns, lognormal values, k={w['k']}, {kind} d=d'={w['d']}, "
                f"prox-CD 1 sweep, FP32, {iters} iterations")
    if w["kind"] == "dense":
        gen = ("uniform[0,1)" if w["gen"] == "uniform" else
               f"planted rank-{w['k']} |N(0,1)| factors + noise")
        kind = {"count": "count sketch", "srht": "SRHT"}.get(w.get("sketch"), "Gaussian sketch")
        return (f"dense {w['m']}x{w['n']} {gen}, k={w['k']}, {kind} d=d'={w['d']}, "
                f"{'prox-CD 1 sweep' if w['solver'] == 'prox_cd' else 'PGD'}, "
                f"sketch GEMM {w['precision'].upper()}, {iters} iterations")
    return name


def make_dense(w, seed=0):
    from paper_2009_02845_amd import synth
    m, n, k = w["m"], w["n"], w["k"]
    if w["gen"] == "uniform":
        M = synth.dense_uniform(m, n, seed)
    else:
        M = synth.planted_dense(m, n, k, seed, noise_sd=w["noise"], noise_relative=w["noise_relative"])
    U0, V0 = synth.init_factors(m, n, k, seed)
    return M, U0, V0


def make_sparse(w, seed=0):
    import scipy.sparse as sp
    from paper_2009_02845_amd import synth
    m, n, k = w["m"], w["n"], w["k"]
    rp, ci, v = synth.sparse_text(m, n, w["nnz"], seed)
    M = sp.csr_matrix((v, ci, rp), shape=(m, n))
    Mt = M.T.tocsr()
    Mt.sort_indices()
    U0, V0 = synth.init_factors(m, n, k, seed)
    return M, Mt, U0, V0


def cpu_baseline(w, M, U0, V0, budget_s=12.0, max_iters=5, Mt=None, half=False):
    """The FP64 oracle, untuned, timed on the host's cores over whole
    iterations (half=True: one U half-iteration, counted as half an
    iteration, for the workloads where a whole one takes about a minute)."""
    from oracle import dsanls as O
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    sketch = O.SKETCH_SUBSAMPLE if w["kind"] == "sparse" else O.SKETCH_GAUSSIAN
    sketch = {"count": O.SKETCH_COUNT, "srht": O.SKETCH_SRHT}.get(w.get("sketch"), sketch)
    cfg = O.Config(k=w["k"], d=w["d"], d_prime=w["d"], sketch=sketch, solver=w["solver"],
                   alpha=w.get("alpha", 1.0), beta=w.get("beta", 1.0))
    M64 = M.astype(np.float64)
    Mt64 = Mt.astype(np.float64) if Mt is not None else None
    U, V = U0.astype(np.float64), V0.astype(np.float64)
    if half:
        t0 = time.perf_counter()
        O.update_U(M64, U, V, 0, cfg)
        el = time.perf_counter() - t0
        return {"value": 0.5 / el, "unit": "iterations/s", "cores": int(cores), "kind": "oracle",
                "sample": f"one U half-iteration (t=0) of the same workload in FP64 numpy, {el:.1f} s, "
                          f"counted as half an iteration"}
    done, t0 = 0, time.perf_counter()
    while done < max_iters:
        U = O.update_U(M64, U, V, done, cfg)
        V = O.update_V(M64, U, V, done, cfg, Mt=Mt64)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "iterations/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{done} full iterations (t=0..{done - 1}) of the same workload in FP64 numpy, "
                      f"{el:.1f} s"}


# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged over the profiled
# launches), each scaled by what the same counter reads for a plain copy of
# 1 GiB on the same GPU (FETCH_SIZE reads 524300 KiB of the 1048576 read:
# x2.0; WRITE_SIZE reads 1048576: x1.0).  The figure holds only for the
# kernel sources it was taken with (sha256 of the listed files, in order);
# after any change to them the traffic is reported as null.
CAL_FETCH, CAL_WRITE = 2.0, 1.0
TRAFFIC = {
    "dense-20000x10000": {"files": ["gemm.hip"],
                          "sha256": "528bbd6a909efc6db290b4aa3aadad6fff075009e7c6bd17c23241f09d68dd09",
                          "fetch_kib": 2419643.13, "write_kib": 120000.0},
    "sparse-500000x200000": {"files": ["nnls.hip"],
                             "sha256": "1f70c9e0ef0a11b1bf1f049d0fe273e332f1c5d0590c79c98b9edd13d5d9d146",
                             "fetch_kib": 192211.72, "write_kib": 146972.8},
    "dense-50000x20000-bf16": {"files": ["gemm.hip"],
                               "sha256": "528bbd6a909efc6db290b4aa3aadad6fff075009e7c6bd17c23241f09d68dd09",
                               "fetch_kib": 19776476.63, "write_kib": 1120000.0},
}


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2009_02845_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(workload):
    t = TRAFFIC.get(workload)
    if t is None or sources_sha256(t["files"]) != t["sha256"]:
        return None
    return 1024.0 * (CAL_FETCH * t["fetch_kib"] + CAL_WRITE * t["write_kib"])


def sparse_roofline(w, M, tm, launches, workload):
    """Roofline of the dominant sparse kernel, the NNLS sweep (the longest
    single launch), with the sampled-column sketch product beside it (HBM; a
    phase of about a dozen short kernels per side).  The sweep moves 12 k
    bytes per row (U and R read, U written) for 2 k^2 flop, k / 6 flop per
    byte: at k = 100 below the FP32 matrix-core ridge (157.3 TFLOP/s over
    8 TB/s, about 19.7 flop/B), so its roof is HBM bandwidth."""
    m, n, k, d = w["m"], w["n"], w["k"], w["d"]
    nnz = M.nnz
    half = launches // 2
    nnls_avg = tm["nnls_ms"] / 1e3 / launches
    prod_avg = tm["product_ms"] / 1e3 / launches
    flops = 2.0 * k * k * (m + n) / 2      # k^2 FMAs per row-sweep, mean over the two sides
    nbytes = 12.0 * k * (m + n) / 2        # U and R read, U written, mean over the two sides
    ach = nbytes / nnls_avg / 1e9
    tflops = flops / nnls_avg / 1e12
    # sampled-column gather: E = nnz d / lng sampled entries per side (their
    # expectation under uniform sampling), each read once from CSR(X^T)
    # (8 B), written to and read back from the sketched rows (16 B); R
    # written (4 k B per row) and the row offsets (8 B per row)
    e_u, e_v = nnz * d / n, nnz * d / m
    moved = (24.0 * (e_u + e_v) + (4.0 * k + 8.0) * (m + n)) / 2
    pach = moved / prod_avg / 1e9
    kern = "prox_cd_mfma_kernel" if k % 4 == 0 and 64 < k <= 100 else "prox_cd_lds_kernel"
    if w.get("sketch") == "count":
        # the count sketch keeps every nonzero: R = (X S) B^T streams all nnz
        # of X, each adding s_j M_ij B^T[h_j, :] (k FMAs, the row of B^T
        # from L2) - 2 nnz k flop per side on the VALU, the dominant phase;
        # HBM moves the CSR (8 B per nnz, 8 B per row) and R (4 k B per row)
        flops_p = 2.0 * nnz * k
        hbm_p = 8.0 * nnz + (8.0 + 4.0 * k) * (m + n) / 2
        tf = flops_p / prod_avg / 1e12
        return {"kernel": "count-sketch product R = (X S) B^T from the nnz stream (csr_rhs_seg_kernel, hashed)",
                "bound": "alu", "achieved": tf, "peak": PEAK["fp32_valu_tflops"], "unit": "TFLOP/s",
                "frac": tf / PEAK["fp32_valu_tflops"], "traffic": None, "flops_per_launch": flops_p,
                "hbm_bytes_per_launch": hbm_p, "hbm_gbs": hbm_p / prod_avg / 1e9,
                "avg_launch_ms": prod_avg * 1e3, "sides_timed": half * 2,
                "nnls": {"kernel": f"prox-CD sweep ({kern})", "bound": "hbm", "achieved": ach,
                         "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": ach / PEAK["hbm_gbs"],
                         "avg_launch_ms": nnls_avg * 1e3}}
    return {"kernel": f"prox-CD sweep ({kern})", "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"],
            "unit": "GB/s", "frac": ach / PEAK["hbm_gbs"], "traffic": traffic_bytes(workload),
            "bytes_per_launch": nbytes, "flops_per_launch": flops, "tflops": tflops,
            "frac_of_fp32_mfma": tflops / PEAK["fp32_mfma_tflops"], "avg_launch_ms": nnls_avg * 1e3,
            "product_phase": {"kernels": "gather_len, scans, gather_entries, row_sort_long, a_rhs, a_rhs_long",
                              "bound": "hbm", "achieved": pach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                              "frac": pach / PEAK["hbm_gbs"], "bytes_per_side": moved,
                              "avg_ms_per_side": prod_avg * 1e3, "sides_timed": half * 2}}


def run_warm(args, w, torch, B):
    """Learned warm start: pair generation, training and cold/warm comparison."""
    import scipy.sparse as sp
    m, n, k, d, H = w["m"], w["n"], w["k"], w["d"], w["hidden"]
    dev = torch.device("cuda", 0)
    print("[bench] generating data", file=sys.stderr, flush=True)
    M, Mt, U0, V0 = make_sparse(w, args.seed)
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
    keep = [to(M.indptr, np.int64), to(M.indices, np.int32), to(M.data, np.float32),
            to(Mt.indptr, np.int64), to(Mt.indices, np.int32), to(Mt.data, np.float32)]
    mat = B.csr_matrix(*keep)
    U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)

    def solver(seed, tol, warm_hidden=0):
        U, V = U0d.clone(), V0d.clone()
        cfg = B.make_config(m, n, k, d, d, sketch="subsample", solver="prox_cd", sweeps=0, tol=tol,
                            max_sweeps=w["max_sweeps"], alpha=w.get("alpha", 1.0), beta=w.get("beta", 1.0), seed=seed,
                            warm_hidden=warm_hidden)
        return B.Solver(cfg, mat, U, V, tensors=keep), U, V

    # 1) training pairs (a_i, u_i^t) -> to-tolerance solution u_i*
    t0 = time.perf_counter()
    per_update = w["pairs"] // (w["runs"] * w["run_iters"] * 2)
    gen = torch.Generator(device="cpu").manual_seed(1234)
    A_parts, Ut_parts, Ys_parts = [], [], []
    for run in range(1, w["runs"] + 1):
        s, U, V = solver(run, w["label_tol"])
        s.keep_sketched_rows(True)
        for t in range(w["run_iters"]):
            for side, W, rows in ((0, U, m), (1, V, n)):
                sel = torch.randint(0, rows, (per_update,), generator=gen, dtype=torch.int32).to(dev)
                ut = W.index_select(0, sel.long()).clone()
                (s.update_U if side == 0 else s.update_V)(t)
                ys = W.index_select(0, sel.long()).clone()
                rp, cols, vals = s.gather_sketched_rows(sel, capacity=per_update * 512)
                A_parts.append(sp.csr_matrix((vals.cpu().numpy(), cols.cpu().numpy(), rp.cpu().numpy()),
                                             shape=(per_update, d)))
                Ut_parts.append(ut.cpu().numpy())
                Ys_parts.append(ys.cpu().numpy())
        s.close()
    A_all = sp.vstack(A_parts).tocsr()
    Ut_all = np.concatenate(Ut_parts)
    Ys_all = np.concatenate(Ys_parts)
    t_pairs = time.perf_counter() - t0
    print(f"[bench] {A_all.shape[0]} pairs in {t_pairs:.1f} s", file=sys.stderr, flush=True)

    # 2) training on the GPU (the library's forward/backward/Adam kernels):
    # the plain two-layer network (the specified form) and the residual
    # variant y = ReLU(u + W2 h + b2), same data, batches and schedule
    from paper_2009_02845_amd import synth
    bs = w["batch"]
    perm = np.random.default_rng(5).permutation(A_all.shape[0])
    batches = []
    for b0 in range(0, len(perm) - bs + 1, bs):
        idx = perm[b0:b0 + bs]
        Ab = A_all[idx]
        Cb = Ab.tocsc()
        batches.append((to(Ab.indptr, np.int32), to(Ab.indices, np.int32), to(Ab.data, np.float32),
                        to(Cb.indptr, np.int32), to(Cb.indices, np.int32), to(Cb.data, np.float32),
                        to(Ut_all[idx], np.float32), to(Ys_all[idx], np.float32)))
    nets, training = {}, {}
    for form in ("plain", "residual"):
        t0 = time.perf_counter()
        p0 = synth.mlp_init(d, k, H, args.seed)
        # data-dependent scales: the sketched values are sqrt(n/d) M_ij, far
        # from unit scale, so W1a starts divided by their mean; the plain
        # network's output bias starts at the mean label (the residual one
        # starts at u_i^t itself)
        p0["W1a"] = (p0["W1a"] / max(float(np.mean(np.abs(A_all.data))), 1e-12)).astype(np.float32)
        if form == "plain":
            p0["b2"] = np.mean(Ys_all, axis=0).astype(np.float32)
        params = B.mlp_pack(p0, device=dev)
        net = B.MLP(d, k, H, params, max_rows=bs, residual=form == "residual")
        losses = []
        for ep in range(w["epochs"]):
            tot = 0.0
            for bt in batches:
                net.train_step(bt, w["lr"])
                tot += net.last_loss()
            losses.append(tot / len(batches))
            print(f"[bench] {form} epoch {ep}: mean loss {losses[-1]:.4g}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        nets[form] = params
        training[form] = {"epoch_loss": losses, "training_s": time.perf_counter() - t0}
    # identity baseline of the loss: predicting u_i^t itself
    ident = float(np.mean(np.sum((Ut_all - Ys_all) ** 2, axis=1)))

    # 3) cold vs warm (both forms) on an unseen sketch seed
    res = {}
    for mode in ("cold", "plain", "residual"):
        s, U, V = solver(6, w["tol"], warm_hidden=0 if mode == "cold" else H)
        if mode != "cold":
            s.set_warm_start(nets[mode], H, residual=mode == "residual")
        s.iteration(0)
        torch.cuda.synchronize()
        U.copy_(U0d)
        V.copy_(V0d)
        base = s.stats()
        s.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(w["iters"]):
            s.iteration(t)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.set_timing(False)
        tm = s.timing()
        st = s.stats()
        rows = st["rows_updated"] - base["rows_updated"]
        res[mode] = {"iterations_per_s": w["iters"] / el, "ms_per_step": 1e3 * el / w["iters"],
                     "sweeps_per_row": (st["sweeps_total"] - base["sweeps_total"]) / rows,
                     "fallback_rate": (st["warm_fallbacks"] - base["warm_fallbacks"]) / rows,
                     "unconverged_rate": (st["rows_unconverged"] - base["rows_unconverged"]) / rows,
                     "nnls_rows_per_s": rows / (tm["nnls_ms"] / 1e3),
                     "phase_ms_per_step": {p: tm[p + "_ms"] / w["iters"] for p in ("sketch", "product", "small", "nnls")},
                     "rel_objective": s.objective()}
        print(f"[bench] {mode}: {res[mode]['iterations_per_s']:.2f} it/s, {res[mode]['sweeps_per_row']:.2f} sweeps/row, "
              f"fallback {res[mode]['fallback_rate']:.2f}", file=sys.stderr, flush=True)
        s.close()
    res["warm"] = res["plain"]
    # algorithmic work of a to-tolerance update: 2 k^2 flop per row-sweep and
    # 2 k^2 per row for its first gradient u Q - q (the block form carries
    # the gradient, so a stopping test is O(k)); mean over the two sides.
    # At k % 4 == 0, 64 < k <= 100 the sweeps run on the matrix cores.
    flops = 2.0 * k * k * (m + n) / 2 * (res["warm"]["sweeps_per_row"] + 1.0)
    nnls_avg = res["warm"]["phase_ms_per_step"]["nnls"] / 2 / 1e3
    ach = flops / nnls_avg / 1e12
    block = k % 4 == 0 and 64 < k <= 100
    kern = "prox_cd_grad_tol_kernel" if block else "prox_cd_tol_kernel"
    peak = PEAK["fp32_mfma_tflops"] if block else PEAK["fp32_valu_tflops"]
    return {
        "value": res["warm"]["iterations_per_s"], "ms_per_step": res["warm"]["ms_per_step"],
        "rel_objective": res["warm"]["rel_objective"],
        "nnls_rows_per_s": res["warm"]["nnls_rows_per_s"],
        "warm_start": {"cold": res["cold"], "warm_plain": res["plain"], "warm_residual": res["residual"],
                       "pairs": int(A_all.shape[0]), "pair_generation_s": t_pairs, "training": training,
                       "identity_loss": ident, "label_tol": w["label_tol"],
                       "sweeps_saved_per_row": {f: res["cold"]["sweeps_per_row"] - res[f]["sweeps_per_row"]
                                                for f in ("plain", "residual")},
                       "speedup_vs_cold": {f: res[f]["iterations_per_s"] / res["cold"]["iterations_per_s"]
                                           for f in ("plain", "residual")}},
        "roofline": {"kernel": f"prox-CD to tolerance ({kern}, all passes of one update)",
                     "bound": "mfma" if block else "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                     "frac": ach / peak, "traffic": None, "flops_per_launch": flops,
                     "avg_launch_ms": nnls_avg * 1e3},
    }


def _timed_run(solver, U, V, U0d, V0d, torch, iters, stop_at=None):
    """Reset U, V and run up to iters iterations, each timed on its own
    between device synchronisations; the objective after each one is outside
    the timed region.  With stop_at, stop at the first iteration whose
    objective is <= stop_at.  Returns (times_s, objectives)."""
    U.copy_(U0d)
    V.copy_(V0d)
    torch.cuda.synchronize()
    times, objs = [], []
    for t in range(iters):
        t0 = time.perf_counter()
        solver.iteration(t)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if stop_at is not None or t == iters - 1:
            objs.append(solver.objective())
            if stop_at is not None and objs[-1] <= stop_at:
                break
    return times, objs


def _per_update_error(M, U0, V0, Ug, sel, w, seed_sketch=0):
    """Relative Frobenius error of one GPU U update on the rows sel against
    the plain FP64 oracle (same U^0, V^0, same S^0), and against the oracle
    of the BF16 form (M and S rounded to bfloat16, products exact)."""
    from oracle import dsanls as O
    k, d = w["k"], w["d"]
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_GAUSSIAN, solver=O.SOLVER_PROX_CD, seed=seed_sketch,
                    alpha=w.get("alpha", 1.0), beta=w.get("beta", 1.0))
    U64, V64 = U0.astype(np.float64), V0.astype(np.float64)
    plain = O.update_U(M, U64, V64, 0, ocfg, rows=sel)
    ocfg.precision = "bf16"
    rounded = O.update_U(M, U64, V64, 0, ocfg, rows=sel)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return rel(Ug, plain), rel(Ug, rounded)


def run_to_eps(args, w, torch, B, K, W):
    """Plain FP32 and the BF16 form to a fixed relative objective (the
    metric), on several data seeds."""
    m, n, k, d = w["m"], w["n"], w["k"], w["d"]
    dev = torch.device("cuda", 0)
    seeds = w["seeds"] if args.seeds is None else tuple(range(args.seeds))
    per_seed, bf16_times, bf16_iters = [], [], 0
    errors, roof, prod_ms = None, None, {}
    for si, seed in enumerate(seeds):
        print(f"[bench] seed {seed}: generating data", file=sys.stderr, flush=True)
        M, U0, V0 = make_dense(w, seed)
        Md = torch.from_numpy(M).to(dev)
        U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
        res = {}
        for form in ("fp32", "bf16"):
            U, V = U0d.clone(), V0d.clone()
            cfg = B.make_config(m, n, k, d, d, sketch="gaussian", solver="prox_cd", precision=form, sweeps=1,
                                alpha=w.get("alpha", 1.0), beta=w.get("beta", 1.0), seed=0)
            solver = B.Solver(cfg, B.dense_matrix(Md), U, V, tensors=[Md])
            if si == 0 and not args.no_oracle_error:
                # one U update from U^0, V^0 against the FP64 oracle on sampled rows
                solver.update_U(0)
                torch.cuda.synchronize()
                g = np.random.default_rng(11)
                sel = np.unique(np.concatenate([g.choice(m, w["sample_rows"], replace=False), [0, m - 1]]))
                Ug = U.cpu().numpy().astype(np.float64)[sel]
                print(f"[bench] {form}: per-update error against the FP64 oracle", file=sys.stderr, flush=True)
                e_plain, e_rounded = _per_update_error(M, U0, V0, Ug, sel, w)
                errors = errors or {}
                errors[form] = {"vs_fp64_oracle": e_plain, "vs_fp64_oracle_of_bf16_inputs": e_rounded,
                                "rows": int(len(sel)), "update": "U at t=0 from U^0, V^0"}
            for t in range(W):
                solver.iteration(t)
            torch.cuda.synchronize()
            print(f"[bench] seed {seed} {form}: timing", file=sys.stderr, flush=True)
            solver.set_timing(True)
            if form == "fp32":
                times, objs = _timed_run(solver, U, V, U0d, V0d, torch, K)
                eps = objs[-1]
                res[form] = {"iterations": K, "time_s": sum(times), "rel_objective": eps}
            else:
                target = res["fp32"]["rel_objective"] * (1 + 1e-3)
                times, objs = _timed_run(solver, U, V, U0d, V0d, torch, w["max_factor"] * K, stop_at=target)
                reached = objs[-1] <= target
                res[form] = {"iterations": len(times), "time_s": sum(times), "rel_objective": objs[-1],
                             "reached": bool(reached)}
                bf16_times += times
                bf16_iters += len(times)
            solver.set_timing(False)
            tm = solver.timing()
            res[form]["iterations_per_s"] = res[form]["iterations"] / res[form]["time_s"]
            res[form]["phase_ms_per_step"] = {p: tm[p + "_ms"] / max(tm["launches"] / 2, 1)
                                              for p in ("sketch", "product", "small", "nnls")}
            prod_ms.setdefault(form, []).append(tm["product_ms"] / max(tm["launches"] / 2, 1))
            solver.close()
            del solver, U, V
        res["eps_star"] = res["fp32"]["rel_objective"]
        res["speedup_time_to_eps"] = res["fp32"]["time_s"] / res["bf16"]["time_s"]
        res["seed"] = seed
        per_seed.append(res)
        del Md, U0d, V0d
        torch.cuda.empty_cache()
        if si == 0:
            keepM = (M, U0, V0)
    med = lambda xs: float(np.median(xs))
    # roofline of the dominant kernel of the BF16 form: one grouped launch per
    # iteration computes A = M S and A' = M^T S' (the V side reuses A')
    flops = 2.0 * m * n * d + 2.0 * n * m * d
    avg_s = med(prod_ms["bf16"]) / 1e3
    ach = flops / avg_s / 1e12
    roof = {"kernel": "BF16 sketch GEMMs A = M S, A' = M^T S' (gemm_nt_bf16_dma_kernel, one launch per iteration)",
            "bound": "mfma", "achieved": ach, "peak": PEAK["bf16_mfma_tflops"], "unit": "TFLOP/s",
            "frac": ach / PEAK["bf16_mfma_tflops"], "traffic": traffic_bytes("dense-50000x20000-bf16"),
            "flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3}
    f_avg = med(prod_ms["fp32"]) / 1e3
    roof_fp32 = {"kernel": "FP32 sketch GEMMs (gemm_nt_f32_dma_kernel)", "bound": "mfma",
                 "achieved": flops / f_avg / 1e12, "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
                 "frac": flops / f_avg / 1e12 / PEAK["fp32_mfma_tflops"], "avg_launch_ms": f_avg * 1e3}
    value = bf16_iters / sum(bf16_times)
    out = {
        "value": value, "ms_per_step": 1e3 * sum(bf16_times) / bf16_iters,
        "rel_objective": med([r["bf16"]["rel_objective"] for r in per_seed]),
        "nnls_rows_per_s": (m + n) / (med([r["bf16"]["phase_ms_per_step"]["nnls"] for r in per_seed]) / 1e3),
        "to_eps": {
            "eps_star_median": med([r["eps_star"] for r in per_seed]),
            "definition": "eps* = plain-FP32 relative objective after K iterations, per data seed; "
                          "a form reaches it at rel <= eps* (1 + 1e-3)",
            "fp32": {"iterations_to_eps": med([r["fp32"]["iterations"] for r in per_seed]),
                     "time_to_eps_s": med([r["fp32"]["time_s"] for r in per_seed]),
                     "iterations_per_s": med([r["fp32"]["iterations_per_s"] for r in per_seed])},
            "bf16": {"iterations_to_eps": med([r["bf16"]["iterations"] for r in per_seed]),
                     "time_to_eps_s": med([r["bf16"]["time_s"] for r in per_seed]),
                     "iterations_per_s": med([r["bf16"]["iterations_per_s"] for r in per_seed]),
                     "all_reached": all(r["bf16"]["reached"] for r in per_seed)},
            "speedup_bf16_vs_fp32_time_to_eps": med([r["speedup_time_to_eps"] for r in per_seed]),
            "per_seed": per_seed},
        "error_vs_fp64_oracle": errors,
        "roofline": roof,
        "roofline_fp32_form": roof_fp32,
    }
    return out, keepM


def run_ksweep(args, w, torch, B, K, W):
    """Rank sweep on the text-shaped CSR workload (the synthetic analogue of
    the paper's k sweep): per k, iterations/s, NNLS rows/s, the relative
    objective after each iteration and its cumulative time."""
    m, n, d = w["m"], w["n"], w["d"]
    dev = torch.device("cuda", 0)
    print("[bench] generating data", file=sys.stderr, flush=True)
    M, Mt, _, _ = make_sparse(dict(w, k=1), args.seed)
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
    keep = [to(M.indptr, np.int64), to(M.indices, np.int32), to(M.data, np.float32),
            to(Mt.indptr, np.int64), to(Mt.indices, np.int32), to(Mt.data, np.float32)]
    mat = B.csr_matrix(*keep)
    from paper_2009_02845_amd import synth
    res = []
    for k in w["ks"]:
        U0, V0 = synth.init_factors(m, n, k, args.seed)
        U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
        U, V = U0d.clone(), V0d.clone()
        cfg = B.make_config(m, n, k, d, d, sketch="subsample", solver="prox_cd", sweeps=1, alpha=w.get("alpha", 1.0),
                            beta=w.get("beta", 1.0),
                            seed=0)
        solver = B.Solver(cfg, mat, U, V, tensors=keep)
        for t in range(W):
            solver.iteration(t)
        torch.cuda.synchronize()
        solver.set_timing(True)
        times, objs = [], []
        U.copy_(U0d)
        V.copy_(V0d)
        torch.cuda.synchronize()
        for t in range(K):
            t0 = time.perf_counter()
            solver.iteration(t)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            objs.append(solver.objective())
        solver.set_timing(False)
        tm = solver.timing()
        nnls_s = tm["nnls_ms"] / 1e3
        # the NNLS sweep: 12 k bytes and 2 k^2 flop per row
        nnls_avg = nnls_s / tm["launches"]
        flops = 2.0 * k * k * (m + n) / 2
        nbytes = 12.0 * k * (m + n) / 2
        block = k > 128 or (k % 4 == 0 and 64 < k <= 100)
        kern = "prox_cd_wide_kernel" if k > 128 else ("prox_cd_mfma_kernel" if block else "prox_cd_lds_kernel")
        peak_f = PEAK["fp32_mfma_tflops"] if block else PEAK["fp32_valu_tflops"]
        res.append({"k": k, "iterations_per_s": K / sum(times), "ms_per_step": 1e3 * sum(times) / K,
                    "nnls_rows_per_s": (m + n) * K / nnls_s,
                    "phase_ms_per_step": {p: tm[p + "_ms"] / K for p in ("sketch", "product", "small", "nnls")},
                    "rel_objective": objs, "cumulative_time_s": [float(x) for x in np.cumsum(times)],
                    "nnls_kernel": kern, "nnls_avg_launch_ms": nnls_avg * 1e3,
                    "nnls_tflops": flops / nnls_avg / 1e12, "nnls_frac_of_peak": flops / nnls_avg / 1e12 / peak_f,
                    "nnls_peak": "fp32 mfma" if block else "fp32 valu",
                    "nnls_gbs": nbytes / nnls_avg / 1e9})
        print(f"[bench] k={k}: {res[-1]['iterations_per_s']:.1f} it/s, objective {objs[-1]:.4f}", file=sys.stderr,
              flush=True)
        solver.close()
        del solver, U, V, U0d, V0d
    main_k = [r for r in res if r["k"] == 100] or res
    r0 = main_k[0]
    # the line's roofline: the NNLS sweep at the headline rank (HBM-bound at
    # k = 100, k / 6 flop per byte); every rank's figures are in k_sweep
    roof = {"kernel": f"prox-CD sweep ({r0['nnls_kernel']}, k = {r0['k']})", "bound": "hbm",
            "achieved": r0["nnls_gbs"], "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": r0["nnls_gbs"] / PEAK["hbm_gbs"], "traffic": None,
            "avg_launch_ms": r0["nnls_avg_launch_ms"]}
    return {"value": r0["iterations_per_s"], "ms_per_step": r0["ms_per_step"], "k_sweep": res, "roofline": roof}


def run_pgd_vs_cd(args, w, torch, B, W):
    """PGD and prox-CD on the same data, seeds and sketches: relative
    objective after every iteration (the synthetic analogue of the paper's
    solver comparison)."""
    dev = torch.device("cuda", 0)
    out = []
    for c in w["cases"]:
        m, n, k, d = c["m"], c["n"], c["k"], c["d"]
        M, U0, V0 = make_dense(dict(c, kind="dense"), args.seed)
        Md = torch.from_numpy(M).to(dev)
        U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
        entry = {"case": c["name"], "m": m, "n": n, "k": k, "d": d}
        for solver_name in ("pgd", "prox_cd"):
            U, V = U0d.clone(), V0d.clone()
            mu = dict(dict(alpha=c.get("alpha", 1.0), beta=c.get("beta", 1.0)), **c.get(solver_name, {}))
            cfg = B.make_config(m, n, k, d, d, sketch="gaussian", solver=solver_name, sweeps=1,
                                alpha=mu["alpha"], beta=mu["beta"],
                                seed=0)
            solver = B.Solver(cfg, B.dense_matrix(Md), U, V, tensors=[Md])
            for t in range(W):
                solver.iteration(t)
            times, objs = _timed_run(solver, U, V, U0d, V0d, torch, c["iters"], stop_at=-1.0)
            entry[solver_name] = {"rel_objective": objs, "cumulative_time_s": [float(x) for x in np.cumsum(times)],
                                  "iterations_per_s": len(times) / sum(times)}
            solver.close()
        print(f"[bench] {c['name']}: PGD {entry['pgd']['rel_objective'][-1]:.4f}, prox-CD "
              f"{entry['prox_cd']['rel_objective'][-1]:.4f}", file=sys.stderr, flush=True)
        out.append(entry)
    return out


def run_mu_grid(args, w, torch, B, W):
    """Relative objective after each workload's iterations for every
    (alpha, beta) of the paper's grid, one run per pair from U^0, V^0."""
    dev = torch.device("cuda", 0)
    out = []
    for name in w["cases"]:
        c = WORKLOADS[name]
        m, n, k, d = c["m"], c["n"], c["k"], c["d"]
        print(f"[bench] {name}: generating data", file=sys.stderr, flush=True)
        if c["kind"] == "dense":
            M, U0, V0 = make_dense(c, args.seed)
            Md = torch.from_numpy(M).to(dev)
            keep, mat, sketch = [Md], B.dense_matrix(Md), "gaussian"
        else:
            M, Mt, U0, V0 = make_sparse(c, args.seed)
            to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
            keep = [to(M.indptr, np.int64), to(M.indices, np.int32), to(M.data, np.float32),
                    to(Mt.indptr, np.int64), to(Mt.indices, np.int32), to(Mt.data, np.float32)]
            mat, sketch = B.csr_matrix(*keep), "subsample"
        U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
        table = []
        for a in w["grid"]:
            for b in w["grid"]:
                U, V = U0d.clone(), V0d.clone()
                cfg = B.make_config(m, n, k, d, d, sketch=sketch, solver="prox_cd", sweeps=1, alpha=a, beta=b, seed=0)
                solver = B.Solver(cfg, mat, U, V, tensors=keep)
                objs = []
                for t in range(c["iters"]):
                    solver.iteration(t)
                    objs.append(solver.objective())
                table.append({"alpha": a, "beta": b, "rel_objective": objs[-1], "trajectory": objs})
                solver.close()
        best = min(table, key=lambda r: r["rel_objective"])
        print(f"[bench] {name}: best alpha={best['alpha']} beta={best['beta']} -> {best['rel_objective']:.5f}",
              file=sys.stderr, flush=True)
        out.append({"workload": name, "iterations": c["iters"], "grid": table,
                    "best": {"alpha": best["alpha"], "beta": best["beta"], "rel_objective": best["rel_objective"]}})
        del keep, mat, U0d, V0d
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed iterations (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the per-update comparison with the FP64 oracle (profiler runs)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", type=int, default=None,
                    help="data seeds of the to-eps* workload (default: the workload's three)")
    ap.add_argument("--alpha", type=float, default=None,
                    help="override the workload's mu_t = alpha + beta t (Sec. 5.2; default: its frozen grid winner)")
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device-to-device three times (calibrates the HBM "
                         "traffic counters against a transfer of known size) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the method's multi-GPU form (an all-reduce of the k x d "
              f"sketch product per half-iteration) is not built; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2009_02845_amd import binding as B
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    B.load()
    w = dict(WORKLOADS[args.workload])
    for key in ("alpha", "beta"):
        if getattr(args, key) is not None:
            w[key] = getattr(args, key)
    K = args.steps if args.steps is not None else w["iters"]
    W = args.warmup
    if w["kind"] == "ksweep":
        r = run_ksweep(args, w, torch, B, K, W)
        out = {"metric": "sketched-ANLS iterations/s across ranks k (relative objective per iteration)",
               "unit": "iterations/s", "n_gpus": 1, "steps": K, "warmup": W, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": describe(args.workload, w, K), "m": w["m"], "n": w["n"], "d": w["d"],
                          "iterations": K, "parallelism": "single GPU"}}
        out.update(r)
        print(json.dumps(out), flush=True)
        return
    if w["kind"] == "mu_grid":
        r = run_mu_grid(args, w, torch, B, W)
        out = {"metric": "relative objective after each workload's iterations, per (alpha, beta) of mu_t",
               "unit": "relative error", "n_gpus": 1, "steps": None, "warmup": 0, "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": "mu_t = alpha + beta t grid over " + ", ".join(w["cases"]),
                          "parallelism": "single GPU"},
               "value": r[0]["best"]["rel_objective"], "cases": r}
        print(json.dumps(out), flush=True)
        return
    if w["kind"] == "pgd_vs_cd":
        r = run_pgd_vs_cd(args, w, torch, B, W)
        out = {"metric": "relative objective per iteration, PGD vs prox-CD", "unit": "relative error",
               "n_gpus": 1, "steps": None, "warmup": W, "higher_is_better": False, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": describe(args.workload, w), "parallelism": "single GPU"},
               "value": r[-1]["prox_cd"]["rel_objective"][-1], "cases": r}
        print(json.dumps(out), flush=True)
        return
    if w["kind"] == "to_eps":
        r, (M, U0, V0) = run_to_eps(args, w, torch, B, K, W)
        out = {"metric": "sketched-ANLS iterations/s (and NNLS rows/s) to a fixed relative objective, "
                         "BF16 form vs plain FP32",
               "unit": "iterations/s", "n_gpus": 1, "steps": K, "warmup": W,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16-sketch/f32",
               "data": "synthetic",
               "config": {"workload": describe(args.workload, w, K), "m": w["m"], "n": w["n"], "k": w["k"],
                          "d": w["d"], "iterations": K, "parallelism": "single GPU"}}
        out.update(r)
        if not args.no_cpu_baseline:
            print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
            out["cpu_baseline"] = cpu_baseline(w, M, U0, V0, half=True)
        print(json.dumps(out), flush=True)
        return
    if w["kind"] == "warm":
        r = run_warm(args, w, torch, B)
        out = {"metric": "sketched-ANLS iterations/s (and NNLS rows/s) to a fixed relative objective",
               "unit": "iterations/s", "n_gpus": 1, "steps": w["iters"], "warmup": 1,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic", "config": {"workload": describe(args.workload, w), "m": w["m"], "n": w["n"],
                                               "k": w["k"], "d": w["d"], "parallelism": "single GPU"}}
        out.update(r)
        print(json.dumps(out), flush=True)
        return
    print(f"[bench] workload {args.workload}: generating data", file=sys.stderr, flush=True)
    m, n, k, d = w["m"], w["n"], w["k"], w["d"]
    dev = torch.device("cuda", 0)
    Mt = None
    if w["kind"] == "dense":
        M, U0, V0 = make_dense(w, args.seed)
        Md = torch.from_numpy(M).to(dev)
        keep = [Md]
        mat = B.dense_matrix(Md)
        sketch = w.get("sketch", "gaussian")
    else:
        M, Mt, U0, V0 = make_sparse(w, args.seed)
        to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
        keep = [to(M.indptr, np.int64), to(M.indices, np.int32), to(M.data, np.float32),
                to(Mt.indptr, np.int64), to(Mt.indices, np.int32), to(Mt.data, np.float32)]
        mat = B.csr_matrix(*keep)
        sketch = w.get("sketch", "subsample")
    U0d, V0d = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
    U, V = U0d.clone(), V0d.clone()
    cfg = B.make_config(m, n, k, d, d, sketch=sketch, solver=w["solver"], precision=w["precision"],
                        sweeps=1, alpha=w.get("alpha", 1.0), beta=w.get("beta", 1.0), seed=0)
    solver = B.Solver(cfg, mat, U, V, tensors=keep)
    print(f"[bench] warmup {W} iterations", file=sys.stderr, flush=True)
    for t in range(W):
        solver.iteration(t)
    torch.cuda.synchronize()
    U.copy_(U0d)
    V.copy_(V0d)
    torch.cuda.synchronize()
    print(f"[bench] timing {K} iterations", file=sys.stderr, flush=True)
    solver.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(K):
        solver.iteration(t)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    solver.set_timing(False)
    tm = solver.timing()
    rel = solver.objective()
    its = K / el
    launches = 2 * K
    if w["kind"] == "dense" and w.get("sketch") in ("count", "srht"):
        # HBM-bound sketch products, one per half-iteration: the count sketch
        # reads X^T once and writes A^T, then transposes it (A read and
        # written); the SRHT reads X once and writes A
        prod_avg_s = tm["product_ms"] / 1e3 / launches
        per_side = []
        for rows, lng in ((m, n), (n, m)):
            extra = 3 if w["sketch"] == "count" else 1
            per_side.append(4.0 * rows * lng + extra * 4.0 * rows * d)
        nbytes = sum(per_side) / 2
        achieved = nbytes / prod_avg_s / 1e9
        name = ("cs_rows_kernel + transpose_kernel" if w["sketch"] == "count" else "srht_rows_kernel")
        roof = {"kernel": f"sketch product A = X S ({name}, one per half-iteration)", "bound": "hbm",
                "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": achieved / PEAK["hbm_gbs"],
                "traffic": None, "bytes_per_launch": nbytes, "avg_launch_ms": prod_avg_s * 1e3}
    elif w["kind"] == "dense":
        # one grouped launch per iteration computes A = M S (m x n x d) and
        # A' = M^T S' (n x m x d'); the V side reuses A'
        prod_avg_s = tm["product_ms"] / 1e3 / K
        flops_launch = 2.0 * m * n * d + 2.0 * n * m * d
        peak = PEAK["bf16_mfma_tflops"] if w["precision"] == "bf16" else PEAK["fp32_mfma_tflops"]
        achieved = flops_launch / prod_avg_s / 1e12
        if w["precision"] == "bf16":
            name = "gemm_nt_bf16_dma_kernel"
        else:   # the LDS-ring kernel needs both contraction lengths (n, m) to be multiples of 16
            name = "gemm_nt_f32_dma_kernel" if m % 16 == 0 and n % 16 == 0 else "gemm_nt_grouped_kernel"
        roof = {"kernel": f"sketch GEMMs A = M S, A' = M^T S' ({name}, one launch per iteration)",
                "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic_bytes(args.workload), "flops_per_launch": flops_launch,
                "avg_launch_ms": prod_avg_s * 1e3}
    else:
        roof = sparse_roofline(w, M, tm, launches, args.workload)
    out = {
        "metric": "sketched-ANLS iterations/s (and NNLS rows/s) to a fixed relative objective",
        "value": its,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-sketch/f32" if w["precision"] == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": describe(args.workload, w, K), "m": m, "n": n, "k": k, "d": d,
                   "iterations": K, "parallelism": "single GPU"},
        "rel_objective": rel,
        "nnls_rows_per_s": (m + n) * K / (tm["nnls_ms"] / 1e3) if tm["nnls_ms"] > 0 else None,
        "phase_ms_per_step": {p: tm[p + "_ms"] / K for p in ("sketch", "product", "small", "nnls")},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        if w["kind"] == "sparse":
            out["cpu_baseline"] = cpu_baseline(w, M, U0, V0, budget_s=1.0, max_iters=1, Mt=Mt)
        else:
            out["cpu_baseline"] = cpu_baseline(w, M, U0, V0)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
