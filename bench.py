#!/usr/bin/env python3
"""Benchmark of the fused recomposition + per-row top-k on one MI355X.

Metric: precision-matrix rows/s of Psi = V diag(psi) V^T -> per-row top-k CSR on
the cell axis of the 1M cells x 20k genes workload (n = 1,000,000, r = 100,
k = 10), BF16-MFMA sweep with exact rescoring, against the FP32-MFMA sweep
(recall of the BF16 output against the FP32 output is reported).

A step is one pass of the whole recomposition path for all n rows: psi
folding, operand repacking, the MFMA sweep, exact rescoring, the exact
fallback for uncertified rows and the CSR emit.  At this size the library
takes the symmetric form of the sweep (tiles on or above the diagonal band,
a bound pass over a column sample, the column side grouped by row); the full
sweep is timed beside it on the same input and must give the same CSR.
Inputs (V, psi) are resident in HBM before timing starts.  Prints ONE JSON
line on stdout; progress goes to stderr.

The other steps of the path are timed once each at the same workload's shape
(reported under "stages", not part of the metric) on the 1M x 20k workload's
own data: log1p(NB counts) at 5% nonzeros with 40 Zipf-sized clusters and a
rank-8 cell factor, drawn on the GPU (synth.nb_log1p_csr_gpu).  Its gene-axis
Gram (the library's path and both paths forced), FP64 eigendecomposition, the
cell-axis factor (r = 100), the eigenvalue MLE on the resulting spectra, the
recomposition on that factor and psi, and the shared-cell path with 1M x 50k
binary peaks at 2% drawn from the same cell factor (transposes, subspace
iteration for cells and peaks with k = 110, q = 2, the three-axis solve).

--profile-run runs one step of the metric path and one 1 GiB device copy (the
reference kernel for scaling HBM traffic counters) and prints nothing else.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "top-k precision rows/s at 1M cells, BF16-MFMA vs FP32, recall ≥0.999"
WORKLOAD_TEXT = {
    "chain": "cell-axis recomposition + top-k of the 1M cells x 20k genes workload (n=1,000,000, r=100, "
             "k=10): the cell factor U = X V diag(e)^-1/2 and psi from the eigenvalue MLE, both computed by "
             "the path from log1p(NB counts) at 5% nonzeros with 40 Zipf-sized clusters (generated, seed 3000)",
    "proxy": "cell-axis recomposition + top-k at the 1M cells x 20k genes workload's shape (n=1,000,000, "
             "r=100, k=10) on a stand-in cell factor (orthonormal, 40 Zipf clusters) and psi = 1/E of a "
             "Marchenko-Pastur + spike spectrum",
}
PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}
# HBM traffic of the dominant sweep kernel at this workload comes from the committed
# rocprofv3 FETCH_SIZE / WRITE_SIZE summary, which records the SHA-256 of the
# sweep's sources it was taken on; when the sources differ the figure no longer
# describes the kernel and traffic is reported as null.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "recompose_bf16_1M_r100_k10_hbm_counters.md")
SWEEP_SOURCES = ["recompose_sweep.h", "sweep_bf16_c32.hip", "sweep_bf16_sym.hip", "mfma_util.h", "recompose.hip"]


def sweep_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_19892_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_sweep_traffic(prec, n, r, k, workload_name):
    """(bytes per launch, note) of the metric's dominant sweep kernel from the
    counter summary."""
    if (prec, n, r, k) != ("bf16", 1_000_000, 100, 10) or not os.path.exists(TRAFFIC_PROFILE):
        return None, "no counter profile for this configuration"
    vals = {}
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            if line.startswith("sweep_traffic_bytes_per_launch:"):
                vals["bytes"] = float(line.split(":", 1)[1])
            elif line.startswith("sweep_sources_sha256:"):
                vals["sha"] = line.split(":", 1)[1].strip()
            elif line.startswith("sweep_workload:"):
                vals["workload"] = line.split(":", 1)[1].strip()
    if vals.get("workload") != workload_name:
        return None, "the counters were taken on another input"
    if "bytes" not in vals or vals.get("sha") != sweep_sources_sha256():
        return None, "the sweep's sources changed since the counters were taken"
    return vals["bytes"], os.path.relpath(TRAFFIC_PROFILE, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(n, r, seed=3000):
    """Stand-ins for the cell factor of the 1M x 20k, 5%-dense, 40-cluster
    workload (synth.cell_factor_proxy: orthonormal columns spanning 40 Zipf
    cluster centroids, the rank-8 factor and per-cell noise) and its psi (1/E of
    a Marchenko-Pastur + spike spectrum of a 20k-gene Gram): a fixed input of
    the same shape, timed beside the path's own factor."""
    import numpy as np

    import synth
    V = synth.cell_factor_proxy(n, r, 40, seed=seed)
    E = synth.spectrum_proxy(20_000, n, 48, seed=seed)
    psi = np.ascontiguousarray(1.0 / E[:r])
    return V, psi


def chain_inputs(g, n, p, r, seed=3000, log_steps=True):
    """The 1M x 20k workload through the path up to the recomposition's inputs:
    log1p(NB counts) at 5% nonzeros with 40 Zipf-sized clusters and a rank-8
    cell factor drawn on the GPU, the gene Gram, its FP64 eigenpairs, the cell
    factor U (r columns) and psi from the eigenvalue MLE of the two spectra."""
    import torch

    import synth
    t0 = time.perf_counter()
    labels = synth.cluster_labels(n, 40, True, seed)
    beta0 = synth._calibrate_beta0(0.05, p, 40, labels, seed)
    A = synth.cell_factor_gpu(n, seed)
    rpd, cd, vd = synth.nb_log1p_csr_gpu(n, p, 40, True, seed, beta0=beta0, A=A)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    t = time.perf_counter()
    G = g.gram(rpd, cd, vd, n, p)
    w, Vt, rank = g.eigh_small(G)
    U = g.sketch(rpd, cd, vd, n, p, Vt, w, r)
    sol = g.solve_eigs([w[:r].contiguous(), w[:rank].contiguous()], [(0, 1)])
    torch.cuda.synchronize()
    nnz = int(rpd[-1])
    if log_steps:
        log(f"chain inputs: {nnz} nonzeros ({nnz / (n * p):.4f} dense) in {t_gen:.1f} s; Gram, eigh, "
            f"cell factor and solve in {time.perf_counter() - t:.1f} s ({sol.info['iterations']} iterations)")
    return {"csr": (rpd, cd, vd), "nnz": nnz, "A": A, "G": G, "w": w, "Vt": Vt, "rank": rank, "U": U,
            "psi": sol.lam[0].contiguous(), "labels": labels, "n": n, "p": p, "r": r}


def cpu_baseline(V, psi, k, n_clusters=40, seed=3000, per_cluster=8, edge=32):
    """The CPU oracle (unchanged) on a stratified sample of rows of the same
    workload: the first and last `edge` rows and `per_cluster` random rows of
    every cluster (384 rows, about 30 s of CPU work at this size)."""
    import numpy as np

    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    n = V.shape[0]
    labels = synth.cluster_labels(n, n_clusters, True, seed)
    rng = np.random.default_rng(7)
    picks = [np.arange(edge), np.arange(n - edge, n)]
    for c in range(n_clusters):
        members = np.flatnonzero(labels == c)
        picks.append(rng.choice(members, min(per_cluster, members.size), replace=False))
    rows = np.unique(np.concatenate(picks))
    t0 = time.perf_counter()
    for lo in range(0, rows.size, 16):
        blk = rows[lo:lo + 16]
        P = oracle.psi_rows(V, psi, blk)
        oracle.topk_csr(P, blk, k)
    dt = time.perf_counter() - t0
    return {"value": rows.size / dt, "unit": "rows/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{rows.size} rows of the n={n}, r={V.shape[1]}, k={k} workload: rows 0-{edge - 1}, "
                      f"the last {edge}, {per_cluster} random rows of each of the {n_clusters} clusters "
                      f"(FP64 row recomposition + exact top-k), {dt:.1f} s; all {n} rows would take "
                      f"{n / (rows.size / dt) / 3600:.1f} h (extrapolated)"}


def stages(g, inp, multimodal=True):
    """Gram, eigendecomposition, cell factor and solve of the chain inputs, each
    timed again on its own; then the Skeptic, the shared-cell path, the tensor
    solve and a full-rank gene axis."""
    import torch

    n, p, r = inp["n"], inp["p"], inp["r"]
    rpd, cd, vd = inp["csr"]
    nnz = inp["nnz"]
    A = inp["A"]
    out = {"input": f"{n} x {p} log1p(NB counts), 5% nonzeros, 40 Zipf-sized clusters, rank-8 cell "
                    f"factor (the NB/log1p recipe drawn on the GPU, seed 3000)", "r": r, "nnz": nnz}
    G = inp.pop("G")

    def timed(fn, reps):
        best = None
        for _ in range(reps):
            g.sync()
            g.kernel_times()
            g.set_timing(True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            g.set_timing(False)
            kms, cnt = g.kernel_times()
            if best is None or wall < best[0]:
                best = (wall, kms, cnt, res)
        return best

    g.gram(rpd, cd, vd, n, p, out=G)                      # warm-up
    wall, kms, cnt, _ = timed(lambda: g.gram(rpd, cd, vd, n, p, out=G), 1)
    row_nnz = torch.diff(rpd).to(torch.float64)
    algo = float(torch.sum(row_nnz * (row_nnz + 1.0)))   # 2 sum_c nnz_c (nnz_c + 1) / 2: the method's products
    del row_nnz
    out["gram"] = {"ms": wall * 1e3, "tile_kernel_ms": kms, "launches": cnt, "bound": "alu",
                   "unit": "TFLOP/s", "achieved": algo / wall / 1e12, "peak": PEAK_TFLOPS["fp32"],
                   "frac": algo / wall / 1e12 / PEAK_TFLOPS["fp32"],
                   "algorithmic_flops": algo,
                   "flops_kind": "2 sum_c nnz_c (nnz_c + 1) / 2: products of each cell's nonzeros (upper half)",
                   "path": "the library's choice from the shape"}
    # both paths forced, for the record of why the choice is made
    pp = (p + 255) // 256 * 256
    for path in ("dense", "sparse"):
        os.environ["GMGM_GRAM_PATH"] = path
        try:
            g.gram(rpd, cd, vd, n, p, out=G)
            w2, k2, c2, _ = timed(lambda: g.gram(rpd, cd, vd, n, p, out=G), 1)
        finally:
            del os.environ["GMGM_GRAM_PATH"]
        rec = {"ms": w2 * 1e3, "tile_kernel_ms": k2, "algorithmic_tflops": algo / w2 / 1e12}
        if path == "dense":
            dense = float(n) * pp * pp                    # 2 n pp^2 / 2: upper tiles incl. diagonal tiles
            rec.update(executed_flops=dense, executed_tflops=dense / (k2 * 1e-3) / 1e12,
                       executed_kind="dense-panel FP32 MFMA, n * p_pad^2 (upper tiles)")
        else:
            rec.update(executed_kind="FP64 products of each row's nonzeros into 128 x 128 LDS tiles")
        out["gram"][path] = rec
    log(f"stages: gram {wall * 1e3:.1f} ms ({out['gram']['achieved']:.2f} TF/s algorithmic); forced paths: "
        f"dense {out['gram']['dense']['ms']:.1f} ms, sparse {out['gram']['sparse']['ms']:.1f} ms")
    del inp["Vt"]
    torch.cuda.empty_cache()
    wall, kms, cnt, res = timed(lambda: g.eigh_small(G), 1)
    w, Vt, rank = res
    out["eigh"] = {"ms": wall * 1e3, "solver_ms": kms, "p": p, "rank": rank,
                   "note": "rocSOLVER divide and conquer on an FP64 copy"}
    log(f"stages: eigh {wall * 1e3:.1f} ms, rank {rank}")
    U = torch.empty(n, r, dtype=torch.float32, device="cuda")
    g.sketch(rpd, cd, vd, n, p, Vt, w, r, out=U)
    wall, kms, cnt, _ = timed(lambda: g.sketch(rpd, cd, vd, n, p, Vt, w, r, out=U), 3)
    byts = nnz * 8 + (n + 1) * 8 + p * r * (4 + 8) + n * r * 4
    out["sketch"] = {"ms": wall * 1e3, "kernel_ms": kms, "bound": "hbm", "unit": "GB/s",
                     "achieved": byts / (kms * 1e-3) / 1e9, "peak": 8000.0,
                     "frac": byts / (kms * 1e-3) / 1e9 / 8000.0, "algorithmic_bytes": byts}
    log(f"stages: sketch {wall * 1e3:.2f} ms ({out['sketch']['achieved']:.0f} GB/s)")
    Ec, Eg = w[:r].contiguous(), w[:rank].contiguous()
    g.solve_eigs([Ec, Eg], [(0, 1)])
    t = time.perf_counter()
    sol = g.solve_eigs([Ec, Eg], [(0, 1)])
    wall = time.perf_counter() - t
    out["solve"] = {"ms": wall * 1e3, "r_c": r, "r_g": rank, **{k: sol.info[k] for k in
                                                            ("iterations", "kkt", "n_pinned")}}
    log(f"stages: solve {wall * 1e3:.1f} ms, {sol.info['iterations']} iterations")
    # the Nonparanormal Skeptic of the same matrix kept sparse (S + 1 z^T), and
    # the Gram of the transform through the rank-two correction
    del Vt, U
    sk = g.skeptic(rpd, cd, vd, n, p)                     # warm-up (workspace)
    del sk
    torch.cuda.synchronize()
    t = time.perf_counter()
    sk = g.skeptic(rpd, cd, vd, n, p)
    torch.cuda.synchronize()
    sk_ms = (time.perf_counter() - t) * 1e3
    wall, kms, cnt, _ = timed(lambda: g.gram(rpd, cd, sk.val, n, p, out=G, shift=(sk.z, sk.csum)), 1)
    out["skeptic"] = {"ms": sk_ms, "nnz": nnz, "gram_shifted_ms": wall * 1e3,
                      "note": "per-gene ranks over all n cells (implicit zeros included) by a segmented "
                              "radix sort; the transform's Gram from S's Gram plus a rank-two FP64 correction"}
    log(f"stages: skeptic {sk_ms:.1f} ms, shifted gram {wall * 1e3:.1f} ms")
    del sk, G
    torch.cuda.empty_cache()
    if multimodal:
        out["shared_cells"] = shared_cells(g, n, p, rpd, cd, vd, nnz, Eg, r, A)
    del rpd, cd, vd, A
    inp.clear()
    torch.cuda.empty_cache()
    out["tensor_solve"] = tensor_solve(g)
    out["gene_axis_recompose"] = gene_axis_recompose(g)
    return out


def tensor_solve(g):
    """The eigenvalue solve at the shape of the paper's COIL-20 run: 20
    modalities (frame, row_i, col_i) of 72 frames x 128 x 128 sharing the frame
    axis (41 axes), with 10 and with all principal components per axis."""
    import numpy as np
    import torch

    import synth
    t0 = time.perf_counter()
    E, mods = library_spectra(g, synth.rotating_objects(20, 72, 128, 128, seed=1))
    out = {"input": "Gram spectra (library Gram + FP64 eigendecomposition of each unfolding) of 20 "
                    "synthetic rotating-object videos, 72 x 128 x 128, seed 1",
           "axes": len(E), "modalities": len(mods)}
    log(f"stages: tensor spectra in {time.perf_counter() - t0:.1f} s")
    for label, r in (("top10", 10), ("all", None)):
        Ed = [e[:r].contiguous() if r else e for e in E]
        g.solve_eigs_tensor(Ed, mods, max_iter=1000, raise_on_noconv=False)   # warm-up (workspace, handles)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sol = g.solve_eigs_tensor(Ed, mods, max_iter=1000, raise_on_noconv=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        out[label] = {"ms": wall * 1e3, "unknowns": int(sum(e.numel() for e in Ed)),
                      **{k: sol.info[k] for k in ("iterations", "kkt", "n_flat", "converged")}}
        log(f"stages: tensor solve ({label}) {wall * 1e3:.1f} ms, {sol.info['iterations']} iterations")
    return out


def library_spectra(g, tensors):
    """Per-axis Gram spectra of order-3 tensors (frames x h x w) sharing the frame
    axis, computed with the library: each unfolding as a dense CSR, gmgm_gram,
    gmgm_eigh_small, the numerically nonzero eigenvalues."""
    import numpy as np
    import torch

    def spectrum(A):                                     # Gram of A's columns: A^T A
        m, p = A.shape
        rp = torch.arange(m + 1, dtype=torch.int64, device="cuda") * p
        col = torch.arange(p, dtype=torch.int32, device="cuda").repeat(m)
        val = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float32)).cuda().view(-1)
        w, _, rank = g.eigh_small(g.gram(rp, col, val, m, p))
        return w[:rank].contiguous()

    frames = tensors[0].shape[0]
    E = [spectrum(np.concatenate([X.reshape(frames, -1).T for X in tensors], axis=0))]
    mods = []
    for i, X in enumerate(tensors):
        E.append(spectrum(np.moveaxis(X, 1, 0).reshape(X.shape[1], -1).T))
        E.append(spectrum(np.moveaxis(X, 2, 0).reshape(X.shape[2], -1).T))
        mods.append((0, 1 + 2 * i, 2 + 2 * i))
    return E, mods


def gene_axis_recompose(g, n=20_000, k=10, seed=3000):
    """Recomposition + top-k of a full-rank gene axis at the 1M x 20k workload's
    size (n = r = 20k, the contraction streamed): a Gaussian factor and psi = 1/E
    of a Marchenko-Pastur + spike spectrum (at this workload the solved gene
    eigenvalues all sit at their bound, which makes Psi_g a multiple of I)."""
    import numpy as np
    import torch

    import synth
    rng = np.random.default_rng(seed)
    V = torch.from_numpy((rng.standard_normal((n, n), dtype=np.float32) / np.float32(np.sqrt(n)))).cuda()
    psi = torch.from_numpy(1.0 / synth.spectrum_proxy(n, 1_000_000, 40, seed=seed)).cuda()
    res = {"input": f"{n} x {n} Gaussian factor, r = {n}, k = {k}"}
    for prec in ("fp32", "bf16"):
        g.recompose_topk(V, psi, k, prec=prec)
        g.sync()
        g.kernel_times()
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = g.recompose_topk(V, psi, k, prec=prec, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.set_timing(False)
        sweep_ms, cnt = g.kernel_times()
        flops = 2.0 * n * n * ((n + 31) // 32 * 32)
        res[prec] = {"ms": dt * 1e3, "sweep_ms": sweep_ms, "sweep_tflops": flops / (sweep_ms * 1e-3) / 1e12,
                     "sweep_frac_of_peak": flops / (sweep_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                     "stats": o.stats}
        log(f"stages: gene axis {prec}: {dt * 1e3:.1f} ms, sweep {sweep_ms:.1f} ms "
            f"({res[prec]['sweep_tflops']:.1f} TF/s), stats {o.stats}")
        del o
    del V, psi
    torch.cuda.empty_cache()
    return res


def shared_cells(g, n, p, rpd, cd, vd, nnz, Eg, r, A, p_pk=50_000, k_over=10, q=2):
    """Cells shared by RNA (the CSR above) and binary ATAC peaks (1M x 50k, 2%,
    Bernoulli(sigmoid) of the RNA's rank-8 cell factor A plus noise):
    subspace iteration for cells on [X_rna | X_pk] and for peaks on X_pk^T, then
    the three-axis solve."""
    import torch

    import synth
    t0 = time.perf_counter()
    prp, pcol = synth.peaks_csr_gpu(A, p_pk, 0.02, seed=4000)
    log(f"stages: peaks generated, {int(prp[-1])} nonzeros in {time.perf_counter() - t0:.1f} s")
    rna = g.CsrMatrix(rpd, cd, vd, n, p)
    pk = g.CsrMatrix(prp, pcol, None, n, p_pk)
    del prp, pcol
    torch.cuda.empty_cache()
    res = {"input": f"RNA {n} x {p} ({nnz} nonzeros) + binary peaks {n} x {p_pk} at 2% from the RNA's "
                    f"cell factor ({pk.nnz} nonzeros), seeds 3000 / 4000", "k": r + k_over, "q": q}
    torch.cuda.synchronize()
    t = time.perf_counter()
    rna_t, pk_t = rna.transpose(), pk.transpose()
    torch.cuda.synchronize()
    res["transpose_ms"] = (time.perf_counter() - t) * 1e3
    gen = torch.Generator(device="cuda").manual_seed(4001)
    k = r + k_over
    om_c = torch.randn(p + p_pk, k, dtype=torch.float64, device="cuda", generator=gen)
    om_p = torch.randn(n, k, dtype=torch.float64, device="cuda", generator=gen)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Ec, Vc = g.subspace_eig([rna, pk], om_c, q, r, blocks_t=[rna_t, pk_t])
    torch.cuda.synchronize()
    res["cells_subspace_ms"] = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    Ep, Vp = g.subspace_eig([pk_t], om_p, q, r, blocks_t=[pk])
    torch.cuda.synchronize()
    res["peaks_subspace_ms"] = (time.perf_counter() - t) * 1e3
    # sparse work of one subspace run: (2q + 2) products over all nonzeros, k FP64 FMAs each
    res["cells_sparse_flops"] = float(2 * (2 * q + 2) * (nnz + pk.nnz) * k)
    t = time.perf_counter()
    sol = g.solve_eigs([Ec, Eg, Ep], [(0, 1), (0, 2)])
    res["solve_ms"] = (time.perf_counter() - t) * 1e3
    res["solve"] = {kk: sol.info[kk] for kk in ("iterations", "kkt", "n_pinned")}
    log(f"stages: shared cells: transposes {res['transpose_ms']:.0f} ms, cells {res['cells_subspace_ms']:.0f} ms, "
        f"peaks {res['peaks_subspace_ms']:.0f} ms, solve {res['solve_ms']:.0f} ms")
    del rna_t, pk_t, pk, om_c, om_p, Vc, Vp
    torch.cuda.empty_cache()
    return res


def threshold_leg(g, Vd, pd, topk_out, k, prec, n, r, steps=5, warmup=2):
    """The fixed-threshold form of the same recomposition (Theorem 3's
    significance rule uses it): rows/s at the threshold that keeps about k
    entries per row, taken as the median over rows of the k-th largest |Psi|
    from the top-k output."""
    import torch
    kth = topk_out[2].view(n, k).abs().min(dim=1).values
    thr = float(kth.median().item())
    res = g.recompose_threshold(Vd, pd, thr, prec=prec)      # sizes the output
    cap = res.nnz
    for _ in range(warmup):
        res = g.recompose_threshold(Vd, pd, thr, prec=prec, capacity=cap)
    g.sync()
    g.kernel_times()
    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = g.recompose_threshold(Vd, pd, thr, prec=prec, capacity=cap)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    g.set_timing(False)
    sweep_ms, cnt = g.kernel_times()
    sweep_ms /= steps            # both sweeps of a call (all rows, then the rows with many candidates)
    flops = 2.0 * r * n * n
    log(f"threshold {thr:.4g}: {dt * 1e3:.2f} ms/step, sweep {sweep_ms:.2f} ms, nnz {res.nnz}")
    return {"thr": thr, "rule": "median over rows of the k-th largest |Psi| (half the rows keep at least k)",
            "rows_per_s": n / dt, "ms_per_step": dt * 1e3, "sweep_ms": sweep_ms,
            "sweep_tflops": flops / (sweep_ms * 1e-3) / 1e12,
            "sweep_frac_of_peak": flops / (sweep_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec], "nnz": res.nnz,
            "sweep_launches_per_call": cnt / steps}


def library_gemm_tflops(dtype_name="bf16", n=16384, iters=10):
    """Context for the roofline: the rate the vendor GEMM (torch.matmul ->
    hipBLASLt) reaches on a large square product of the same dtype on this GPU,
    i.e. the practically attainable share of the published MFMA peak."""
    import torch
    dt = {"bf16": torch.bfloat16, "fp32": torch.float32}[dtype_name]
    a = torch.randn(n, n, device="cuda", dtype=dt)
    b = torch.randn(n, n, device="cuda", dtype=dt)
    for _ in range(3):
        c = a @ b
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(iters):
        c = a @ b
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / iters
    del a, b, c
    torch.cuda.empty_cache()
    return 2.0 * n ** 3 / (ms * 1e-3) / 1e12


def profile_run(g, Vd, pd, k, prec, n):
    """One metric step and one 1 GiB device copy (counter calibration)."""
    import torch
    out = (torch.empty(n + 1, dtype=torch.int64, device="cuda"), torch.empty(n * k, dtype=torch.int32, device="cuda"),
           torch.empty(n * k, dtype=torch.float32, device="cuda"))
    g.recompose_topk(Vd, pd, k, prec=prec, out=out)
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log("profile run done")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--r", type=int, default=100)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp8", "fp32"])
    ap.add_argument("--compare", default="fp32", help="precisions timed beside the metric")
    ap.add_argument("--compare-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gemm-reference", action="store_true", help="skip timing the library BF16 GEMM")
    ap.add_argument("--no-threshold", action="store_true", help="skip the fixed-threshold recomposition")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage timings")
    ap.add_argument("--no-multimodal", action="store_true", help="skip the shared-cell-axis stage")
    ap.add_argument("--profile-run", action="store_true", help="one step + a 1 GiB copy, no JSON")
    ap.add_argument("--workload", default="chain", choices=["chain", "proxy"],
                    help="chain: the cell factor and psi the path computes from the generated 1M x 20k "
                         "counts; proxy: the stand-in factor and spectrum")
    ap.add_argument("--no-standin", action="store_true", help="skip timing the stand-in factor beside the chain")
    ap.add_argument("--sources-sha", action="store_true", help="print the SHA-256 of the sweep's sources")
    ap.add_argument("--tensor-solve-only", action="store_true",
                    help="only the tensor-variate eigenvalue solve at the COIL-20 shape (its own JSON line)")
    args = ap.parse_args()

    if args.sources_sha:
        print(sweep_sources_sha256())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the path is measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2407_19892_amd as g

    if args.tensor_solve_only:
        g.load()
        print(json.dumps({"tensor_solve": tensor_solve(g)}), flush=True)
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    g.load()
    n, r, k = args.n, args.r, args.k
    inp = None
    if args.workload == "chain":
        log(f"building the path's inputs n={n} p=20000 r={r}")
        inp = chain_inputs(g, n, 20_000, r)
        Vd, pd = inp["U"], inp["psi"]
    else:
        log(f"generating the stand-in workload n={n} r={r}")
        V, psi = workload(n, r)
        Vd = torch.from_numpy(V).cuda()
        pd = torch.from_numpy(psi).cuda()
    if args.profile_run:
        profile_run(g, Vd, pd, k, args.prec, n)
        return

    def alloc():
        return (torch.empty(n + 1, dtype=torch.int64, device="cuda"),
                torch.empty(n * k, dtype=torch.int32, device="cuda"),
                torch.empty(n * k, dtype=torch.float32, device="cuda"))

    def run(prec, steps, warmup, out, form=None):
        # form: "full" or "symmetric" forces the library's choice (None: its size rule)
        if form is None:
            os.environ.pop("GMGM_RECOMPOSE_PATH", None)
        else:
            os.environ["GMGM_RECOMPOSE_PATH"] = form
        for _ in range(warmup):
            g.recompose_topk(Vd, pd, k, prec=prec, out=out, check=False)
        g.sync()
        g.kernel_times()
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.recompose_topk(Vd, pd, k, prec=prec, out=out, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.set_timing(False)
        sweep_ms, cnt = g.kernel_times()
        g.sync()
        st = g.recompose_topk(Vd, pd, k, prec=prec, out=out, stats=True).stats
        os.environ.pop("GMGM_RECOMPOSE_PATH", None)
        return dt / steps, sweep_ms / max(cnt, 1), st

    out_main = alloc()
    log(f"timing {args.prec}: warmup {args.warmup}, steps {args.steps}")
    step_s, sweep_ms, st_main = run(args.prec, args.steps, args.warmup, out_main)
    log(f"{args.prec}: {step_s * 1e3:.2f} ms/step, sweep {sweep_ms:.2f} ms, stats {st_main}")

    flops = 2.0 * r * n * n
    # the dominant kernel's algorithmic work: every pair (i, j) for the full
    # sweep, each pair once (r n^2) for the symmetric form
    kflops = r * float(n) * n if st_main["symmetric"] else flops
    traffic, traffic_note = profiled_sweep_traffic(args.prec, n, r, k, args.workload)
    result = {
        "metric": METRIC, "value": n / step_s, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "n": n, "r": r, "k": k, "prec": args.prec, "global_batch": n, "seq_len": None,
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "mfma",
                     "kernel": "sweep_kernel (symmetric form)" if st_main["symmetric"] else "sweep_kernel",
                     "achieved": kflops / (sweep_ms * 1e-3) / 1e12, "peak": PEAK_TFLOPS[args.prec],
                     "unit": "TFLOP/s", "frac": kflops / (sweep_ms * 1e-3) / 1e12 / PEAK_TFLOPS[args.prec],
                     "traffic": traffic, "traffic_unit": "bytes", "traffic_source": traffic_note,
                     "sweep_ms": sweep_ms,
                     "algorithmic_flops_per_launch": kflops,
                     "executed_mfma_flops_per_step": st_main["mfma_flops"]},
        "stats": st_main,
    }
    ref = out_main
    if st_main["symmetric"]:
        # the full sweep on the same input, for comparison (same output required)
        out = alloc()
        log(f"timing {args.prec} full sweep: {args.compare_steps + 1} steps")
        s, sw, st = run(args.prec, args.compare_steps + 1, 1, out, form="full")
        same = bool(torch.equal(out[1], ref[1]) and torch.equal(out[2], ref[2]))
        result["full_sweep"] = {"rows_per_s": n / s, "ms_per_step": s * 1e3, "sweep_ms": sw,
                                "sweep_tflops": flops / (sw * 1e-3) / 1e12,
                                "sweep_frac_of_peak": flops / (sw * 1e-3) / 1e12 / PEAK_TFLOPS[args.prec],
                                "stats": st, "same_csr_as_symmetric": same}
        log(f"{args.prec} full sweep: {s * 1e3:.2f} ms/step, sweep {sw:.2f} ms, same CSR {same}")
        del out
    for prec in [p for p in args.compare.split(",") if p in PEAK_TFLOPS and p != args.prec]:
        out = alloc()
        log(f"timing {prec}: {args.compare_steps} steps")
        s, sw, st = run(prec, args.compare_steps, 1, out)
        same = (out[1].view(n, k).unsqueeze(2) == ref[1].view(n, k).unsqueeze(1)).any(2).sum().item()
        result[prec] = {"rows_per_s": n / s, "ms_per_step": s * 1e3, "sweep_ms": sw,
                        "sweep_tflops": flops / (sw * 1e-3) / 1e12,
                        "sweep_frac_of_peak": flops / (sw * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                        "stats": st, f"recall_of_{args.prec}_vs_{prec}": same / (n * k)}
        log(f"{prec}: {s * 1e3:.2f} ms/step, sweep {sw:.2f} ms, recall {same / (n * k):.6f}")
        del out
    if not args.no_threshold:
        result["threshold"] = threshold_leg(g, Vd, pd, out_main, k, args.prec, n, r)
    if args.prec == "bf16" and not args.no_gemm_reference:
        lib = library_gemm_tflops("bf16")
        result["roofline"]["library_gemm_tflops"] = lib
        result["roofline"]["frac_of_library_gemm"] = result["roofline"]["achieved"] / lib
        log(f"library BF16 GEMM 16384^3: {lib:.1f} TFLOP/s")
    if "fp32" in result:
        result["recall_vs_fp32"] = result["fp32"][f"recall_of_{args.prec}_vs_fp32"]
        result["speedup_vs_fp32"] = result["fp32"]["ms_per_step"] / result["ms_per_step"]
    if args.workload == "chain" and not args.no_standin:
        # the stand-in factor used before the full chain was run here, for continuity
        V0, psi0 = workload(n, r)
        V0d, p0d = torch.from_numpy(V0).cuda(), torch.from_numpy(psi0).cuda()
        del V0, psi0
        Vd_m, pd_m = Vd, pd
        Vd, pd = V0d, p0d
        s0, sw0, st0 = run(args.prec, 3, 1, out_main)
        Vd, pd = Vd_m, pd_m
        result["stand_in_workload"] = {"input": WORKLOAD_TEXT["proxy"], "rows_per_s": n / s0,
                                       "ms_per_step": s0 * 1e3, "sweep_ms": sw0, "stats": st0}
        log(f"stand-in factor: {s0 * 1e3:.2f} ms/step, sweep {sw0:.2f} ms, stats {st0}")
        del V0d, p0d
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on sampled rows)")
        result["cpu_baseline"] = cpu_baseline(Vd.cpu().numpy(), pd.cpu().numpy(), k)
    if not args.no_stages:
        del out_main, ref
        torch.cuda.empty_cache()
        if inp is None:
            inp = chain_inputs(g, n, 20_000, r)
        del Vd, pd
        result["stages"] = stages(g, inp, multimodal=not args.no_multimodal)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
