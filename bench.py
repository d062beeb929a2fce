"""Benchmark of the SAIT hot path on one MI355X.

Workload: 3D 7-point Poisson on a 128^3 grid (n = 2,097,152), ILU(0),
SAIT_Thr(tau = 1e-3, m = 3) factors M_L, M_U.  One timed step is one
preconditioner application z = M_U (M_L r) (Sec. 3.1) with the factors and
vectors already resident in HBM; `value` is the algorithmic bytes of that
apply divided by the measured time per step (GB/s), beside the fraction of
the 8 TB/s HBM peak.  The second half of the metric -- time to a 1e-10
true relative residual with FGMRES(40), FP32 / BF16 factors against the
FP64 form -- is measured after the timed loop and reported in
`time_to_residual` (also to 1e-8, the residual the metric's name quotes,
under `rtol_1e-8`).  `batched` reports the batched workload (256 anisotropic
2D systems x 8 right-hand sides, GMRES(30) to 1e-8, one persistent launch):
wall time, systems/s, pair-iterations/s and the modelled bytes per second
(batched_bytes).  `other_workloads`: FP64 apply GB/s on the random
diagonally dominant matrices and on the 2D convection-diffusion factors
(also after a cache-evicting write), and the forward / adjoint solve times
of the differentiable 512^2 workload.  `paper_experiment`: the paper's
PCG experiment (3D Laplace 100^3, level-0 and level-1 ILU, 1e-10) with the
SAIT preconditioners of its tables, 1..15 Jacobi sweeps, the exact
triangular solves and no preconditioner: iterations and seconds per solve.
`eigen_experiment`: the paper's LOBPCG experiment (the 4 smallest
eigenpairs of the same matrix, SAIT_Thr(0.01, 10) block preconditioning,
beside the exact solves and none): steps, seconds, error against the
closed-form spectrum.  `parilu_experiment`: the ILU factors built on the
device by fine-grained parallel ILU sweeps: build time and PCG iterations
against the host ILU(0).  `curves_experiment`: ratio, PCG iterations and
seconds against m for SAIT_Thr / SAIT_Pat and against tau at m = 10 (the
curves of Sec. 4.1-4.2).

Algorithmic bytes of one apply (s_v = value bytes, s_y = bytes of the
intermediate vector y = M_L r: 8 for FP64, 4 for the binary32 forms):
    sum over T in {L, U} of nnz(M_T) (s_v + 4) + 4 (n + 1)
    + n (8 [read r] + s_y [write y] + s_y [read y] + 8 [write z])
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SAIT-apply GB/s (% of HBM peak); time-to-1e-8 residual, mixed vs FP64"
VALUE_BYTES = {"f64": 8, "f32": 4, "bf16": 2}


def apply_bytes(n, nnz_L, nnz_U, prec, nrhs=1):
    sv = VALUE_BYTES[prec]
    sy = 8 if prec == "f64" else 4
    mat = (nnz_L + nnz_U) * (sv + 4) + 2 * 4 * (n + 1)
    vec = nrhs * n * (8 + 2 * sy + 8)
    return mat + vec


def launch_bytes(n, nnz, prec, first):
    """Algorithmic bytes of one SpMV launch of the apply."""
    sv = VALUE_BYTES[prec]
    sy = 8 if prec == "f64" else 4
    vec = n * (8 + sy)  # first: read r (8) + write y (s_y); second: read y + write z (8)
    return nnz * (sv + 4) + 4 * (n + 1) + vec


def kernel_name(shape):
    if shape in (-64, -65):
        return f"k_spmv_sell<{2 if shape == -64 else 1}, double> (sliced ELL)"
    if shape in (-8, -16):
        return f"k_spmv_stream<{2 if shape == -8 else 4}, double> (LDS-staged CSR)"
    return f"k_spmv<{shape}, double> (wavefront CSR)"


def measured_traffic(shape):
    """Per-launch HBM bytes of the FP64 apply SpMV from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the streaming-copy
    calibration recorded there), or None when the summary does not cover
    this kernel or the kernel source changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_spmv_sell_c3_128_traffic.txt")
    src = os.path.join(ROOT, "paper_2106_12836_amd", "csrc", "k_spmv.hip")
    if shape != -64 or not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    fields = {}
    for line in open(path):
        if line.startswith("f64:"):
            fields.update(kv.split("=") for kv in line[4:].split())
        elif line.startswith("k_spmv_sha256="):
            fields["sha"] = line.strip().split("=")[1]
    if fields.get("sha") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def copy_bandwidth(torch, dev, mib=1024, reps=20):
    """Rate of the library's plain streaming copy (read + write bytes)."""
    from paper_2106_12836_amd import sait_copy

    a = torch.empty(mib * 2**20 // 8, dtype=torch.float64, device=dev).uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        sait_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sait_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * mib * 2**20 / (ms * 1e-3) / 1e9


def cpu_baseline(A, tau, m, target_seconds=10.0):
    """The CPU oracle's FP64 apply on the host cores (bounded sample)."""
    import oracle

    t0 = time.time()
    L, U = oracle.ilu0(A)
    ML, MU = oracle.sait_factors(L, U, m, tau=tau)
    t_build = time.time() - t0
    r = np.random.default_rng(11).uniform(-1, 1, A.n)
    oracle.apply(ML, MU, r)  # warm
    reps, t = 0, 0.0
    t0 = time.time()
    while reps < 2 or (time.time() - t0 < target_seconds and reps < 5000):
        oracle.apply(ML, MU, r)
        reps += 1
    t = (time.time() - t0) / reps
    b = apply_bytes(A.n, ML.nnz, MU.nnz, "f64")
    return {
        "value": round(b / t / 1e9, 3),
        "unit": "GB/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{reps} FP64 applies z = M_U (M_L r) of the full 128^3 factors "
                  f"({ML.nnz + MU.nnz} stored entries), {reps * t:.1f} s; oracle build {t_build:.1f} s",
        "ms_per_apply": round(t * 1e3, 3),
    }


def batched_bytes(sys_ptr, rp_A, rp_ML, rp_MU, iters, k, RP):
    """Modelled HBM bytes of a batched solve (one persistent launch).

    The launch runs in global cycles of up to k Arnoldi steps; system s takes
    part in step j of cycle c while one of its pairs still has iterations
    left there: steps_s(c) = max_q min(k, max(0, I_sq - k c)).  Per system
    step (vec = rows_s * RP * 8 bytes, entries 12 bytes each):
        SpMM chain  (nnz_ML + nnz_MU + nnz_A) * 12 + 6 vec
        inner products over V_0..V_{j-1}, u, z   (j + 2) vec
        update (reads V_0..V_{j-1}, u, z, writes two vectors)  (j + 4) vec
    per cycle: the true residual nnz_A * 12 + 4 vec, after a full cycle
    the closing inner products (k + 1) vec, and the cycle end
    (steps + 1) vec + (nnz_ML + nnz_MU) * 12 + 7 vec.
    """
    total = 0.0
    for s in range(len(sys_ptr) - 1):
        r0, r1 = int(sys_ptr[s]), int(sys_ptr[s + 1])
        rows = r1 - r0
        vec = rows * RP * 8.0
        nA, nL, nU = (float(rp[r1] - rp[r0]) for rp in (rp_A, rp_ML, rp_MU))
        I = np.asarray(iters[s])
        ncyc = int(np.max((I + k - 1) // k)) if I.size else 0
        for c in range(ncyc + 1):
            total += nA * 12 + 4 * vec
            if c == ncyc:
                break
            steps = int(np.max(np.minimum(k, np.maximum(0, I - k * c))))
            j = np.arange(steps)
            total += steps * ((nL + nU + nA) * 12 + 6 * vec) + float(np.sum(2 * j + 6)) * vec
            if steps == k:
                total += (k + 1) * vec
            total += (steps + 1) * vec + (nL + nU) * 12 + 7 * vec
    return total


def batched_solve(torch, dev):
    """Full batched workload: 256 anisotropic 2D systems (sides U{32..512}),
    8 right-hand sides each, ILU(0) + SAIT_Thr(1e-2, 3), GMRES(30) to 1e-8,
    all pairs in one persistent launch."""
    from paper_2106_12836_amd import SaitPreconditioner
    from workloads import config

    t0 = time.time()
    c = config("c4")
    A, sp, Bh = c["A"], c["sys_ptr"], c["B"]
    nsys, R = len(sp) - 1, Bh.shape[1]
    t_gen = time.time() - t0
    t0 = time.time()
    pre = SaitPreconditioner(A, nsys=nsys, sys_ptr=sp, m=c["m"], tau=c["tau"])
    torch.cuda.synchronize()
    t_build = time.time() - t0
    Bt = torch.tensor(Bh, dtype=torch.float64, device=dev)
    pre.solve(Bt, restart=c["restart"], maxit=2, rtol=c["rtol"])  # allocates the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, infos = pre.solve(Bt, restart=c["restart"], rtol=c["rtol"])
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    its = np.array([i.iterations for i in infos]).reshape(nsys, R)
    bytes_model = batched_bytes(sp, A.rp, pre.row_ptr("ML"), pre.row_ptr("MU"), its, c["restart"],
                                1 if R == 1 else 2 if R == 2 else 4 if R <= 4 else 8)
    out = dict(
        workload=f"{nsys} anisotropic 2D systems (sides U{{32..512}}, n={A.n}), {R} RHS each, ILU(0) + "
                 f"SAIT_Thr(1e-2, 3), GMRES({c['restart']}) to {c['rtol']}, one persistent launch",
        seconds=round(ts, 4), build_s=round(t_build, 3), generate_s=round(t_gen, 2),
        systems_per_s=round(nsys / ts, 3), pair_iterations=int(its.sum()),
        pair_iterations_per_s=round(float(its.sum()) / ts, 1),
        iterations_min_mean_max=[int(its.min()), round(float(its.mean()), 1), int(its.max())],
        nonconverged=int(sum(i.status != 0 for i in infos)),
        max_true_relres=max(i.true_relres for i in infos),
        modelled_bytes=bytes_model, modelled_gbs=round(bytes_model / ts / 1e9, 1),
        pct_hbm_peak=round(100 * bytes_model / ts / 1e9 / HBM_PEAK_GBS, 1))
    pre.close()
    return out


def apply_rate(torch, dev, A, opts, cache_evict_mib=0, reps=50):
    """FP64 apply of one workload: GB/s from HIP events around each apply
    (inputs resident); with cache_evict_mib > 0 a write of that many MiB
    precedes every timed apply, so the factors come from HBM rather than the
    256 MB last-level cache."""
    from paper_2106_12836_amd import SaitPreconditioner, sait_time_apply
    from workloads import uniform_vector

    t0 = time.time()
    pre = SaitPreconditioner(A, **opts)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    pre.autotune()
    q = pre.query()
    r = torch.tensor(uniform_vector(A.n, 11), dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    B = apply_bytes(A.n, q["nnz_ML"], q["nnz_MU"], "f64")
    out = dict(n=A.n, nnz_A=A.nnz, nnz_ML=q["nnz_ML"], nnz_MU=q["nnz_MU"], bytes_apply=B, build_s=round(t_build, 3))
    _, _, ms = sait_time_apply(pre.handle, r, z, reps=reps)
    out["gbs_apply"] = round(B / (ms * 1e-3) / 1e9, 1)
    out["pct_hbm_peak"] = round(100 * out["gbs_apply"] / HBM_PEAK_GBS, 1)
    if cache_evict_mib:
        scratch = torch.empty(cache_evict_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for i in range(reps):
            scratch.fill_(float(i))
            e0.record()
            pre.apply(r, z)
            e1.record()
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        out["gbs_apply_after_cache_evict"] = round(B / (tot / reps * 1e-3) / 1e9, 1)
        out["cache_evict_mib"] = cache_evict_mib
        del scratch
    pre.close()
    return out


def extra_workloads(torch, dev):
    """Apply throughput on the random diagonally dominant matrices (banded and
    scattered columns) and on the 2D convection-diffusion factors, and the
    forward + adjoint solve time of the differentiable workload."""
    from paper_2106_12836_amd import SaitPreconditioner
    from paper_2106_12836_amd.autograd import sait_solve_autograd
    from workloads import config

    out = {}
    for name in ("rdd-b", "rdd-s"):
        c = config(name)
        out[name] = apply_rate(torch, dev, c["A"], dict(m=c["m"], tau=c["tau"]))
        out[name]["workload"] = (f"random diagonally dominant n=2^22, 8 off-diagonals "
                                 f"{'within +-2^14' if name == 'rdd-b' else 'anywhere'}, ILU(0) + SAIT_Thr(1e-2, 3)")
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    c = config("c2")
    out["c2"] = apply_rate(torch, dev, c["A"], dict(ilu_kind=1, ilut_tau=c["ilut_tau"], ilut_fill=c["ilut_fill"],
                                                   m=c["m"], tau=c["tau"]), cache_evict_mib=512)
    out["c2"]["workload"] = "2D upwind convection-diffusion 1024^2, Pe = 10, ILUT(1e-3, 10) + SAIT_Thr(1e-3, 4)"
    print(f"[bench] c2: {out['c2']}", file=sys.stderr, flush=True)
    # differentiable workload: forward FGMRES + adjoint FGMRES + gradient, 512^2
    c = config("c5")
    A, At_, b = c["A"], c["A_target"], c["b"]
    pre = SaitPreconditioner(A, m=c["m"], tau=c["tau"], build_transpose=1)
    xt = torch.zeros(A.n, dtype=torch.float64, device=dev)  # the loss's target only shapes the adjoint rhs
    times = []
    for _ in range(2):
        vals = torch.tensor(A.v, dtype=torch.float64, device=dev, requires_grad=True)
        bt = torch.tensor(b, dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = sait_solve_autograd(vals, bt, pre, restart=c["restart"], rtol=c["rtol"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ((x - xt) ** 2).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fi, ai = pre.last_forward_info, pre.last_adjoint_info
    out["c5"] = dict(workload=f"2D GRF diffusion 512^2 (n=262144), ILU(0) + SAIT_Thr(1e-2, 3), FGMRES(30) to "
                              f"{c['rtol']:g}; backward = adjoint FGMRES on A^T with transposed factors + gradient "
                              "on A's pattern",
                     forward_s=round(times[-1][0], 4), backward_s=round(times[-1][1], 4),
                     forward_iterations=fi.iterations, forward_status=fi.status,
                     forward_true_relres=fi.true_relres, adjoint_iterations=ai.iterations,
                     adjoint_status=ai.status, adjoint_true_relres=ai.true_relres)
    pre.close()
    print(f"[bench] c5: {out['c5']}", file=sys.stderr, flush=True)
    return out


def paper_experiment(torch, dev):
    """The paper's 3D experiment (Sec. 4) on one MI355X: 7-point Laplace on
    the 100^3 interior of a 102^3 mesh, level-0 and level-1 ILU, PCG to
    1e-10 with SAIT_Thr(0.05 / 0.02 / 0.01, 10), SAIT_Pat(1 / 2 / 3, 10),
    1..15 Jacobi sweeps per factor, the exact triangular solves and no
    preconditioner; f ~ U[0, 1) (seed 0).  Iterations and wall time per
    solve (build excluded, reported apart); the paper's printed iteration
    counts beside."""
    from paper_2106_12836_amd import SaitPreconditioner
    from workloads import poisson3d

    A = poisson3d(100)
    f = torch.tensor(np.random.default_rng(0).uniform(0.0, 1.0, A.n), dtype=torch.float64, device=dev)
    golden_all = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_table_pcg_iterations.json")))

    def timed_pcg(pre):
        pre.solve(f, rtol=1e-10, method="pcg")  # warm-up: allocates the PCG vectors
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, (info,) = pre.solve(f, rtol=1e-10, method="pcg")
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    out = dict(workload="3D 7-point Laplace 100^3 (n = 10^6), level-0 / level-1 ILU, PCG to 1e-10, "
                        "f ~ U[0,1) (seed 0)")
    for level in (0, 1):
        golden = golden_all[f"level{level}"]
        printed = {("thr", t): it for t, m, it in golden["sait_thr"]}
        printed.update({("pat", q): it for q, m, it in golden["sait_pat"]})
        printed_jac = dict(golden["jacobi"])
        ilu = {} if level == 0 else dict(ilu_kind="iluk", ilu_level=1)
        rec = dict(sait=[], jacobi=[], exact=None, none=None)
        for kind, param in (("thr", 0.05), ("thr", 0.02), ("thr", 0.01), ("pat", 1), ("pat", 2), ("pat", 3)):
            opts = dict(m=10, tau=param) if kind == "thr" else dict(m=10, pattern_p=param)
            t0 = time.time()
            pre = SaitPreconditioner(A, **opts, **ilu)
            torch.cuda.synchronize()
            tb = time.time() - t0
            q = pre.query()
            ts, info = timed_pcg(pre)
            rec["sait"].append(dict(preconditioner=f"SAIT_{'Thr' if kind == 'thr' else 'Pat'}({param}, 10)",
                                    ratio_L=round(q["ratio_L"], 4), ratio_U=round(q["ratio_U"], 4),
                                    iterations=info.iterations, seconds=round(ts, 4), build_s=round(tb, 3),
                                    status=info.status, true_relres=info.true_relres,
                                    paper_iterations=printed[(kind, param)]))
            if kind == "thr" and param == 0.05:
                for sw in range(1, 16):
                    pre.set_preconditioner("jacobi", sw)
                    ts, info = timed_pcg(pre)
                    rec["jacobi"].append(dict(sweeps=sw, iterations=info.iterations, seconds=round(ts, 4),
                                              status=info.status, paper_iterations=printed_jac[sw]))
                pre.set_preconditioner("exact")
                ts, info = timed_pcg(pre)
                rec["exact"] = dict(iterations=info.iterations, seconds=round(ts, 4), status=info.status)
                if level == 0:
                    pre.set_preconditioner("none")
                    ts, info = timed_pcg(pre)
                    out["none"] = dict(iterations=info.iterations, seconds=round(ts, 4), status=info.status)
            pre.close()
            print(f"[bench] paper experiment, level-{level} ILU: {rec['sait'][-1]}", file=sys.stderr, flush=True)
        out[f"level{level}"] = rec
    return out


def curves_experiment(torch, dev):
    """The curves of Sec. 4.1-4.2 on the paper's 100^3 Laplacian, for the
    level-0 and level-1 ILU factors: for SAIT_Thr(tau, m), tau = 0.01, 0.02,
    0.05, and SAIT_Pat(p, m), p = 1, 2, 3, with m = 1..10, the ratio
    nnz(M_L) / nnz(L), the PCG iterations to 1e-10 (f ~ U[0, 1), seed 0)
    and the seconds per solve; the nonzero ratio without dropping (tau = 0)
    for m = 1..10; and SAIT_Thr(tau, 10) over a wider range of tau (level 0)
    for the runtime optimum of Sec. 4.2."""
    from paper_2106_12836_amd import SaitPreconditioner
    from workloads import poisson3d

    A = poisson3d(100)
    f = torch.tensor(np.random.default_rng(0).uniform(0.0, 1.0, A.n), dtype=torch.float64, device=dev)

    def point(solve=True, **opts):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = SaitPreconditioner(A, **opts)
        torch.cuda.synchronize()
        rec = dict(ratio_L=round(pre.query()["ratio_L"], 4), build_s=round(time.perf_counter() - t0, 3))
        if solve:
            pre.solve(f, rtol=1e-10, method="pcg")  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, (info,) = pre.solve(f, rtol=1e-10, method="pcg", maxit=3000)
            torch.cuda.synchronize()
            rec.update(iterations=info.iterations, seconds=round(time.perf_counter() - t0, 4), status=info.status)
        pre.close()
        return rec

    out = dict(workload="3D 7-point Laplace 100^3, SAIT of the level-0 / level-1 ILU factors, PCG to 1e-10, "
                        "f ~ U[0,1) (seed 0)")
    for level in (0, 1):
        ilu = {} if level == 0 else dict(ilu_kind="iluk", ilu_level=1)
        for tau in (0.01, 0.02, 0.05):
            out[f"level{level}_thr_{tau}"] = [dict(m=m, **point(m=m, tau=tau, **ilu)) for m in range(1, 11)]
        for pp in (1, 2, 3):
            out[f"level{level}_pat_{pp}"] = [dict(m=m, **point(m=m, pattern_p=pp, **ilu)) for m in range(1, 11)]
        print(f"[bench] curves level {level} done", file=sys.stderr, flush=True)
    out["level0_thr_0_ratio"] = [dict(m=m, **point(solve=False, m=m, tau=0.0)) for m in range(1, 11)]
    out["level0_thr_m10"] = [dict(tau=t, **point(m=10, tau=t))
                             for t in (0.1, 0.05, 0.03, 0.02, 0.01, 0.005, 0.003, 0.002, 0.001, 0.0)]
    print("[bench] curves done", file=sys.stderr, flush=True)
    return out


def parilu_experiment(torch, dev):
    """ILU factors built on the device by synchronous fixed-point sweeps
    (fine-grained parallel ILU) instead of the row-wise host ILU(0), on the
    paper's 100^3 problem, for 1, 2, 3 and 5 sweeps on the ILU(0) pattern
    beside the host ILU(0): build time with m = 0 (the factorisation and the
    device copies, no Horner passes) and with SAIT_Thr(0.02, 10); GMRES(30)
    and PCG iterations to 1e-10 (f ~ U[0, 1), seed 0) with that SAIT
    preconditioner.  GMRES takes any preconditioner; PCG needs a symmetric
    one, which intermediate synchronous sweeps do not give (each sweep
    divides by the previous sweep's pivots); the symmetric (incomplete
    Cholesky) form, 1, 2 and 3 sweeps, does."""
    from paper_2106_12836_amd import SaitPreconditioner
    from workloads import poisson3d

    A = poisson3d(100)
    f = torch.tensor(np.random.default_rng(0).uniform(0.0, 1.0, A.n), dtype=torch.float64, device=dev)

    def build(**opts):
        SaitPreconditioner(A, **opts).close()  # warm-up (first-use allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pre = SaitPreconditioner(A, **opts)
        torch.cuda.synchronize()
        return pre, time.perf_counter() - t0

    def run(**ilu):
        pre0, t0 = build(m=0, tau=0.02, **ilu)
        pre0.close()
        pre, tb = build(m=10, tau=0.02, **ilu)
        x, (gi,) = pre.solve(f, rtol=1e-10, method="gmres", restart=30, maxit=5000)
        x, (pi,) = pre.solve(f, rtol=1e-10, method="pcg", maxit=5000)
        rec = dict(build_m0_s=round(t0, 4), build_s=round(tb, 4), ratio_L=round(pre.query()["ratio_L"], 4),
                   gmres_iterations=gi.iterations, gmres_status=gi.status, pcg_iterations=pi.iterations,
                   pcg_status=pi.status)
        pre.close()
        return rec

    out = dict(workload="3D 7-point Laplace 100^3, SAIT_Thr(0.02, 10), GMRES(30) / PCG to 1e-10, f ~ U[0,1) "
                        "(seed 0)", host_ilu0=run())
    for sw in (1, 2, 3, 5):
        out[f"parilu_{sw}"] = run(ilu_kind="parilu", ilu_level=0, parilu_sweeps=sw)
    for sw in (1, 2, 3):
        out[f"paric_{sw}"] = run(ilu_kind="paric", ilu_level=0, parilu_sweeps=sw)
    print(f"[bench] parilu: {out}", file=sys.stderr, flush=True)
    return out


def eigen_experiment(torch, dev, levels=(0, 1), comparators=True):
    """The paper's eigenvalue experiment (Sec. 4): the 4 smallest eigenpairs
    of the 7-point Laplacian on the 100^3 interior by LOBPCG, preconditioned
    by SAIT_Thr(0.01, 10) of the level-0 / level-1 ILU factors (the residual
    block through two sparse matrix-matrix products per step), beside the
    exact triangular solves and no preconditioner; tolerance 1e-8 relative
    per eigenpair; start block U[-1, 1] (seed 0).  Wall time per solve (the
    build reported apart), steps, and the error of the Ritz values against
    the closed-form spectrum."""
    from paper_2106_12836_amd import SaitPreconditioner
    from workloads import poisson3d

    s = 100
    A = poisson3d(s)
    t = np.sin(np.arange(1, 5) * np.pi / (2 * (s + 1))) ** 2
    exact = np.sort([4 * (t[i] + t[j] + t[l]) for i in range(4) for j in range(4) for l in range(4)])[:4]
    X0 = torch.tensor(np.random.default_rng(0).uniform(-1.0, 1.0, (A.n, 4)), device=dev)

    def timed(pre, maxit):
        pre.lobpcg(X0, tol=1e-8, maxit=2)  # warm-up: allocates the blocks
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, X, info = pre.lobpcg(X0, tol=1e-8, maxit=maxit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dict(iterations=info["iterations"], status=info["status"], p_drops=info["p_drops"],
                    relres=info["relres"], seconds=round(dt, 4),
                    ms_per_step=round(1e3 * dt / max(info["iterations"], 1), 4),
                    max_rel_err_vs_closed_form=float(np.max(np.abs(lam - exact) / exact)))

    out = dict(workload="3D 7-point Laplace 100^3 (n = 10^6), LOBPCG, 4 smallest eigenpairs, tol 1e-8, "
                        "X0 ~ U[-1,1] (seed 0)", eigenvalues_closed_form=[float(x) for x in exact])
    for level in levels:
        opts = dict(m=10, tau=0.01)
        if level:
            opts.update(ilu_kind="iluk", ilu_level=1)
        t0 = time.time()
        pre = SaitPreconditioner(A, **opts)
        torch.cuda.synchronize()
        rec = dict(build_s=round(time.time() - t0, 3), ratio_L=round(pre.query()["ratio_L"], 4))
        rec["sait"] = timed(pre, 3000)
        if comparators:
            pre.set_preconditioner("exact")
            rec["exact"] = timed(pre, 3000)
        if level == 0 and comparators:
            pre.set_preconditioner("none")
            out["none"] = timed(pre, 5000)
        pre.close()
        out[f"level{level}"] = rec
        print(f"[bench] eigen experiment, level-{level} ILU: {rec}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel shapes")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 256-system solve")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads (rdd, c2, c5)")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's PCG experiment (100^3)")
    ap.add_argument("--no-eigen", action="store_true", help="skip the paper's LOBPCG experiment (100^3)")
    ap.add_argument("--no-parilu", action="store_true", help="skip the device ILU (ParILU) experiment (100^3)")
    ap.add_argument("--no-curves", action="store_true", help="skip the ratio / iteration curves (100^3)")
    ap.add_argument("--parilu-only", action="store_true",
                    help="run only the device ILU (ParILU) experiment and print its record (for profiling)")
    ap.add_argument("--eigen-only", action="store_true",
                    help="run only the level-0 SAIT LOBPCG solve and print its record (for profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched solve and print its record (for profiling that launch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_12836_amd import SaitPreconditioner, sait_get_apply_lanes, sait_time_apply
    from workloads import config, poisson3d, spmv_rhs, uniform_vector

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batched_only:
        print(json.dumps({"batched": batched_solve(torch, dev)}), flush=True)
        return
    if args.parilu_only:
        print(json.dumps({"parilu_experiment": parilu_experiment(torch, dev)}), flush=True)
        return
    if args.eigen_only:
        print(json.dumps({"eigen_experiment": eigen_experiment(torch, dev, levels=(0,), comparators=False)}),
              flush=True)
        return
    s = args.grid
    A = poisson3d(s) if s != 128 else config("c3")["A"]
    n = A.n
    tau, m = 1e-3, 3
    print(f"[bench] workload 3D Poisson {s}^3 n={n} nnz(A)={A.nnz}", file=sys.stderr, flush=True)

    results = {}
    pres = {}
    for prec in ("f64", "f32", "bf16"):
        t0 = time.time()
        pre = SaitPreconditioner(A, m=m, tau=tau, precision=prec)
        torch.cuda.synchronize()
        t_build = time.time() - t0
        lanes = pre.autotune() if not args.no_autotune else sait_get_apply_lanes(pre.handle)
        q = pre.query()
        pres[prec] = pre
        results[prec] = dict(build_s=round(t_build, 3), lanes=lanes, nnz_ML=q["nnz_ML"], nnz_MU=q["nnz_MU"],
                             ratio_L=round(q["ratio_L"], 4), ratio_U=round(q["ratio_U"], 4))
        print(f"[bench] built {prec}: {results[prec]}", file=sys.stderr, flush=True)

    r = torch.tensor(uniform_vector(n, 11), dtype=torch.float64, device=dev)
    z = torch.empty_like(r)

    # --- timed region: FP64 applies -------------------------------------
    pre = pres["f64"]
    for _ in range(args.warmup):
        pre.apply(r, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pre.apply(r, z)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3
    q = pre.query()
    B = apply_bytes(n, q["nnz_ML"], q["nnz_MU"], "f64")
    value = B / (ms_step * 1e-3) / 1e9
    print(f"[bench] timed {args.steps} FP64 applies: {ms_step:.4f} ms/step, {value:.1f} GB/s",
          file=sys.stderr, flush=True)

    # --- per-launch kernel timing (HIP events on the launch stream) -------
    apply_stats = {}
    roof = None
    for prec, p in pres.items():
        ms_L, ms_U, ms_apply = sait_time_apply(p.handle, r, z, reps=max(20, args.steps // 2))
        qq = p.query()
        bL = launch_bytes(n, qq["nnz_ML"], prec, True)
        bU = launch_bytes(n, qq["nnz_MU"], prec, False)
        Bp = apply_bytes(n, qq["nnz_ML"], qq["nnz_MU"], prec)
        apply_stats[prec] = dict(ms_spmv_L=round(ms_L, 5), ms_spmv_U=round(ms_U, 5), ms_apply=round(ms_apply, 5),
                                 bytes_apply=Bp, gbs_apply=round(Bp / (ms_apply * 1e-3) / 1e9, 1),
                                 pct_hbm_peak=round(100 * Bp / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                                 **results[prec])
        if prec == "f64":
            per_launch_bytes = (bL + bU) / 2
            avg_launch_ms = (ms_L + ms_U) / 2
            achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(results["f64"]["lanes"][0]),
                    "kernel": kernel_name(results["f64"]["lanes"][0]) + " (SpMV of M_L and M_U)",
                    "bytes_per_launch": per_launch_bytes, "avg_launch_ms": round(avg_launch_ms, 5)}
    print(f"[bench] per-precision apply: {json.dumps(apply_stats)}", file=sys.stderr, flush=True)

    # --- time to residual: FGMRES(40) to 1e-10, FP64 vs FP32 vs BF16 factors ---
    ttr = None
    if not args.no_solve:
        xt = uniform_vector(n, 2)
        b = torch.tensor(spmv_rhs(A, xt), dtype=torch.float64, device=dev)
        ttr = {}
        for prec, p in pres.items():
            p.solve(b, restart=40, rtol=1e-10, flexible=True)  # warm-up (allocates the basis)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = p.solve(b, restart=40, rtol=1e-10, flexible=True)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            err = float(torch.linalg.norm(x - torch.tensor(xt, device=dev)) / np.linalg.norm(xt))
            ttr[prec] = dict(seconds=round(ts, 4), iterations=info[0].iterations,
                             true_relres=info[0].true_relres, rel_error_vs_x_true=err,
                             status=info[0].status)
            print(f"[bench] solve {prec}: {ttr[prec]}", file=sys.stderr, flush=True)
        base = ttr["f64"]["seconds"]
        for prec in ("f32", "bf16"):
            ttr[prec]["speedup_vs_f64"] = round(base / ttr[prec]["seconds"], 3)
        ttr["method"] = "FGMRES(40), FP64 basis/dots/Hessenberg/true residual, rtol 1e-10, x0 = 0, b = A x_true"
        # the same solves to 1e-8, the residual the metric's name quotes
        r8 = {}
        for prec, p in pres.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = p.solve(b, restart=40, rtol=1e-8, flexible=True)
            torch.cuda.synchronize()
            r8[prec] = dict(seconds=round(time.perf_counter() - t0, 4), iterations=info[0].iterations,
                            true_relres=info[0].true_relres, status=info[0].status)
        for prec in ("f32", "bf16"):
            r8[prec]["speedup_vs_f64"] = round(r8["f64"]["seconds"] / r8[prec]["seconds"], 3)
        ttr["rtol_1e-8"] = r8
        print(f"[bench] solves to 1e-8: {r8}", file=sys.stderr, flush=True)

    for p in pres.values():
        p.close()
    copy_gbs = copy_bandwidth(torch, dev)
    if roof is not None:
        roof["copy_kernel_gbs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)

    extra = None
    if not args.no_extra:
        extra = extra_workloads(torch, dev)

    paper = None
    if not args.no_paper:
        paper = paper_experiment(torch, dev)
    eigen = None
    if not args.no_eigen:
        eigen = eigen_experiment(torch, dev)
    parilu = None
    if not args.no_parilu:
        parilu = parilu_experiment(torch, dev)
    curves = None
    if not args.no_curves:
        curves = curves_experiment(torch, dev)

    batched = None
    if not args.no_batched:
        print("[bench] batched solve (256 systems x 8 RHS) ...", file=sys.stderr, flush=True)
        batched = batched_solve(torch, dev)
        print(f"[bench] batched: {json.dumps(batched)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(A, tau, m)
        print(f"[bench] cpu: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point Poisson {s}^3 (n={n}), ILU(0), SAIT_Thr(tau=1e-3, m=3), FP64 factors; "
                        "step = one apply z = M_U (M_L r)",
            "n": n, "nnz_A": A.nnz, "nnz_ML": q["nnz_ML"], "nnz_MU": q["nnz_MU"], "bytes_per_step": B,
        },
        "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "apply_by_precision": apply_stats,
        "time_to_residual": ttr,
        "batched": batched,
        "other_workloads": extra,
        "paper_experiment": paper,
        "eigen_experiment": eigen,
        "parilu_experiment": parilu,
        "curves_experiment": curves,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
