#!/usr/bin/env python3
"""Benchmark of the RFP Cholesky hot path on one MI355X.

Workload (one "step"): for n = 20000 and n = 20001 and each of the eight RFP
layouts (TRANSR N/T x UPLO L/U), restore the pristine FP64 RFP array and the
right-hand sides, then PFTRF + PFTRS with nrhs = 128.  A = M M^T / n + I with
M n x n N(0,1) (seeded), B N(0,1).  The timed region holds exactly K steps
(restores included) between device synchronisations; value = nominal FP64
flops (PFTRF n^3/3 + PFTRS 2 n^2 nrhs) over the timed wall time.

The headline is timed with the library's kernel profiler off.  A second,
identical timed region with the profiler on gives the kernel table and the
roofline.

Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic FLOP/s over its event-timed
                launches inside the profiled timed region, against the FP64
                MFMA peak;
  cpu_baseline  the CPU oracle timed on a bounded sample on the host cores;
  pftri         PFTRI GFLOP/s (nominal 2 n^3 / 3) on the same matrices;
  accuracy      per layout: normwise backward error of the solve, forward
                error against a known solution (B = A X_true), and
                ||L L^T - A||_F / ||A||_F of the factor;
  conversions   TRTTF / TFTTR times and bandwidth (excluded from the factor
                times, as in the paper);
  cfg1          n = 1001, TRANSR=N, UPLO=L, nrhs = 4: PFTRF, PFTRS, PFTRI;
  mixed         n = 40000 (TRANSR=N, UPLO=L), nrhs = 16, A = M M^T / k + alpha I
                with M n x k (k = n/2) and alpha for cond ~1e3 and ~1e6: the
                FP64 PFTRF+PFTRS time against the low-precision factor with
                FP64 refinement (FP16, BF16 and FP32 factors tried; the fastest
                that reaches the FP64 path's backward error bound of 1e-14),
                each backward error measured with the dense FP64 A;
  batched_medium 512 systems, n log-uniform in [256, 4096], cond 1e2..1e8,
                PFTRI on every system, FP64 and FP16/BF16/FP32 factors with
                FP64 refinement, in one persistent launch each;
  batched       20000 systems, n uniform in [16, 256], random layout, nrhs
                uniform in [1, 8], A_i = M_i M_i^T / n_i + I: one persistent
                launch in FP64 and with FP32 factors + FP64 refinement, with
                and without PFTRI, against the single-system routines launched
                one system at a time (timed on the first 300 systems).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RFP PFTRF+PFTRS GFLOP/s: FP64 vs mixed-prec+IR at equal backward error"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_trf(n):
    return n ** 3 / 3.0


def flops_trs(n, nrhs):
    return 2.0 * n * n * nrhs


def flops_tri(n):
    return 2.0 * n ** 3 / 3.0


def src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel_name):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current GEMM source; else None."""
    path = os.path.join(ROOT, "profiles", "gemm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    cur = src_hash(os.path.join(ROOT, "paper_0901_1696_amd", "csrc", "gemm.hip"))
    if rec.get("gemm_source_sha256_16") != cur:
        return None
    return rec.get("kernels", {}).get(kernel_name, {}).get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n=12000, nrhs=128, full_sizes=(20000, 20001), layouts=8):
    """The oracle (definition-path PFTRF + PFTRS) on the host, bounded sample."""
    import numpy as np
    import oracle
    import synth
    import torch

    if torch.cuda.is_available():
        A, B = synth.spd_device(n, nrhs=nrhs, seed=n)
        A = A.cpu().numpy()
        B = np.asfortranarray(B.cpu().numpy())
    else:
        A, B = synth.spd(n, nrhs=nrhs, seed=n)
    arf = oracle.trttf("N", "L", A)
    t0 = time.perf_counter()
    f, info = oracle.pftrf("N", "L", n, arf)
    oracle.pftrs("N", "L", n, f, B)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate = (flops_trf(n) + flops_trs(n, nrhs)) / dt
    full = sum(layouts / len(full_sizes) * (flops_trf(m) + flops_trs(m, nrhs)) for m in full_sizes)
    return {"value": round(rate / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"oracle PFTRF+PFTRS (definition path, OpenMP rows) on one n={n} TRANSR=N UPLO=L "
                      f"matrix of the same recipe, nrhs={nrhs}; {dt:.1f} s",
            "full_step_estimate_s": round(full / rate, 1),
            "scaling": "the rate of the n=12000 sample applied to the benchmark step's nominal flops "
                       "(n=20000 and 20001, 8 layouts, nrhs=128); the oracle's cost grows as n^3"}


def roofline_of(prof):
    """Roofline object of the dominant kernel and the top of the kernel table,
    from the library's per-launch event timing.  Dominant = the kernel that
    carries the largest share of the section's algorithmic work: a one-
    workgroup, latency-bound kernel (the 128-row leaf) can have a large summed
    event time (it also counts its wait for a free slot on a busy GPU) while
    using a negligible share of the machine; it stays visible in the table."""
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["flops"])
    total_kernel_ms = sum(v["total_ms"] for v in prof.values())
    avg_ms = dom["total_ms"] / dom["launches"]
    flops_per_launch = dom["flops"] / dom["launches"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                "traffic": traffic_for(dom_name), "kernel": dom_name, "launches": dom["launches"],
                "avg_launch_ms": round(avg_ms, 5), "algorithmic_flops_per_launch": flops_per_launch,
                "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"],
                "share_of_kernel_time": round(dom["total_ms"] / total_kernel_ms, 4),
                "share_of_flops": round(dom["flops"] / sum(v["flops"] for v in prof.values()), 4)}
    kernels = sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])[:8]
    table = [{"kernel": k, "launches": v["launches"], "total_ms": round(v["total_ms"], 3),
              "tflops": round(v["flops"] / max(v["total_ms"], 1e-9) / 1e9, 2)} for k, v in kernels]
    return roofline, table


def backward_error_dense(A, B, X):
    """max over columns ||B - A X||_inf / (||A||_inf ||X||_inf + ||B||_inf), FP64 on the GPU."""
    R = B - A @ X
    anorm = A.abs().sum(dim=1).max()
    return (R.abs().amax(dim=0) / (anorm * X.abs().amax(dim=0) + B.abs().amax(dim=0))).max().item()


def bench_cfg1(h, reps=10):
    """n = 1001 (odd), TRANSR='N', UPLO='L', nrhs = 4, A = M M^T/n + I (seed
    1001): median times of PFTRF, PFTRS and PFTRI (input restored outside the
    timed events)."""
    import statistics
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    n, nrhs = 1001, 4
    dev = torch.device("cuda:0")
    A, B = synth.spd_device(n, nrhs=nrhs, seed=n, device=dev)
    pristine = torch.empty(rfp.nt(n), dtype=torch.float64, device=dev)
    rfp.rfp_dtrttf(h, "N", "L", n, A, pristine)
    w = torch.empty_like(pristine)
    x = B.clone()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    times = {"pftrf": [], "pftrs": [], "pftri": []}
    for r in range(reps + 1):
        w.copy_(pristine)
        x.copy_(B)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        rfp.rfp_dpftrf(h, "N", "L", n, w, info)
        ev[1].record()
        rfp.rfp_dpftrs(h, "N", "L", n, w, x)
        ev[2].record()
        rfp.rfp_dpftri(h, "N", "L", n, w, info)
        ev[3].record()
        ev[3].synchronize()
        if r:
            for k, (a, b) in zip(times, [(0, 1), (1, 2), (2, 3)]):
                times[k].append(ev[a].elapsed_time(ev[b]))
    if int(info.item()) != 0:
        raise SystemExit(f"cfg1: INFO={int(info.item())}")
    med = {k: statistics.median(v) for k, v in times.items()}
    fl = {"pftrf": flops_trf(n), "pftrs": flops_trs(n, nrhs), "pftri": flops_tri(n)}
    out = {"n": n, "layout": "NL", "nrhs": nrhs, "reps": reps}
    for k in med:
        out[k] = {"ms": round(med[k], 4), "gflops": round(fl[k] / (med[k] * 1e-3) / 1e9, 1)}
    out["pftrf+pftrs_gflops"] = round((fl["pftrf"] + fl["pftrs"]) / ((med["pftrf"] + med["pftrs"]) * 1e-3) / 1e9, 1)
    out["backward_error"] = backward_error_dense(A, B, x)
    log(f"[bench] cfg1 {out}")
    return out


def bench_complex(h, sizes=(20000, 20001), layouts=("NL", "NU", "CL", "CU"), nrhs=128):
    """Complex Hermitian path: ZPFTRF, ZPFTRS and ZPFTRI on A = M M^H/n + I
    (M with N(0,1) real and imaginary parts, seed n), each layout timed once
    with events (the input restored outside the timed events).  Flops count a
    complex multiply-add as 8 real flops: 4n^3/3, 8n^2 nrhs, 8n^3/3."""
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    dev = torch.device("cuda:0")
    tot = {"zpftrf": [0.0, 0.0], "zpftrs": [0.0, 0.0], "zpftri": [0.0, 0.0]}
    worst = 0.0
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    for n in sizes:
        A, B = synth.hpd_device(n, nrhs=nrhs, seed=n, device=dev)
        w = torch.empty(rfp.nt(n), dtype=torch.complex128, device=dev)
        for lay in layouts:
            t, u = lay[0], lay[1]
            rfp.rfp_ztrttf(h, t, u, n, A, w)
            x = B.clone()
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            rfp.rfp_zpftrf(h, t, u, n, w, info)
            ev[1].record()
            rfp.rfp_zpftrs(h, t, u, n, w, x)
            ev[2].record()
            rfp.rfp_zpftri(h, t, u, n, w, info)
            ev[3].record()
            ev[3].synchronize()
            if int(info.item()) != 0:
                raise SystemExit(f"complex {lay}{n}: INFO={int(info.item())}")
            fl = {"zpftrf": 4 * n ** 3 / 3, "zpftrs": 8.0 * n * n * nrhs, "zpftri": 8 * n ** 3 / 3}
            for k, (a, b) in zip(tot, [(0, 1), (1, 2), (2, 3)]):
                tot[k][0] += ev[a].elapsed_time(ev[b])
                tot[k][1] += fl[k]
            r = B - A @ x
            eta = (r.abs().amax(0) / (torch.linalg.matrix_norm(A, ord=float("inf")) * x.abs().amax(0)
                                      + B.abs().amax(0))).max().item()
            worst = max(worst, eta)
            del x, r
        del A, B, w
        torch.cuda.empty_cache()
    runs = len(sizes) * len(layouts)
    out = {"n": list(sizes), "layouts": list(layouts), "nrhs": nrhs,
           "flop_model": "complex multiply-add = 8 flops: ZPFTRF 4n^3/3, ZPFTRS 8n^2 nrhs, ZPFTRI 8n^3/3"}
    for k, (ms, fl) in tot.items():
        out[k] = {"gflops": round(fl / (ms * 1e-3) / 1e9, 1), "ms_per_call": round(ms / runs, 2)}
    out["max_backward_error"] = worst
    log(f"[bench] complex {out}")
    return out


def bench_pf_vs_po(h, sizes=(20000, 40000), nrhs=128, hbm_bytes=288e9):
    """The paper's central comparison (PF against PO, Section 8) on this GPU:
    FP64 PFTRF and PFTRS on the RFP array against the vendor's full-storage
    Cholesky and solve as torch calls them (ROCm's LAPACK-style potrf/potrs on
    the n x n array; PFTRI is timed alone), on the same matrix at equal n,
    each event-timed once after a warm-up; plus the storage each needs and
    the largest n whose matrix fits in the GPU's memory."""
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    dev = torch.device("cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    rows = []
    for n in sizes:
        A, B = synth.spd_device(n, nrhs=nrhs, seed=n, device=dev)
        w = torch.empty(rfp.nt(n), dtype=torch.float64, device=dev)
        pf, po = {}, {}

        def timed(fn):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1), out

        for rep in range(2):
            rfp.rfp_dtrttf(h, "N", "L", n, A, w)
            x = B.clone()
            pf["trf"], _ = timed(lambda: rfp.rfp_dpftrf(h, "N", "L", n, w, info))
            pf["trs"], _ = timed(lambda: rfp.rfp_dpftrs(h, "N", "L", n, w, x))
            pf["tri"], _ = timed(lambda: rfp.rfp_dpftri(h, "N", "L", n, w, info))
            del x
            po["trf"], L = timed(lambda: torch.linalg.cholesky(A))
            po["trs"], y = timed(lambda: torch.cholesky_solve(B, L))
            del L, y
            torch.cuda.empty_cache()
        if int(info.item()) != 0:
            raise SystemExit(f"pf_vs_po n={n}: INFO={int(info.item())}")
        fl = {"trf": flops_trf(n), "trs": flops_trs(n, nrhs), "tri": flops_tri(n)}
        row = {"n": n, "nrhs": nrhs, "layout": "NL"}
        for k in fl:
            row[f"pf_{k}_gflops"] = round(fl[k] / (pf[k] * 1e-3) / 1e9, 1)
            if k in po:
                row[f"po_{k}_gflops"] = round(fl[k] / (po[k] * 1e-3) / 1e9, 1)
                row[f"pf_over_po_{k}"] = round(po[k] / pf[k], 3)
        row["pf_bytes"] = 8 * rfp.nt(n)
        row["po_bytes"] = 8 * n * n
        rows.append(row)
        del A, B, w
        torch.cuda.empty_cache()
    nmax_pf = int(((1 + hbm_bytes) ** 0.5 - 1) / 2)  # 8 n (n + 1) / 2 = 4 n (n + 1) <= bytes
    nmax_po = int((hbm_bytes / 8) ** 0.5)
    out = {"runs": rows, "po": "torch.linalg.cholesky / cholesky_solve (FP64, n x n storage); the vendor inverse "
                                "through torch (cholesky_inverse) fails at these n, so PO inversion is not compared",
           "largest_n_fitting_288GB": {"pf": nmax_pf, "po": nmax_po}}
    log(f"[bench] pf_vs_po {out}")
    return out


def bench_mixed(h, n, nrhs=16, kappas=(1e3, 1e6), reps=2):
    """FP64 PFTRF+PFTRS vs low-precision factor + FP64 refinement at equal backward error."""
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    k = n // 2
    dev = torch.device("cuda:0")
    log(f"[bench] mixed: generating n={n}, k={k}")
    G, B = synth.spd_device(n, k=k, alpha=0.0, nrhs=nrhs, seed=n + 3, device=dev)  # M M^T / k
    arf = torch.empty(rfp.nt(n), dtype=torch.float64, device=dev)
    work = torch.empty_like(arf)
    x = torch.empty((nrhs, n), dtype=torch.float64, device=dev).t()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {"n": n, "nrhs": nrhs, "layout": "NL", "tol": 1e-14, "cases": []}
    diag = torch.arange(n, device=dev)
    alpha_prev = 0.0
    for kappa in kappas:
        alpha = synth.cond_alpha(n, k, kappa)
        G[diag, diag] += alpha - alpha_prev
        alpha_prev = alpha
        rfp.rfp_dtrttf(h, "N", "L", n, G, arf)
        torch.cuda.synchronize()

        def fp64():
            work.copy_(arf)
            x.copy_(B)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rfp.rfp_dpftrf(h, "N", "L", n, work, info)
            rfp.rfp_dpftrs(h, "N", "L", n, work, x)
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        fp64()
        t64 = min(fp64() for _ in range(reps))
        eta64 = backward_error_dense(G, B, x)
        case = {"kappa": kappa, "fp64_ms": round(t64 * 1e3, 2), "fp64_backward_error": eta64,
                "fp64_gflops": round((flops_trf(n) + flops_trs(n, nrhs)) / t64 / 1e9, 1)}
        best = None
        for prec, name in [(rfp.PREC_FP16, "fp16"), (rfp.PREC_BF16, "bf16"), (rfp.PREC_FP32, "fp32")]:
            codes = torch.zeros(2, dtype=torch.int32, device=dev)

            def mixed():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rfp.rfp_dpfsv_ir(h, prec, "N", "L", n, arf, B, x, codes[0:1], codes[1:2], tol=1e-14, max_iter=15)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                it, inf = (int(v) for v in codes.cpu())
                return dt, it, inf
            mixed()
            runs = [mixed() for _ in range(reps)]
            tm, it, inf = min(runs)
            eta = backward_error_dense(G, B, x)
            rec = {"factor": name, "ms": round(tm * 1e3, 2), "sweeps_or_fallback": it, "backward_error": eta}
            case.setdefault("tried", []).append(rec)
            log(f"[bench] mixed kappa={kappa:g} {name}: {tm*1e3:.1f} ms, code {it}, eta {eta:.2e}")
            if it > 0 and eta <= 1e-14 and (best is None or tm < best[0]):
                best = (tm, name, it, eta)
        if best is not None:
            case.update({"mixed_ms": round(best[0] * 1e3, 2), "mixed_factor": best[1], "sweeps": best[2],
                         "mixed_backward_error": best[3], "speedup_vs_fp64": round(t64 / best[0], 3),
                         "mixed_gflops_nominal": round((flops_trf(n) + flops_trs(n, nrhs)) / best[0] / 1e9, 1)})
        out["cases"].append(case)
        log(f"[bench] mixed kappa={kappa:g}: fp64 {t64*1e3:.1f} ms, best {best}")
    del G, B, arf, work, x
    torch.cuda.empty_cache()
    return out


def batch_fractions(fl, tm, ao, bo):
    """A batched run against both of its bounds: the FP64 MFMA peak, and HBM
    at its least traffic (every RFP array and right-hand side read once and
    written once, 8 bytes an entry)."""
    byt = 2 * 8 * (ao + bo)
    return {"frac_fp64_peak": round(fl / tm / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
            "hbm_min_bytes": byt, "hbm_gbs_at_min_bytes": round(byt / tm / 1e9, 1),
            "frac_hbm": round(byt / tm / 1e9 / HBM_PEAK_GBS, 4)}


def bench_batched(h, count=20000, seed=4, one_at_a_time=300, reps=3):
    """Persistent batched launch vs the single-system routines one system at a time."""
    import numpy as np
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    dev = torch.device("cuda:0")
    ns, lays, nrs = synth.batch_sizes(count, 16, 256, 1, 8, seed=seed)
    systems, ao, bo = [], 0, 0
    for n, li, nr in zip(ns, lays, nrs):
        n, nr = int(n), int(nr)
        t, u = rfp.LAYOUTS[int(li)]
        systems.append((n, ao, bo, n, nr, t, u))
        ao += rfp.nt(n)
        bo += n * nr
    log(f"[bench] batched: generating {count} systems ({ao * 8 / 1e9:.2f} GB RFP)")
    arf = torch.empty(ao, dtype=torch.float64, device=dev)
    b = torch.empty(bo, dtype=torch.float64, device=dev)
    g = synth.rng(seed + 1)
    for (n, a0, b0, ldb, nr, t, u) in systems:
        M = torch.from_numpy(g.standard_normal((n, n))).to(dev)
        A = (M @ M.t()) / n
        A.diagonal().add_(1.0)
        rfp.rfp_dtrttf(h, t, u, n, A.t(), arf[a0:a0 + rfp.nt(n)])
        b[b0:b0 + n * nr] = torch.from_numpy(g.standard_normal(n * nr)).to(dev)
    raw = rfp.sys_table(systems)
    table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    info = torch.zeros(count, dtype=torch.int32, device=dev)
    it = torch.zeros_like(info)
    fl_f = sum(flops_trf(s[0]) for s in systems)
    fl_s = sum(flops_trs(s[0], s[4]) for s in systems)
    fl_i = sum(flops_tri(s[0]) for s in systems)
    a1, b1 = arf.clone(), b.clone()
    out = {"systems": count, "n_range": [16, 256], "nrhs_range": [1, 8], "rfp_gb": round(ao * 8 / 1e9, 3),
           "nominal_gflop": {"pftrf": round(fl_f / 1e9, 2), "pftrs": round(fl_s / 1e9, 2),
                             "pftri": round(fl_i / 1e9, 2)}, "runs": []}
    for mode, name in [(rfp.PREC_FP64, "fp64"), (rfp.PREC_FP32, "fp32_factor+fp64_ir")]:
        for pftri in (False, True):
            def run():
                a1.copy_(arf)
                b1.copy_(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rfp.rfp_pfsv_vbatched(h, mode, count, table, a1, b1, info, it, sys_host=raw, do_pftri=pftri)
                torch.cuda.synchronize()
                return time.perf_counter() - t0
            run()
            tm = min(run() for _ in range(reps))
            fl = fl_f + fl_s + (fl_i if pftri else 0.0)
            bad = int((info != 0).sum().item())
            rec = {"mode": name, "pftri": pftri, "ms": round(tm * 1e3, 2), "gflops": round(fl / tm / 1e9, 1),
                   "info_nonzero": bad, "max_sweeps": int(it.max().item()), "min_code": int(it.min().item())}
            rec.update(batch_fractions(fl, tm, ao, bo))
            out["runs"].append(rec)
            log(f"[bench] batched {rec}")
    # the same work through the single-system routines, one system at a time
    a1.copy_(arf)
    b1.copy_(b)
    inf1 = torch.zeros(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (n, a0, b0, ldb, nr, t, u) in systems[:one_at_a_time]:
        av = a1[a0:a0 + rfp.nt(n)]
        bv = b1[b0:b0 + n * nr].view(nr, n).t()
        rfp.rfp_dpftrf(h, t, u, n, av, inf1)
        rfp.rfp_dpftrs(h, t, u, n, av, bv)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    proj = t1 * count / one_at_a_time
    fp64 = out["runs"][0]["ms"]
    out["one_at_a_time_fp64"] = {"systems_timed": one_at_a_time, "ms": round(t1 * 1e3, 2),
                                 "projected_ms_all": round(proj * 1e3, 1),
                                 "batched_speedup": round(proj * 1e3 / fp64, 1)}
    log(f"[bench] batched one-at-a-time {out['one_at_a_time_fp64']}")
    del arf, b, a1, b1
    torch.cuda.empty_cache()
    return out


def bench_batched_medium(h, count=512, seed=5, reps=2, one_at_a_time=24):
    """512 systems, n log-uniform in [256, 4096], A_i = M_i M_i^T / k_i +
    alpha_i I with k_i = ceil(n_i / 2) and alpha_i for cond 10^U(2, 8), random
    layout, nrhs uniform in [1, 8]; PFTRI on every system; one persistent
    launch per mode (FP64, and FP16 / BF16 / FP32 factors with FP64
    refinement and FP64 fall-back), against the single-system routines
    launched one system at a time (timed on the first systems)."""
    import math
    import numpy as np
    import torch
    import paper_0901_1696_amd as rfp
    import synth

    dev = torch.device("cuda:0")
    ns, lays, nrs = synth.batch_sizes(count, 256, 4096, 1, 8, seed=seed, log_uniform=True)
    g = synth.rng(seed + 1)
    kap = 10.0 ** g.uniform(2.0, 8.0, size=count)
    systems, ao, bo = [], 0, 0
    for n, li, nr in zip(ns, lays, nrs):
        n, nr = int(n), int(nr)
        t, u = rfp.LAYOUTS[int(li)]
        systems.append((n, ao, bo, n, nr, t, u))
        ao += rfp.nt(n)
        bo += n * nr
    log(f"[bench] batched medium: generating {count} systems ({ao * 8 / 1e9:.2f} GB RFP)")
    arf = torch.empty(ao, dtype=torch.float64, device=dev)
    b = torch.empty(bo, dtype=torch.float64, device=dev)
    for q, (n, a0, b0, ldb, nr, t, u) in enumerate(systems):
        k = int(math.ceil(n / 2))
        M = torch.from_numpy(g.standard_normal((n, k))).to(dev)
        A = (M @ M.t()) / k
        A.diagonal().add_(synth.cond_alpha(n, k, float(kap[q])))
        rfp.rfp_dtrttf(h, t, u, n, A.t(), arf[a0:a0 + rfp.nt(n)])
        b[b0:b0 + n * nr] = torch.from_numpy(g.standard_normal(n * nr)).to(dev)
        del M, A
    raw = rfp.sys_table(systems)
    table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    info = torch.zeros(count, dtype=torch.int32, device=dev)
    it = torch.zeros_like(info)
    fl_f = sum(flops_trf(s[0]) for s in systems)
    fl_s = sum(flops_trs(s[0], s[4]) for s in systems)
    fl_i = sum(flops_tri(s[0]) for s in systems)
    a1, b1 = arf.clone(), b.clone()
    out = {"systems": count, "n_range": [256, 4096], "n_max": int(max(ns)), "nrhs_range": [1, 8],
           "cond_range": [1e2, 1e8], "rfp_gb": round(ao * 8 / 1e9, 3),
           "nominal_gflop": {"pftrf": round(fl_f / 1e9, 1), "pftrs": round(fl_s / 1e9, 1),
                             "pftri": round(fl_i / 1e9, 1)}, "runs": []}
    for mode, name in [(rfp.PREC_FP64, "fp64"), (rfp.PREC_FP16, "fp16_factor+fp64_ir"),
                       (rfp.PREC_BF16, "bf16_factor+fp64_ir"), (rfp.PREC_FP32, "fp32_factor+fp64_ir")]:
        def run():
            a1.copy_(arf)
            b1.copy_(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rfp.rfp_pfsv_vbatched(h, mode, count, table, a1, b1, info, it, sys_host=raw, do_pftri=True,
                                  max_iter=30)
            torch.cuda.synchronize()
            return time.perf_counter() - t0
        run()
        tm = min(run() for _ in range(reps))
        fl = fl_f + fl_s + fl_i
        itc = it.cpu().numpy()
        rec = {"mode": name, "pftri": True, "ms": round(tm * 1e3, 2), "gflops": round(fl / tm / 1e9, 1),
               "info_nonzero": int((info != 0).sum().item()),
               "refined": int((itc > 0).sum()), "fallback": {str(c): int((itc == c).sum()) for c in (-1, -2, -3, -4)},
               "max_sweeps": int(itc.max())}
        rec.update(batch_fractions(fl, tm, ao, bo))
        # backward error of the solves of a sample of systems (dense FP64 check)
        worst = 0.0
        for (n, a0, b0, ldb, nr, t, u) in systems[:16]:
            A = torch.zeros((n, n), dtype=torch.float64, device=dev).t()
            rfp.rfp_dtfttr(h, t, u, n, arf[a0:a0 + rfp.nt(n)], A)
            A = A if u == "L" else A.t()
            A = torch.tril(A) + torch.tril(A, -1).t()
            B0 = b[b0:b0 + n * nr].view(nr, n).t()
            X = b1[b0:b0 + n * nr].view(nr, n).t()
            worst = max(worst, backward_error_dense(A, B0, X))
            del A
        rec["max_backward_error_16_systems"] = worst
        out["runs"].append(rec)
        log(f"[bench] batched medium {rec}")
    # the FP64 path through the single-system routines, one system at a time
    a1.copy_(arf)
    b1.copy_(b)
    inf1 = torch.zeros(1, dtype=torch.int32, device=dev)
    sub = systems[:one_at_a_time]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (n, a0, b0, ldb, nr, t, u) in sub:
        av = a1[a0:a0 + rfp.nt(n)]
        bv = b1[b0:b0 + n * nr].view(nr, n).t()
        rfp.rfp_dpftrf(h, t, u, n, av, inf1)
        rfp.rfp_dpftrs(h, t, u, n, av, bv)
        rfp.rfp_dpftri(h, t, u, n, av, inf1)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    fl_sub = sum(flops_trf(s[0]) + flops_trs(s[0], s[4]) + flops_tri(s[0]) for s in sub)
    proj = t1 * (fl_f + fl_s + fl_i) / fl_sub
    out["one_at_a_time_fp64"] = {"systems_timed": len(sub), "ms": round(t1 * 1e3, 2),
                                 "projected_ms_all_by_flops": round(proj * 1e3, 1),
                                 "batched_speedup": round(proj * 1e3 / out["runs"][0]["ms"], 2)}
    log(f"[bench] batched medium one-at-a-time {out['one_at_a_time_fp64']}")
    del arf, b, a1, b1
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sizes", default="20000,20001")
    ap.add_argument("--layouts", default="NL,NU,TL,TU")
    ap.add_argument("--nrhs", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pftri", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--mixed-n", type=int, default=40000)
    ap.add_argument("--no-kernel-profile", action="store_true",
                    help="skip the per-launch event timing (and the roofline); for counter collection runs")
    ap.add_argument("--no-complex", action="store_true")
    ap.add_argument("--no-pf-vs-po", action="store_true")
    ap.add_argument("--only", choices=["pftri", "pftrs", "mixed", "batched", "batched_medium", "cfg1", "complex",
                                       "pf_vs_po"],
                    help="run one section alone (for profiler runs) and print its JSON")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nel = args.calibrate_copy // 8
        src = torch.rand(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": nel * 8, "calibrate_copy_bytes_written": nel * 8,
                          "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0901_1696_amd as rfp
    import synth

    if args.only in ("mixed", "batched", "batched_medium", "cfg1", "complex", "pf_vs_po"):
        h = rfp.Handle(0)
        fn = {"mixed": lambda: bench_mixed(h, args.mixed_n), "batched": lambda: bench_batched(h),
              "batched_medium": lambda: bench_batched_medium(h), "cfg1": lambda: bench_cfg1(h),
              "complex": lambda: bench_complex(h), "pf_vs_po": lambda: bench_pf_vs_po(h)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        h.close()
        return

    sizes = [int(s) for s in args.sizes.split(",")]
    layouts = [(s[0], s[1]) for s in args.layouts.split(",")]
    nrhs = args.nrhs
    dev = torch.device("cuda:0")
    h = rfp.Handle(0)

    # ---- inputs (not timed): pristine RFP arrays per (n, layout), RHS per n
    log(f"[bench] generating inputs n={sizes} layouts={layouts} nrhs={nrhs}")
    pristine, rhs, dense = {}, {}, {}
    for n in sizes:
        A, B = synth.spd_device(n, nrhs=nrhs, seed=n, device=dev)
        for t, u in layouts:
            arf = torch.empty(rfp.nt(n), dtype=torch.float64, device=dev)
            rfp.rfp_dtrttf(h, t, u, n, A, arf)
            pristine[(n, t, u)] = arf
        rhs[n] = B
        dense[n] = A if not args.no_check else None
        torch.cuda.synchronize()
    nmax = max(sizes)
    work = torch.empty(rfp.nt(nmax), dtype=torch.float64, device=dev)
    bwork = torch.empty((nmax, nrhs), dtype=torch.float64, device=dev).t().contiguous().t()
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    combos = [(n, t, u) for n in sizes for t, u in layouts]

    def run_one(n, t, u):
        w = work[:rfp.nt(n)]
        w.copy_(pristine[(n, t, u)])
        b = bwork[:n]
        b.copy_(rhs[n])
        rfp.rfp_dpftrf(h, t, u, n, w, info)
        rfp.rfp_dpftrs(h, t, u, n, w, b)

    def step():
        for c in combos:
            run_one(*c)

    if args.only in ("pftri", "pftrs"):
        # one section alone: PFTRF, then PFTRI or PFTRS (nrhs), per layout
        tot_ms = 0.0
        s = torch.cuda.current_stream()
        for i in range(args.steps):
            for n, t, u in combos:
                w = work[:rfp.nt(n)]
                w.copy_(pristine[(n, t, u)])
                rfp.rfp_dpftrf(h, t, u, n, w, info)
                b = bwork[:n]
                b.copy_(rhs[n])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                if args.only == "pftri":
                    rfp.rfp_dpftri(h, t, u, n, w, info)
                else:
                    rfp.rfp_dpftrs(h, t, u, n, w, b)
                e1.record(s)
                e1.synchronize()
                tot_ms += e0.elapsed_time(e1)
            log(f"[bench] {args.only} step {i + 1}/{args.steps} done")
        fl = args.steps * sum(flops_tri(n) if args.only == "pftri" else flops_trs(n, nrhs) for n, _, _ in combos)
        print(json.dumps({args.only: {"gflops": round(fl / (tot_ms * 1e-3) / 1e9, 1),
                                      "ms_per_call": round(tot_ms / (args.steps * len(combos)), 3)}}), flush=True)
        h.close()
        return

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")

    # headline: K steps, kernel profiler off
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if int(info.item()) != 0:
        raise SystemExit(f"PFTRF reported INFO={int(info.item())}")
    elapsed = t1 - t0
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s")
    work_flops = sum(flops_trf(n) + flops_trs(n, nrhs) for n, _, _ in combos)
    value = args.steps * work_flops / elapsed / 1e9

    # roofline: up to 3 of the same steps again, every kernel launch
    # bracketed by HIP events on its own stream (the library creates its
    # event pool when profiling is enabled, large enough for this region, so
    # nothing is created or folded inside it)
    roofline, kernel_table, prof_region = None, [], None
    if not args.no_kernel_profile:
        psteps = min(args.steps, 3)
        rfp.rfp_profile_enable(h, True)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i in range(psteps):
            step()
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        prof = rfp.rfp_profile_read(h)
        rfp.rfp_profile_enable(h, False)
        prof_region = {"steps": psteps, "ms_per_step": round((p1 - p0) / psteps * 1e3, 3)}
        roofline, kernel_table = roofline_of(prof)
        log(f"[bench] profiled region {prof_region}")

    # ---- accuracy of every (n, layout) solve (independent check with torch)
    accuracy = None
    if not args.no_check:
        worst, per = {"backward_error": 0.0, "forward_error": 0.0, "factor_residual": 0.0}, {}
        g = torch.Generator(device=dev).manual_seed(7)
        for n, t, u in combos:
            A = dense[n]
            run_one(n, t, u)
            rec = {"backward_error": backward_error_dense(A, rhs[n], bwork[:n])}
            # forward error against a known solution: B = A X_true
            xt = torch.randn((n, 8), dtype=torch.float64, device=dev, generator=g)
            bt = (A @ xt).t().contiguous().t()
            w = work[:rfp.nt(n)]
            rfp.rfp_dpftrs(h, t, u, n, w, bt)
            rec["forward_error"] = ((bt - xt).abs().amax(0) / xt.abs().amax(0)).max().item()
            # ||L L^T - A||_F / ||A||_F of the factor in w
            L = torch.zeros((n, n), dtype=torch.float64, device=dev).t()
            rfp.rfp_dtfttr(h, t, "L" if u == "L" else "U", n, w, L)
            L = L if u == "L" else L.t()
            L = torch.tril(L)
            rec["factor_residual"] = (torch.linalg.matrix_norm(L @ L.t() - A) / torch.linalg.matrix_norm(A)).item()
            del L, xt, bt
            per[f"{t}{u}{n}"] = rec
            for k in worst:
                worst[k] = max(worst[k], rec[k])
        accuracy = {"max_" + k: v for k, v in worst.items()}
        accuracy.update({"layouts_checked": len(combos), "per_layout": per})
        log(f"[bench] accuracy {accuracy['max_backward_error']:.3e} {accuracy['max_forward_error']:.3e} "
            f"{accuracy['max_factor_residual']:.3e}")

    # ---- TRTTF / TFTTR (not part of the factor times, as in the paper)
    conversions = None
    if not args.no_check:
        rows = []
        for n, t, u in combos:
            A = dense[n]
            w = work[:rfp.nt(n)]
            full = torch.zeros((n, n), dtype=torch.float64, device=dev).t()
            for name, fn in (("trttf", lambda: rfp.rfp_dtrttf(h, t, u, n, A, w)),
                             ("tfttr", lambda: rfp.rfp_dtfttr(h, t, u, n, w, full))):
                fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    fn()
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / 3
                byts = 2.0 * 8 * rfp.nt(n)  # every stored entry read once and written once
                rows.append({"routine": name, "layout": f"{t}{u}{n}", "ms": round(ms, 4),
                             "GB/s": round(byts / ms / 1e6, 1), "hbm_frac": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)})
            del full
        conversions = {"bytes_model": "16 n(n+1)/2 (each stored entry read and written once)", "runs": rows}
        log(f"[bench] conversions {[(r['routine'], r['layout'], r['GB/s']) for r in rows]}")

    # ---- PFTRI (event timed, after its own PFTRF)
    pftri = None
    if not args.no_pftri:
        s = torch.cuda.current_stream()
        tot_ms, tot_fl = 0.0, 0.0
        for n, t, u in combos:
            w = work[:rfp.nt(n)]
            w.copy_(pristine[(n, t, u)])
            rfp.rfp_dpftrf(h, t, u, n, w, info)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            rfp.rfp_dpftri(h, t, u, n, w, info)
            e1.record(s)
            e1.synchronize()
            tot_ms += e0.elapsed_time(e1)
            tot_fl += flops_tri(n)
        if int(info.item()) != 0:
            raise SystemExit(f"PFTRI reported INFO={int(info.item())}")
        pftri = {"value": round(tot_fl / (tot_ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s",
                 "ms_per_call": round(tot_ms / len(combos), 3)}
        log(f"[bench] PFTRI {pftri}")

    del pristine, rhs, dense, work, bwork
    torch.cuda.empty_cache()
    cfg1 = bench_cfg1(h)
    mixed = None if args.no_mixed else bench_mixed(h, args.mixed_n)
    batched = None if args.no_batched else bench_batched(h)
    batched_medium = None if args.no_batched else bench_batched_medium(h)
    complex_ = None if args.no_complex else bench_complex(h)
    pf_vs_po = None if args.no_pf_vs_po else bench_pf_vs_po(h)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        cpu = cpu_baseline()

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 PFTRF+PFTRS, n in {" + ",".join(map(str, sizes)) + "} x RFP layouts "
                   + ",".join(t + u for t, u in layouts) + f", nrhs={nrhs}, A=M M^T/n+I (seeded N(0,1))",
                   "n": sizes, "layouts": [t + u for t, u in layouts], "nrhs": nrhs},
        "roofline": roofline, "profiled_region": prof_region, "cpu_baseline": cpu, "pftri": pftri,
        "accuracy": accuracy, "conversions": conversions, "cfg1": cfg1,
        "mixed": mixed, "batched": batched, "batched_medium": batched_medium, "complex": complex_,
        "pf_vs_po": pf_vs_po,
        "kernels": kernel_table,
        "paper_context": "PFTRF 90.7-93.0 GFLOP/s at n=20000 on a 16-core Intel Tigerton with MKL "
                         "(paper's zootfac_vendor table); another machine, not the target",
    }
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
