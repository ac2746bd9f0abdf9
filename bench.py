#!/usr/bin/env python3
"""GSE-TDVP1 time-step benchmark on one MI355X.

One "step" is a full GSE-TDVP1 time step through the C-ABI: global Krylov
vectors by MPO application + basis extension (tdvp_expand_basis), the
one-site TDVP sweep (tdvp_sweep) and the measurement of energy, norm and
<S^z_i> (tdvp_measure).  Inputs are seeded synthetic workloads resident on
the device before the timed region starts.

Default workload (--workload 3): the chi_max = 1024 J1-J2 cylinder 4 x 16
with U(1) S^z charges, real-time quench from Neel (see cylinder_mode): the
state is grown to chi_max untimed, then each precision runs W warmup and K
timed steps from it, BF16-input/FP32-accumulate contractions against FP64
(and FP32).  --workload 1: the rung-decoupled Heisenberg ladder, leg length
32 (64 sites, zigzag path), imaginary time from a seeded random MPS of bond
dimension 16, dtau = 0.5, Krylov order k = 3, chi_max = 256, FP64; W warmup
steps are evolved first (the bond dimension grows), then K steps are timed.

Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "TDVP sweep time/step & H_eff matvec TFLOP/s, mixed vs FP64, at fixed fidelity"
# dense matrix-core peaks of the arithmetic each precision runs on
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}
# matrix-core flops issued per algorithmic flop (8 per complex multiply-add):
# the FP64 and FP32 GEMMs form a complex product from three real products
# (6 flops), the BF16 kernel from four, the BF16X3 split from twelve
MFMA_PER_FLOP = {"fp64": 0.75, "fp32": 0.75, "bf16": 1, "bf16x3": 3}


COPY_PROBE_BYTES = 64 * 1024 * 1024
CSRC_KERNELS = os.path.join(ROOT, "paper_2005_06104_amd", "csrc", "kernels.hip")
CSRC_BLOCKS = os.path.join(ROOT, "paper_2005_06104_amd", "csrc", "blocks.cpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, seconds: float, chi_probe: int):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    GSE-TDVP1 steps from the same seeded initial state until `seconds` have
    elapsed, plus one one-site H_eff application at bond dimension chi_probe."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gse, mpo, tdvp as OT
    from paper_2005_06104_amd import inputs as I

    N = w.lattice.n_sites
    Ws = mpo.build_mpo(N, w.terms)
    Wop = mpo.build_mpo(N, w.terms, 1.0, -1j * w.tau)
    psi = w.initial_mps()
    t0 = time.perf_counter()
    n = 0
    bonds = 1
    last = 0.0
    # whole steps only; another step is started only when it should end within
    # the budget (steps grow with the bond dimension: taken as twice the last)
    while n < w.n_steps and (n == 0 or time.perf_counter() - t0 + 2.0 * last <= seconds):
        ts = time.perf_counter()
        psi, _ = gse.gse_step(psi, Ws, Wop, w.dt, w.k, w.eps_K, w.eps_M, w.eps, w.chi_max, 1e-12, 30, w.normalize)
        last = time.perf_counter() - ts
        n += 1
        bonds = max(t.shape[2] for t in psi)
    el = time.perf_counter() - t0
    # one H_eff application at the full bond dimension (synthetic tensors)
    wmax = max(W.shape[1] for W in Ws)
    L = I.random_hermitian_env(chi_probe, wmax, 1)
    R = I.random_hermitian_env(chi_probe, wmax, 2)
    C = I.random_complex((chi_probe, 2, chi_probe), 3)
    Wm = I.random_mpo_site(wmax, wmax, 4)
    t1 = time.perf_counter()
    OT.heff_apply(L, Wm, R, C)
    mv_ms = (time.perf_counter() - t1) * 1e3
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": n / el if el > 0 else None, "unit": "GSE-TDVP1 steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"first {n} steps of the same workload from the same seed (bond dims up to {bonds}), "
                      f"{el:.1f} s; one-site H_eff application at chi={chi_probe}, w={wmax}: {mv_ms:.0f} ms",
            "matvec_ms": mv_ms, "steps_timed": n, "max_bond_reached": int(bonds)}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def traffic_from_profile(name: str, sources):
    """HBM bytes per H_eff GEMM launch from the committed counter summary
    profiles/<name>, or None when the sources it names (the GEMM kernel, and
    for charged states the block-sparse maps) changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    rec = dict(line.split(":", 1) for line in txt.splitlines()
               if line.startswith(("kernels_sha256:", "sources_sha256:", "bytes_per_launch:")))
    got = rec.get("sources_sha256", rec.get("kernels_sha256", "")).strip()
    if got != sources_sha256(sources):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_workload(T, ctx, w, prec, warmup, steps, label, mark=False):
    """Evolve the workload from its seeded initial state; time `steps` steps
    after `warmup` (mark: marker kernels right before and after the timed
    steps, for cutting a kernel trace)."""
    import torch
    N = w.lattice.n_sites
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    psi = T.tdvp_mps_from_host(ctx, w.initial_mps())
    torch.cuda.synchronize()

    def step():
        e = T.tdvp_expand_basis(ctx, [psi], [op], w.k, w.eps_K, w.eps_M, w.chi_max, prec)[0]
        s = T.tdvp_sweep(ctx, [psi], [H], w.dt, w.eps, w.chi_max, 1e-12, 30, prec, w.normalize)[0]
        m = T.tdvp_measure(ctx, [psi], [H])[0]
        return e, s, m

    for i in range(warmup):
        t = time.perf_counter()
        e, s, m = step()
        log(f"[{label}] warmup {i}: {1e3 * (time.perf_counter() - t):.1f} ms, max bond {max(m['bond_dims'])}, "
            f"E={m['energy']:.10f}, matvecs {s['n_matvec']}")
    torch.cuda.synchronize()
    if mark:
        torch.cuda._sleep(1000)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = {"ms_heff_gemm": 0.0, "flops_heff_gemm": 0.0, "n_heff_gemm": 0, "ms_matvec": 0.0, "flops_matvec": 0.0,
           "n_matvec": 0, "ms_sweep": 0.0, "ms_krylov": 0.0, "ms_extend": 0.0}
    for i in range(steps):
        ts = time.perf_counter()
        e, s, m = step()
        for k in ("ms_heff_gemm", "flops_heff_gemm", "n_heff_gemm", "ms_matvec", "flops_matvec", "n_matvec"):
            acc[k] += s[k]
        acc["ms_sweep"] += s["ms"]
        acc["ms_krylov"] += e["ms_krylov"]
        acc["ms_extend"] += e["ms_extend"]
        log(f"[{label}] step {i}: {1e3 * (time.perf_counter() - ts):.1f} ms (krylov {e['ms_krylov']:.1f}, "
            f"extend {e['ms_extend']:.1f}, sweep {s['ms']:.1f}), max bond {max(m['bond_dims'])}, E={m['energy']:.10f}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if mark:
        torch.cuda._sleep(1000)
        torch.cuda.synchronize()
    acc["elapsed"] = el
    acc["final"] = T.tdvp_measure(ctx, [psi], [H])[0]
    acc["H"], acc["op"], acc["psi"] = H, op, psi
    return acc


def summarize(acc, steps, prec):
    gemm_tf = acc["flops_heff_gemm"] / (acc["ms_heff_gemm"] * 1e-3) / 1e12 if acc["ms_heff_gemm"] > 0 else None
    mv_tf = acc["flops_matvec"] / (acc["ms_matvec"] * 1e-3) / 1e12 if acc["ms_matvec"] > 0 else None
    return {
        "value": steps / acc["elapsed"],
        "ms_per_step": 1e3 * acc["elapsed"] / max(steps, 1),
        "matvec_tflops": mv_tf,
        "heff_gemm_tflops": gemm_tf,
        "heff_gemm_frac_of_peak": (gemm_tf / PEAK_TFLOPS[prec]) if gemm_tf else None,
        "heff_gemm_mfma_frac_of_peak": (gemm_tf * MFMA_PER_FLOP[prec] / PEAK_TFLOPS[prec]) if gemm_tf else None,
        "split_ms_per_step": {"krylov": acc["ms_krylov"] / steps, "extend": acc["ms_extend"] / steps,
                              "sweep": acc["ms_sweep"] / steps, "heff_matvec": acc["ms_matvec"] / steps},
        "heff_gemm_launches": acc["n_heff_gemm"],
        "heff_gemm_avg_us": 1e3 * acc["ms_heff_gemm"] / acc["n_heff_gemm"] if acc["n_heff_gemm"] else None,
        "max_bond": max(acc["final"]["bond_dims"]),
        "energy": acc["final"]["energy"],
    }


def oat_mode(args):
    """One-axis twisting (section II.B): N spins, H = (S^z_tot)^2 (w = 3 MPO),
    from the +x product state, eps = 0, with the section's two settings:
    dt = 0.025, k = 3, eps_K = eps_M = 1e-4, or dt = 0.05, k = 5, eps_K = 1e-4,
    eps_M = 1e-8 (the default).
    Each timed step is expand + sweep + the total-spin moments of eqs.
    (13)-(15) measured on the device as MPO expectation values, and xi^2 of
    eq. (15) from them by the library.  After the timer stops the trajectory
    is checked against the closed form of eq. (13) and the exact
    symmetric-subspace squeezing parameter (oracle, not timed)."""
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    torch.cuda.set_device(0)
    N = args.oat_n
    if abs(args.oat_dt - 0.025) < 1e-12:
        w = I.oat_workload(N, dt=0.025, k=3, eps_K=1e-4, eps_M=1e-4)
    else:
        w = I.oat_workload(N, dt=args.oat_dt, k=5, eps_K=1e-4, eps_M=1e-8)
    ctx = T.Context(0)
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    names = ("x", "yy", "zz", "yz")
    mops = {k: T.tdvp_create_mpo(ctx, N, I.spin_moment_terms(N, k)) for k in names}
    psi = T.tdvp_mps_from_host(ctx, w.initial_mps())
    e0 = T.tdvp_measure(ctx, [psi], [H])[0]["energy"]
    dt = w.dt.real
    rows = []

    split = {"krylov": 0.0, "extend": 0.0, "sweep": 0.0}

    def step(i):
        e = T.tdvp_expand_basis(ctx, [psi], [op], w.k, w.eps_K, w.eps_M, w.chi_max, "fp64")[0]
        sw = T.tdvp_sweep(ctx, [psi], [H], w.dt, w.eps, w.chi_max, 1e-12, 30, "fp64", False)[0]
        if i >= args.warmup:
            split["krylov"] += e["ms_krylov"] / args.steps
            split["extend"] += e["ms_extend"] / args.steps
            split["sweep"] += sw["ms"] / args.steps
        mom = {k: T.tdvp_measure(ctx, [psi], [mops[k]])[0]["energy"] for k in names}
        m = T.tdvp_measure(ctx, [psi], [H])[0]
        xi2 = T.tdvp_squeezing_xi2(N, mom["x"], mom["yy"], mom["zz"], mom["yz"])
        rows.append({"t": (i + 1) * dt, "sx": mom["x"], "xi2": xi2,
                     "energy_rel_drift": abs(m["energy"] - e0) / abs(e0), "max_bond": max(m["bond_dims"])})
        r = rows[-1]
        log(f"[oat{N}] step {i}: t={r['t']:.3f} <Sx>={r['sx']:.8f} xi2={xi2:.6f} max bond {r['max_bond']}")

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        step(i)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    # checks against the exact dynamics, after timing
    from oracle import observables as O
    for r in rows:
        r["sx_exact"] = O.oat_sx_exact(N, r["t"])
        r["xi2_exact"] = O.oat_xi2_dicke(N, r["t"])
    out = {
        "metric": "GSE-TDVP1 steps/s on one-axis twisting, with squeezing moments",
        "value": args.steps / el, "unit": "GSE-TDVP1 steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / max(args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"one-axis twisting N={N}, +x start", "dt": dt, "k": w.k, "eps_K": w.eps_K,
                   "eps_M": w.eps_M, "eps": 0.0, "mpo_w_max": int(max(H.dims)), "parallelism": "single GPU"},
        "sx_max_rel_err_vs_eq13": max(abs(r["sx"] - r["sx_exact"]) / (0.5 * N) for r in rows),
        "xi2_max_rel_err_vs_exact": max(abs(r["xi2"] - r["xi2_exact"]) / r["xi2_exact"] for r in rows),
        "energy_max_rel_drift": max(r["energy_rel_drift"] for r in rows),
        "xi2_min": min(r["xi2"] for r in rows), "t_at_xi2_min": min(rows, key=lambda r: r["xi2"])["t"],
        "t_opt_formula": O.oat_t_opt(N), "max_bond": max(r["max_bond"] for r in rows),
        "split_ms_per_step": split,
        "krylov_plus_extension_over_sweep": (split["krylov"] + split["extend"]) / split["sweep"] if split["sweep"] else None,
        "trajectory": rows,
    }
    print(json.dumps(out), flush=True)


def apply_compare_mode(args):
    """The two MPO applications of section I.C on the state of the main bench
    (64-site ladder brought to chi = 256 by four imaginary-time GSE steps):
    one Krylov vector (1 - i tau H)|psi> with the bench's eps_K and chi_max by
    the density-matrix algorithm and by variational fitting with 1 and 3
    passes, each timed K times, with the fidelity between the results."""
    import numpy as np
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    torch.cuda.set_device(0)
    ctx = T.Context(0)
    w = I.workload(1)
    N = w.lattice.n_sites
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    psi = T.tdvp_mps_from_host(ctx, w.initial_mps())
    for i in range(4):
        T.tdvp_expand_basis(ctx, [psi], [op], w.k, w.eps_K, w.eps_M, w.chi_max, "fp64")
        T.tdvp_sweep(ctx, [psi], [H], w.dt, w.eps, w.chi_max, 1e-12, 30, "fp64", w.normalize)
    log(f"[apply] state: max bond {max(psi.bond_dims())}, MPO bond dimension up to {max(op.dims)}")
    rows, outs = {}, {}
    for name, method, passes in (("denmat", "denmat", 1), ("fit1", "fit", 1), ("fit3", "fit", 3)):
        times = []
        for r in range(args.steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, disc = T.tdvp_apply_mpo(ctx, psi, op, method, w.eps_K, w.chi_max, passes)
            torch.cuda.synchronize()
            if r > 0:
                times.append(1e3 * (time.perf_counter() - t0))
            if r < args.steps:
                del h
        outs[name] = h
        rows[name] = {"ms": float(np.median(times)), "max_bond": max(h.bond_dims()), "discarded": disc}
        log(f"[apply] {name}: {rows[name]['ms']:.1f} ms, max bond {rows[name]['max_bond']}, discarded {disc:.3e}")
    for name in ("fit1", "fit3"):
        o = T.tdvp_measure(ctx, [outs["denmat"]], None, [outs[name]])[0]
        rows[name]["infidelity_vs_denmat"] = float(1.0 - abs(o["overlap"]) ** 2)
        log(f"[apply] 1 - |<denmat|{name}>|^2 = {rows[name]['infidelity_vs_denmat']:.3e}")
    print(json.dumps({"mode": "apply_compare", "workload": w.name, "chi_max": w.chi_max, "eps_K": w.eps_K,
                      "steps": args.steps, "results": rows}))


def tdvp2_compare_mode(args):
    """GSE-TDVP1 against two-site TDVP at the same bond dimension m' (the cost
    statement closing section I.C, made for real time with k = 5 and m' ~ 3m):
    the 64-site ladder of the main bench is prepared at bond dimension
    m = chi/3 (four imaginary-time GSE steps), quenched to the rung-coupled
    ladder and evolved in real time with dt = 0.05, k = 5, eps_K = 1e-4,
    eps_M = 1e-8, eps = 0 (the section II.B settings for dt = 0.05).  Timed:
    one GSE-TDVP1 step from the bond-m state (its extension grows the bonds to
    m' <= chi), and one two-site TDVP sweep of a state already at m' with the
    cap m'; each K times from the same states."""
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    torch.cuda.set_device(0)
    ctx = T.Context(0)
    w0 = I.workload(1)
    N = w0.lattice.n_sites
    chi = w0.chi_max
    m = chi // 3
    H0 = T.tdvp_create_mpo(ctx, N, w0.terms)
    op0 = T.tdvp_create_mpo(ctx, N, w0.terms, 1.0, -1j * w0.tau)
    psi = T.tdvp_mps_from_host(ctx, w0.initial_mps())
    for i in range(4):
        T.tdvp_expand_basis(ctx, [psi], [op0], w0.k, w0.eps_K, w0.eps_M, m, "fp64")
        T.tdvp_sweep(ctx, [psi], [H0], w0.dt, w0.eps, m, 1e-12, 30, "fp64", True)
    lat1 = I.ladder(32, 1.0, 1.0, "zigzag")
    terms1 = I.heisenberg_terms(lat1.couplings)
    dt, k, eK, eM = 0.05, 5, 1e-4, 1e-8
    H1 = T.tdvp_create_mpo(ctx, N, terms1)
    op1 = T.tdvp_create_mpo(ctx, N, terms1, 1.0, -1j * dt)
    start = T.tdvp_mps_to_host(psi)
    m0 = T.tdvp_measure(ctx, [psi], [H1])[0]
    log(f"[compare] prepared: max bond {max(m0['bond_dims'])}, E(H1) = {m0['energy']:.10f}")
    del psi
    split = {"krylov": 0.0, "extend": 0.0, "sweep": 0.0}
    ms_gse = 0.0
    mprime = 0
    after = None
    for i in range(args.steps + 1):
        g = T.tdvp_mps_from_host(ctx, start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e = T.tdvp_expand_basis(ctx, [g], [op1], k, eK, eM, chi, "fp64")[0]
        sw = T.tdvp_sweep(ctx, [g], [H1], dt, 0.0, chi, 1e-12, 30, "fp64", False)[0]
        torch.cuda.synchronize()
        el = 1e3 * (time.perf_counter() - t0)
        mprime = max(mprime, e["max_bond"])
        log(f"[compare] GSE-TDVP1 step from m = {max(m0['bond_dims'])}: {el:.0f} ms (krylov {e['ms_krylov']:.0f}, "
            f"extend {e['ms_extend']:.0f}, sweep {sw['ms']:.0f}), m' = {e['max_bond']}")
        if i > 0:
            ms_gse += el / args.steps
            split["krylov"] += e["ms_krylov"] / args.steps
            split["extend"] += e["ms_extend"] / args.steps
            split["sweep"] += sw["ms"] / args.steps
        after = T.tdvp_mps_to_host(g)
        del g
    ms_t2 = 0.0
    for i in range(args.steps + 1):
        g2 = T.tdvp_mps_from_host(ctx, after)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = T.tdvp_sweep2(ctx, [g2], [H1], dt, 0.0, mprime, 1e-12, 30, "fp64", False)[0]
        torch.cuda.synchronize()
        el = 1e3 * (time.perf_counter() - t0)
        log(f"[compare] TDVP2 sweep at m' = {mprime}: {el:.0f} ms, pair matvecs {st['n_matvec']}")
        if i > 0:
            ms_t2 += el / args.steps
        del g2
    out = {
        "metric": "GSE-TDVP1 step time over two-site TDVP step time at equal bond dimension",
        "value": ms_gse / ms_t2, "unit": "ratio", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": ms_gse, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2x32 ladder prepared at m = chi/3, quenched to J_rung = 1, real time",
                   "n_sites": N, "m": max(m0["bond_dims"]), "m_prime": mprime, "chi_max": chi, "dt": dt, "k": k,
                   "eps_K": eK, "eps_M": eM, "eps": 0.0, "parallelism": "single GPU"},
        "ms_per_gse_step": ms_gse, "ms_per_tdvp2_step": ms_t2, "gse_split_ms": split,
        "gse_steps12_over_step3": (split["krylov"] + split["extend"]) / split["sweep"] if split["sweep"] else None,
        "paper_ratio_context": "section I.C reports about 0.36 for this ratio and about 1/3 for steps 1+2 over "
                               "step 3 (CPU, ITensor)",
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def batch_mode(args):
    """Many independent ladders (seeded leg lengths U{8..32}, couplings
    U[0.5,1.5]) stepped together: each C-ABI call takes all instances and runs
    them concurrently on worker streams.  Reports instance-steps/s, and the
    same instances stepped one call at a time for comparison."""
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    torch.cuda.set_device(0)
    ws = I.ladder_batch(args.batch_size, 5)
    prec = args.prec or "fp32"
    w0 = ws[0]
    ctx = T.Context(0)
    Hs = [T.tdvp_create_mpo(ctx, w.lattice.n_sites, w.terms) for w in ws]
    ops = [T.tdvp_create_mpo(ctx, w.lattice.n_sites, w.terms, 1.0, -1j * w.tau) for w in ws]
    psis = [T.tdvp_mps_from_host(ctx, w.initial_mps()) for w in ws]

    def step(idx):
        ps, os_, hs = [psis[j] for j in idx], [ops[j] for j in idx], [Hs[j] for j in idx]
        T.tdvp_expand_basis(ctx, ps, os_, w0.k, w0.eps_K, w0.eps_M, w0.chi_max, prec)
        T.tdvp_sweep(ctx, ps, hs, w0.dt, w0.eps, w0.chi_max, 1e-12, 30, prec, w0.normalize)
        return T.tdvp_measure(ctx, ps, hs)

    allidx = list(range(len(ws)))
    if args.batch_serial:
        for i in range(args.warmup + args.steps):
            for j in allidx:
                try:
                    step([j])
                except Exception as e:
                    log(f"[serial] step {i} instance {j} ({ws[j].name}): {e}")
                    raise
            log(f"[serial] step {i} done")
        return
    for i in range(args.warmup):
        t = time.perf_counter()
        m = step(allidx)
        log(f"[batch] warmup {i}: {1e3 * (time.perf_counter() - t):.0f} ms, max bond {max(max(x['bond_dims']) for x in m)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        t = time.perf_counter()
        m = step(allidx)
        log(f"[batch] step {i}: {1e3 * (time.perf_counter() - t):.0f} ms")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    batched = len(ws) * args.steps / el
    # the same instances, one call per instance (one step each)
    t1 = time.perf_counter()
    for j in allidx:
        step([j])
    torch.cuda.synchronize()
    seq = len(ws) / (time.perf_counter() - t1)
    out = {"metric": "GSE-TDVP1 instance-steps/s on independent ladders", "value": batched,
           "unit": "instance-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
           "config": {"workload": f"{len(ws)} ladders, leg U{{8..32}}, J U[0.5,1.5], seed 5",
                      "chi_max": w0.chi_max, "k": w0.k, "dt": [w0.dt.real, w0.dt.imag],
                      "n_sites_total": sum(w.lattice.n_sites for w in ws), "parallelism": "16 worker streams"},
           "one_call_per_instance": seq, "speedup_concurrent": batched / seq,
           "mean_energy_per_site": sum(x["energy"] / w.lattice.n_sites for x, w in zip(m, ws)) / len(ws)}
    del psis, Hs, ops
    ctx.close()
    print(json.dumps(out), flush=True)


def kernel_only(args):
    """Short run for hardware-counter passes: H_eff applications at the bench
    workload's full size (chi = 256, w = 8, FP64 by default) and a plain copy
    of known size.  With --kernel-chi / --kernel-w other sizes (the chi = 1024,
    w = 20 cylinder shapes) are timed, with the two H_eff GEMM shapes timed
    apart as well."""
    import numpy as np
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    chi, w = args.kernel_chi, args.kernel_w
    ctx = T.Context(0)
    dt = torch.complex128 if args.prec in (None, "fp64") else torch.complex64
    kp = None if args.prec in (None, "fp64") else args.prec
    L = torch.from_numpy(I.random_hermitian_env(chi, w, 1)).to(dt).cuda()
    Rt = torch.from_numpy(np.ascontiguousarray(I.random_hermitian_env(chi, w, 2).transpose(1, 2, 0))).to(dt).cuda()
    Cin = torch.from_numpy(I.random_complex((chi, 2, chi), 3)).to(dt).cuda()
    Y = torch.empty_like(Cin)
    W = I.random_mpo_site(w, w, 4)
    nnz = int(np.count_nonzero(W))
    ws = torch.empty((4 * w + 32) * chi * chi, dtype=dt, device="cuda")
    for _ in range(3):
        T.tdvp_heff_apply(ctx, W, L, Rt, Cin, Y, ws, prec=kp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        T.tdvp_heff_apply(ctx, W, L, Rt, Cin, Y, ws, prec=kp)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(args.steps, 1)
    fl = 8.0 * (2 * chi ** 3 * w * 2 + nnz * chi * chi)
    log(f"kernel-only: H_eff application {ms * 1e3:.1f} us incl. host W upload, {fl / ms / 1e9:.1f} TFLOP/s")
    # the two GEMM stages alone (the same kernels, launched through tdvp_gemm)
    peak = PEAK_TFLOPS[args.prec or "fp64"]
    T1 = torch.empty((chi * w, 2 * chi), dtype=dt, device="cuda")
    for name, (M_, N_, K_, A_, B_, C_) in {"GEMM1 L.C": (chi * w, 2 * chi, chi, L, Cin, T1),
                                           "GEMM2 T2.Rt": (2 * chi, chi, w * chi, T1, Rt, Y)}.items():
        for _ in range(2):
            T.tdvp_gemm(ctx, 0, 0, M_, N_, K_, 1.0, A_, K_, 0, B_, N_, 0, 0.0, C_, N_, 0, 1, prec=kp)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            T.tdvp_gemm(ctx, 0, 0, M_, N_, K_, 1.0, A_, K_, 0, B_, N_, 0, 0.0, C_, N_, 0, 1, prec=kp)
        e1.record()
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / max(args.steps, 1)
        gfl = 8.0 * M_ * N_ * K_
        log(f"kernel-only: {name} M={M_} N={N_} K={K_}: {gms * 1e3:.1f} us, {gfl / gms / 1e9:.1f} TFLOP/s "
            f"({100 * gfl / gms / 1e9 / peak:.1f}% of the {args.prec or 'fp64'} peak)")
    src = torch.empty(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"kernel-only: {args.steps} H_eff applications at chi={chi}, w={w}; copied {src.numel() * 8} bytes")
    ctx.close()


def cylinder_mode(args):
    """The chi = 1024 workload: J1-J2 cylinder 4 x 16 (64 sites, J2 = 0.5,
    snake path, MPO bond dimension 20), real-time quench from the Neel state
    with U(1) S^z charges on every bond, dt = 0.1, k = 3, eps_K = 1e-4,
    eps_M = 1e-8, eps = 0, chi_max = 1024, Krylov vectors by variational
    fitting (two passes; the density-matrix route's double-layer environments
    would take ~430 GB at this size).

    The state is first grown from Neel (untimed, FP32) until the largest bond
    reaches chi_max; from that state each precision runs W + K steps, the last
    K timed.  The headline mixed precision (default FP32 contractions; the
    Lanczos recurrences, factorisations and stored tensors stay FP64) and
    BF16 inputs with FP32 accumulation (split into two BF16 terms, and
    plain) are compared with FP64 on the same steps: fidelity, energy and
    <S^z_i> differences of the final states."""
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T
    torch.cuda.set_device(0)
    w = I.workload(3)
    N = w.lattice.n_sites
    prec = args.prec or "fp32"
    chi = w.chi_max
    passes = 2
    ctx = T.Context(0)
    H = T.tdvp_create_mpo(ctx, N, w.terms)
    op = T.tdvp_create_mpo(ctx, N, w.terms, 1.0, -1j * w.tau)
    states = w.lattice.neel()
    g = T.tdvp_mps_from_host(ctx, I.product_mps(states), I.product_charges(states))
    log(f"workload {w.name} (charges): N={N}, w={max(H.dims)}, chi_max={chi}, k={w.k}, dt={w.dt}")
    t_prep = time.perf_counter()
    prep_steps = 0
    prep_elapsed = []    # cumulative time after each preparation step
    while prep_steps < 30:
        T.tdvp_expand_basis(ctx, [g], [op], w.k, w.eps_K, w.eps_M, chi, "fp32", apply="fit", fit_passes=passes)
        T.tdvp_sweep(ctx, [g], [H], w.dt, w.eps, chi, 1e-12, 30, "fp32", False)
        prep_steps += 1
        mb = max(g.bond_dims())
        prep_elapsed.append(time.perf_counter() - t_prep)
        log(f"[prepare] step {prep_steps}: max bond {mb} ({prep_elapsed[-1]:.1f} s)")
        if mb >= chi:
            break
    snap, snapq = T.tdvp_mps_to_host(g), T.tdvp_mps_charges(g)
    del g
    q = snapq[N // 2]
    sectors = {int(c): int((q == c).sum()) for c in sorted(set(q.tolist()))}

    def run(p):
        psi = T.tdvp_mps_from_host(ctx, snap, snapq)
        torch.cuda.synchronize()
        acc = {"ms_heff_gemm": 0.0, "flops_heff_gemm": 0.0, "n_heff_gemm": 0, "ms_matvec": 0.0,
               "flops_matvec": 0.0, "n_matvec": 0, "ms_sweep": 0.0, "ms_krylov": 0.0, "ms_extend": 0.0}
        t0 = None
        mark = args.mark_timed and p == prec
        for i in range(args.warmup + args.steps):
            if i == args.warmup:
                torch.cuda.synchronize()
                if mark:   # a kernel trace is cut to the dispatches between the two marks
                    torch.cuda._sleep(1000)
                    torch.cuda.synchronize()
                t0 = time.perf_counter()
            ts = time.perf_counter()
            e = T.tdvp_expand_basis(ctx, [psi], [op], w.k, w.eps_K, w.eps_M, chi, p, apply="fit",
                                    fit_passes=passes)[0]
            s = T.tdvp_sweep(ctx, [psi], [H], w.dt, w.eps, chi, 1e-12, 30, p, False)[0]
            m = T.tdvp_measure(ctx, [psi], [H])[0]
            if i >= args.warmup:
                for k in ("ms_heff_gemm", "flops_heff_gemm", "n_heff_gemm", "ms_matvec", "flops_matvec", "n_matvec"):
                    acc[k] += s[k]
                acc["ms_sweep"] += s["ms"]
                acc["ms_krylov"] += e["ms_krylov"]
                acc["ms_extend"] += e["ms_extend"]
            log(f"[{p}] {'warmup' if i < args.warmup else 'step'} {i}: {1e3 * (time.perf_counter() - ts):.0f} ms "
                f"(krylov {e['ms_krylov']:.0f}, extend {e['ms_extend']:.0f}, sweep {s['ms']:.0f}), "
                f"max bond {max(m['bond_dims'])}, E={m['energy']:.10f}")
        torch.cuda.synchronize()
        acc["elapsed"] = time.perf_counter() - (t0 if t0 is not None else time.perf_counter())
        if mark:
            torch.cuda._sleep(1000)
            torch.cuda.synchronize()
            # a plain device copy of known size (64 MiB read, 64 MiB written)
            # after the window: the calibration of the HBM byte counters
            src = torch.empty(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
        acc["final"] = T.tdvp_measure(ctx, [psi], [H])[0]
        acc["H"], acc["psi"] = H, psi
        return acc

    # the FP64 run is the reference every mixed run is compared with
    ref_run = run("fp64") if prec != "fp64" and args.fp64_ref else None
    main_run = run(prec)
    res = summarize(main_run, args.steps, prec)
    gemm_tf = res["heff_gemm_tflops"]
    peak = PEAK_TFLOPS[prec]
    t_total = abs(w.dt) * (args.warmup + args.steps)

    def against_fp64(run_, r):
        if ref_run is None:
            return
        ov = T.tdvp_measure(ctx, [run_["psi"]], None, [ref_run["psi"]])[0]
        fid = abs(ov["overlap"]) ** 2 / (ref_run["final"]["norm"] ** 2 * run_["final"]["norm"] ** 2)
        r["fidelity_vs_fp64"] = fid
        r["fidelity_loss_per_unit_time"] = (1 - fid) / t_total
        r["energy_diff_vs_fp64"] = run_["final"]["energy"] - ref_run["final"]["energy"]
        r["max_abs_sz_diff_vs_fp64"] = float(abs(run_["final"]["sz"] - ref_run["final"]["sz"]).max())

    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "GSE-TDVP1 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": w.name + " (U(1) S^z charges)", "n_sites": N, "chi_max": chi, "k": w.k,
                   "dt": [w.dt.real, w.dt.imag], "eps_K": w.eps_K, "eps_M": w.eps_M, "eps": w.eps,
                   "mpo_w_max": int(max(H.dims)), "krylov_route": f"variational fitting, {passes} passes (contractions in the run's precision, splits FP64)",
                   "prepared_by": f"{prep_steps} FP32 GSE-TDVP1 steps from Neel (untimed)",
                   "charge_sectors_mid_bond": sectors, "parallelism": "single GPU"},
    }
    out.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step")})
    against_fp64(main_run, out)
    out["heff_gemm_flops_count"] = "nonzero charge blocks only (8 flops per complex MAC)"
    traffic = traffic_from_profile(f"heff_gemm_counters_cyl4x16_chi1024_{prec}.md", [CSRC_KERNELS, CSRC_BLOCKS])
    out["roofline"] = {"bound": "mfma", "kernel": "one-site H_eff GEMM (TAG=1), block-sparse by charge",
                       "achieved": gemm_tf, "peak": peak, "unit": "TFLOP/s",
                       "frac": (gemm_tf / peak) if gemm_tf else None, "traffic": traffic,
                       "issued_mfma_frac": (gemm_tf * MFMA_PER_FLOP[prec] / peak) if gemm_tf else None}
    if ref_run is not None:
        rf = summarize(ref_run, args.steps, "fp64")
        out["speedup_vs_fp64"] = res["value"] / rf["value"]
        out["fp64"] = rf
    others = args.compare.split(",") if args.compare else ["bf16x3", "bf16"]
    for other in others if args.compare_prec else []:
        if other in (prec, "fp64") or other not in PEAK_TFLOPS:
            continue
        alt = run(other)
        ra = summarize(alt, args.steps, other)
        against_fp64(alt, ra)
        if ref_run is not None:
            ra["speedup_vs_fp64"] = ra["value"] / out["fp64"]["value"]
        out[other] = ra
        del alt
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for up to {args.cpu_seconds:.0f} s ...")
        cb = cpu_baseline(w, args.cpu_seconds, chi)
        cb["sample"] += " (dense tensors: the oracle has no charges)"
        n = cb["steps_timed"]
        if 0 < n <= len(prep_elapsed):
            # the device on the same sample: the first n preparation steps (FP32, charges)
            cb["gpu_steps_per_s_same_sample"] = n / prep_elapsed[n - 1]
        out["cpu_baseline"] = cb
    del main_run, ref_run
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", type=int, default=3,
                    help="0..3: the benchmark workloads (3, the default: the chi = 1024 cylinder with charges)")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "bf16x3"], default=None)
    ap.add_argument("--compare", default=None,
                    help="comma-separated precisions run after the main one on the same workload "
                         "(default: fp32,bf16x3,bf16 after fp64; fp64 after a mixed precision)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-ref", dest="fp64_ref", action="store_false",
                    help="cylinder: skip the FP64 reference run (no fidelity or speedup figures)")
    ap.add_argument("--mark-timed", action="store_true",
                    help="launch a short marker kernel (torch.cuda._sleep) right before and after the "
                         "headline precision's timed steps, for cutting a kernel trace or counter file (cylinder: "
                         "and a plain 64 MiB device copy after them for calibrating the byte counters)")
    ap.add_argument("--no-compare-prec", dest="compare_prec", action="store_false",
                    help="skip the runs in the other precisions (mixed vs FP64)")
    ap.add_argument("--batch", action="store_true",
                    help="many independent ladders stepped concurrently (instance-steps/s)")
    ap.add_argument("--batch-size", type=int, default=64)
    ap.add_argument("--batch-serial", action="store_true", help="step the batch one instance per call")
    ap.add_argument("--tdvp2-compare", action="store_true",
                    help="GSE-TDVP1 step against a two-site TDVP step at the same bond dimension")
    ap.add_argument("--apply-compare", action="store_true",
                    help="one Krylov vector by the density-matrix and the variational MPO application")
    ap.add_argument("--kernel-chi", type=int, default=256)
    ap.add_argument("--kernel-w", type=int, default=8)
    ap.add_argument("--oat", action="store_true",
                    help="one-axis twisting workload with squeezing moments (section II.B)")
    ap.add_argument("--oat-n", type=int, default=100)
    ap.add_argument("--oat-dt", type=float, default=0.05, help="0.025 (k = 3) or 0.05 (k = 5)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only H_eff applications at full size plus a plain copy (for counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the GSE-TDVP1 sweep of one MPS is sequential over sites and "
              f"the library has no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    if args.steps is None:
        args.steps = 2 if args.workload == 3 else 6
    if args.warmup is None:
        args.warmup = 1 if args.workload == 3 else 4
    if args.kernel_only:
        kernel_only(args)
        return
    if args.batch:
        batch_mode(args)
        return
    if args.oat:
        oat_mode(args)
        return
    if args.tdvp2_compare:
        tdvp2_compare_mode(args)
        return
    if args.apply_compare:
        apply_compare_mode(args)
        return
    if args.workload == 3:
        cylinder_mode(args)
        return
    import torch

    from paper_2005_06104_amd import inputs as I
    from paper_2005_06104_amd import tdvp as T

    torch.cuda.set_device(0)
    w = I.workload(args.workload)
    prec = args.prec or ("fp64" if w.prec == "fp64" else "fp32")
    N = w.lattice.n_sites
    ctx = T.Context(0)
    log(f"workload {w.name}: N={N}, chi_max={w.chi_max}, k={w.k}, dt={w.dt}, prec={prec}")
    main_run = run_workload(T, ctx, w, prec, args.warmup, args.steps, prec, mark=args.mark_timed)
    res = summarize(main_run, args.steps, prec)
    gemm_tf = res["heff_gemm_tflops"]
    peak = PEAK_TFLOPS[prec]
    traffic = traffic_from_profile("heff_gemm_traffic_ladder64_chi256.md", [CSRC_KERNELS]) \
        if prec == "fp64" and args.workload == 1 else None
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "GSE-TDVP1 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": w.name, "n_sites": N, "chi_max": w.chi_max, "k": w.k,
                   "dt": [w.dt.real, w.dt.imag], "eps_K": w.eps_K, "eps_M": w.eps_M, "eps": w.eps,
                   "mpo_w_max": int(max(main_run["H"].dims)), "parallelism": "single GPU"},
    }
    out.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step")})
    out["roofline"] = {"bound": "mfma", "kernel": "one-site H_eff GEMM (gemm_kernel TAG=1)",
                       "achieved": gemm_tf, "peak": peak, "unit": "TFLOP/s",
                       "frac": (gemm_tf / peak) if gemm_tf else None, "traffic": traffic}
    if args.compare_prec:
        others = args.compare.split(",") if args.compare else (
            ["fp32", "bf16x3", "bf16"] if prec == "fp64" else ["fp64"])
        for other in others:
            if other == prec or other not in PEAK_TFLOPS:
                continue
            alt = run_workload(T, ctx, w, other, args.warmup, args.steps, other)
            ra = summarize(alt, args.steps, other)
            ov = T.tdvp_measure(ctx, [alt["psi"]], None, [main_run["psi"]])[0]
            fid = abs(ov["overlap"]) ** 2 / (main_run["final"]["norm"] ** 2 * alt["final"]["norm"] ** 2)
            ra["fidelity_vs_" + prec] = fid
            ra["energy_diff_vs_" + prec] = ra["energy"] - res["energy"]
            ra["max_abs_sz_diff_vs_" + prec] = float(abs(alt["final"]["sz"] - main_run["final"]["sz"]).max())
            ra["speedup_vs_" + prec] = ra["value"] / res["value"]
            t_total = abs(w.dt) * (args.warmup + args.steps)
            ra["fidelity_loss_per_unit_time"] = (1 - fid) / t_total
            out[other] = ra
            del alt
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for up to {args.cpu_seconds:.0f} s ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, min(w.chi_max, res["max_bond"]))
    del main_run
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
