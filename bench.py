#!/usr/bin/env python
"""Steps/s of the KSA-XL-BOMD hot path on the 840-atom carbon cluster.

One step = one pass of the whole per-step path of the method (paper,
Methods sections 3-6): leapfrog and damped X-Verlet integration (eqs. 27-29,
35), Fock build F = h + G(X) (eq. 17), the finite-temperature density matrix
with its chemical potential (eqs. 7, 8, 19), the rank-m Krylov kernel with m
canonical responses (eqs. 34, 36), and the eq. 37 forces with the shadow
energy.  Workload: the 840-atom synthetic carbon cluster (3360 x 3360 Fock,
T_e = 5000 K, rank m = 6, dt = 0.5 fs), seeded; inputs are resident in HBM
before the timed region.  Every timed step starts from the same prepared MD
state (--trajectory free runs one continuous NVE trajectory instead).

Prints one JSON line.  --gpus N > 1 is rejected: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "XL-BOMD steps/s at 840 C atoms; split-BF16 vs FP64, force err ≤1e-4 eV/Å"
MODES = ["fp64", "bf16x3", "bf16x6", "fp16x3", "dm64_bf16x3", "dm64_bf16x6", "dm64_fp16x3"]
PEAK_F64, PEAK_LOWP = 78.6, 2500.0     # TFLOP/s, dense MFMA (FP64; BF16 and FP16)
DTYPE = {"fp64": "f64", "bf16x3": "bf16", "bf16x6": "bf16", "fp16x3": "f16",
         "dm64_bf16x3": "bf16", "dm64_bf16x6": "bf16", "dm64_fp16x3": "f16"}
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_state(binding, torch, sys_, X0, dev):
    n = sys_.n_orb
    Xr = torch.zeros((7, n, n), dtype=torch.float64, device=dev)
    Xr[0] = X0
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev).contiguous()
    return binding.MDState(R=t(sys_.R), V=t(sys_.V), A=torch.zeros((sys_.n_atoms, 3), dtype=torch.float64,
                                                                  device=dev),
                           X=Xr, Y=torch.zeros((n, n), dtype=torch.float64, device=dev), head=0,
                           mu=float("nan"))


def cpu_baseline(sys_, w, X, threads=0):
    """Oracle (plain FP64 NumPy) on a bounded sample of the same step: one Fock
    build, one density matrix by eigendecomposition, one Krylov direction
    (G(V) plus canonical response) and the forces; the step time is
    t_fock + t_dm + m * t_dir + t_forces.  threads > 0 limits the BLAS pools."""
    if threads > 0:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=threads):
            return cpu_baseline(sys_, w, X)
    import numpy as np
    from oracle import model, density, dynamics
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        pools = threadpool_info()
        cores = max([i.get("num_threads", 1) for i in pools] + [1])
        blas = ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in pools
                                 if i.get("user_api") == "blas"})) or blas
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    p = sys_.params
    beta = density.beta_of(w["T_e"])
    t0 = time.perf_counter()
    F = model.fock(X, sys_.R, sys_.onecenter, sys_.noise, p)
    t1 = time.perf_counter()
    dm = density.density_matrix(F, sys_.n_elec, beta)
    t2 = time.perf_counter()
    V = dm["P"] - X
    V = V / np.linalg.norm(V)
    F1 = model.two_electron(V, sys_.R, sys_.onecenter, sys_.noise, p)
    density.response(F, F1, sys_.n_elec, beta, dm)
    t3 = time.perf_counter()
    dynamics.forces(sys_.R, dm["P"], X, p, sys_.noise)
    t4 = time.perf_counter()
    t_step = (t1 - t0) + (t2 - t1) + w["m"] * (t3 - t2) + (t4 - t3)
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
            "host": {"cpus": os.cpu_count(), "blas": blas},
            "sample": (f"one oracle step at the 840-atom state assembled from timed parts: Fock build "
                       f"{t1 - t0:.1f} s, eigendecomposition density matrix {t2 - t1:.1f} s, one Krylov "
                       f"direction (G(V) + Loewner response) {t3 - t2:.1f} s x m={w['m']}, forces "
                       f"{t4 - t3:.1f} s; {t4 - t0:.1f} s of CPU work measured")}


def kernel_traffic(kclass):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (two rocprofv3 --pmc runs, FETCH_SIZE and WRITE_SIZE, scaled by the
    same counters on a plain copy), or None when the summary is missing or was
    taken on a different version of the kernel's source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c840.json")
    src = {"gemm_f64": "gemm_f64.hip", "gemm_split": "gemm_split.hip", "fock": "pairs.hip"}.get(kclass)
    if not src or not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kclass)
    if not rec:
        return None
    with open(os.path.join(ROOT, "paper_2303_00689_amd", "csrc", src), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["hbm_bytes_per_launch"]


def run_ensemble(args, binding, torch, dev):
    """Batch steps/s of a ragged ensemble: member i is the cluster of
    ensemble_sizes()[i] atoms from seed 4000 + i, on a stream of its own;
    every timed step restarts each member from its prepared state."""
    from synth import carbon_cluster, ensemble_sizes
    sizes = ensemble_sizes(args.ensemble)
    w = {"T_e": 3000.0, "m": 4, "dt": 0.5}
    t = time.perf_counter()
    hs, states, snaps, streams = [], [], [], []
    for i, na in enumerate(sizes):
        sys_ = carbon_cluster(int(na), 4000 + i)
        n = sys_.n_orb
        R0 = torch.tensor(sys_.R, dtype=torch.float64, device=dev)
        hi = binding.handle_for(sys_, w, prec="fp16x3")
        hi.set_geometry(R0)
        X0 = torch.eye(n, dtype=torch.float64, device=dev) * (sys_.n_elec / n)
        hi.scf(X0, m=8, tol=1e-12, max_iter=0, allow_noconv=True)   # 50 mixing steps
        hi.close()
        strm = torch.cuda.Stream()
        h = binding.Handle(sys_.n_atoms, sys_.n_elec, sys_.onecenter, sys_.noise, sys_.params, prec=args.prec,
                           T_e=w["T_e"], m=w["m"], dt=w["dt"], stream=strm.cuda_stream)
        st = make_state(binding, torch, sys_, X0, dev)
        torch.cuda.synchronize()
        h.md_init(st)
        torch.cuda.synchronize()
        hs.append(h)
        states.append(st)
        streams.append(strm)
        snaps.append((st.R.clone(), st.V.clone(), st.A.clone(), st.X.clone(), st.Y.clone(), st.head, st.mu))
    log(f"ensemble of {len(hs)} prepared ({time.perf_counter() - t:.1f} s)")

    def restore():
        for st, sn in zip(states, snaps):
            for dst, src in zip((st.R, st.V, st.A, st.X, st.Y), sn[:5]):
                dst.copy_(src)
            st.head, st.mu = sn[5], sn[6]
        torch.cuda.synchronize()

    def timed(fn):
        tot = 0.0
        for k in range(args.warmup + args.steps):
            restore()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if k >= args.warmup:
                tot += time.perf_counter() - t0
        return tot / args.steps

    t_ens = timed(lambda: binding.ensemble_step(hs, states, 1, report=False))
    log("ensemble steps done")
    t_seq = timed(lambda: [h.step(st, 1, report=False) for h, st in zip(hs, states)])
    log("sequential steps done")
    for h in hs:
        h.close()
    print(json.dumps({
        "metric": "ensemble batch steps/s (ragged carbon clusters, one step of every member per batch step)",
        "value": 1.0 / t_ens, "unit": "batch steps/s", "ms_per_batch_step": 1e3 * t_ens,
        "sequential_ms_per_batch_step": 1e3 * t_seq, "members": len(hs),
        "atoms": int(sum(sizes)), "sizes": [int(x) for x in sizes], "dtype": DTYPE[args.prec],
        "config": {"workload": f"{len(hs)} clusters of 20-300 atoms (seed 4000 + i), T_e 3000 K, rank 4, "
                               f"dt 0.5 fs", "precision": args.prec},
        "steps": args.steps, "warmup": args.warmup, "data": "synthetic"}))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="dm64_bf16x3", choices=MODES)
    ap.add_argument("--workload", default="c840")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="BLAS threads of the oracle leg (0: all)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--drift-steps", type=int, default=6,
                    help="free NVE steps per precision for the shadow-energy drift of the comparison")
    ap.add_argument("--init-mix", type=int, default=200, help="linear-mixing steps before MD")
    ap.add_argument("--no-report", action="store_true", help="skip the untimed report step after timing")
    ap.add_argument("--trajectory", choices=["reset", "free"], default="reset",
                    help="reset: every step starts from the prepared MD state (default); "
                         "free: one continuous NVE trajectory")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="instead: the ragged ensemble of this many clusters (20-300 atoms, 3000 K, "
                         "rank 4) through xlbomd_ensemble_step, against the same members stepped one "
                         "after another")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from synth import workload
    from paper_2303_00689_amd import binding

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.copy_bytes:
        # one elementwise kernel that reads and writes copy_bytes each: the
        # reference for scaling the FETCH_SIZE / WRITE_SIZE counters
        x = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": 5}))
        return
    if args.ensemble:
        run_ensemble(args, binding, torch, dev)
        return
    sys_, w = workload(args.workload)
    n = sys_.n_orb

    # ---- initial state (untimed): linear mixing from the uniform density
    # (X <- X + 0.04 (D0[X] - X), 50 steps per library call) in the fast
    # FP16x3 chain (a kernel instance the timed modes do not use, so profiles
    # of the timed path stay clean); the clusters' SCF is stiff, so MD starts
    # from this partially converged density and the residual is reported
    t = time.perf_counter()
    R0 = torch.tensor(sys_.R, dtype=torch.float64, device=dev)
    hi = binding.handle_for(sys_, w, prec="fp16x3")
    hi.set_geometry(R0)
    X0 = torch.eye(n, dtype=torch.float64, device=dev) * (sys_.n_elec / n)
    res = float("nan")
    for k in range(args.init_mix // 50):
        res = hi.scf(X0, m=8, tol=1e-12, max_iter=0, allow_noconv=True)
        log(f"init mixing {50 * (k + 1)} steps: residual {res:.3e} ({time.perf_counter() - t:.1f} s)")
    hi.close()
    h = binding.handle_for(sys_, w, prec=args.prec)
    h.set_geometry(R0)
    state = make_state(binding, torch, sys_, X0, dev)
    h.md_init(state)
    # The seeded random clusters are far from mechanical equilibrium (forces of
    # tens of eV/Angstrom), so a free NVE trajectory heats by thousands of K per
    # few steps and its per-step cost drifts with it.  By default every step
    # therefore starts from the same prepared state (t0 after md_init); the
    # restore is a few device copies on the library's stream, inside the
    # timed region.  A step writes the nuclei, Y and the one ring slot of X it
    # advances into, (head + 6) % 7; those are what the restore puts back.
    slot = (state.head + 6) % 7
    snap = (state.R.clone(), state.V.clone(), state.A.clone(), state.X[slot].clone(), state.Y.clone(),
            state.head, state.mu)

    def restore():
        if args.trajectory == "reset":
            for dst, src in zip((state.R, state.V, state.A, state.X[slot], state.Y), snap[:5]):
                dst.copy_(src)
            state.head, state.mu = snap[5], snap[6]

    for k in range(args.warmup):
        restore()
        h.step(state, 1, report=False)
        log(f"warmup step {k + 1} done")

    # ---- timed region
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        restore()
        h.step(state, 1, report=False)
    torch.cuda.synchronize()
    log("timed steps done")
    elapsed = time.perf_counter() - t0
    prof = h.profile_read()
    h.profile(False)
    steps_per_s = args.steps / elapsed
    # one more (untimed) step with the full report: shadow energy, chain depth
    restore()
    rep = None if args.no_report else h.step(state, 1, report=True)[0]

    # dominant kernel: the GEMM class with the larger share of the timed region
    split_kind = args.prec.split("_")[-1]
    g64, gs = prof["gemm_f64"], prof["gemm_split"]
    # profiled work is executed MFMA flops (every split product counts)
    if gs["ms"] >= g64["ms"]:
        g, peak, kname, kcls = gs, PEAK_LOWP, f"split GEMM ({split_kind})", "gemm_split"
    else:
        g, peak, kname, kcls = g64, PEAK_F64, "FP64 GEMM", "gemm_f64"
    gemm_tfs = g["work"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    fk = prof["fock"]
    fock_gbs = fk["work"] / (fk["ms"] * 1e-3) / 1e9 if fk["ms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded 840-atom carbon cluster, random-init integrals)",
        "config": {"workload": "840-atom carbon cluster, 3360x3360 Fock, T_e 5000 K, Krylov rank 6, dt 0.5 fs",
                   "n_atoms": sys_.n_atoms, "n_orb": n, "T_e_K": w["T_e"], "rank": w["m"], "dt_fs": w["dt"],
                   "precision": args.prec, "init_mixing_steps": args.init_mix, "trajectory": args.trajectory,
                   "init_residual": res},
        "roofline": {"bound": "mfma", "kernel": kname, "achieved": gemm_tfs, "peak": peak,
                     "unit": "TFLOP/s", "frac": gemm_tfs / peak, "traffic": kernel_traffic(kcls),
                     "launches": g["launches"], "avg_launch_us": 1e3 * g["ms"] / max(g["launches"], 1),
                     "share_of_step": g["ms"] * 1e-3 / elapsed},
        "other_gemm": {"fp64_ms_per_step": g64["ms"] / args.steps, "split_ms_per_step": gs["ms"] / args.steps,
                       "fp64_tflops": (g64["work"] / (g64["ms"] * 1e-3) / 1e12) if g64["ms"] > 0 else 0.0,
                       "split_executed_tflops": (gs["work"] / (gs["ms"] * 1e-3) / 1e12) if gs["ms"] > 0 else 0.0,
                       "fp64_launches": g64["launches"], "split_launches": gs["launches"]},
        "step_report": None if rep is None else {k: rep[k] for k in ("E_tot", "mu", "W0", "relres", "rank",
                                                                      "levels", "mu_passes")},
        "fock_roofline": {"bound": "hbm", "achieved": fock_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": fock_gbs / HBM_PEAK_GBS, "traffic": kernel_traffic("fock"), "launches": fk["launches"],
                          "avg_launch_us": 1e3 * fk["ms"] / max(fk["launches"], 1)},
    }

    # ---- split vs FP64 at the same state (untimed): D0, the response D1 to a
    # seeded G(V), the Krylov kernel Y, forces and U at the prepared state, and
    # the shadow-energy drift of a short free trajectory from it
    if args.prec != "fp64" and not args.no_compare:
        restore()
        Xsnap = state.X.clone()  # the whole prepared history
        Xc = state.x_current().clone()
        rng = np.random.default_rng(11)
        Vd = rng.standard_normal((n, n))
        Vd = torch.tensor(Vd + Vd.T, dtype=torch.float64, device=dev)
        beta = 1.0 / (8.617333262e-5 * w["T_e"])
        cmp = {}
        for pr, hh in (("split", h), ("fp64", None)):
            hnd = hh or binding.handle_for(sys_, w, prec="fp64")
            hnd.set_geometry(state.R)
            F = torch.empty_like(Xc)
            P = torch.empty_like(Xc)
            hnd.fock(Xc, F, True)
            _, S = hnd.fermi_dm(F, P, mu=state.mu)
            f = torch.empty((sys_.n_atoms, 3), dtype=torch.float64, device=dev)
            e = hnd.forces(P, Xc, f)
            F1 = torch.empty_like(Xc)
            hnd.fock(Vd, F1, False)
            P1 = torch.empty_like(Xc)
            hnd.dm_response(F1, P1)
            Y = torch.empty_like(Xc)
            hnd.krylov_kernel(Xc, P, w["m"], Y)
            U = e[0] + e[1] + e[2] - 2.0 * S / beta
            # drift: E_tot over a short free NVE trajectory from the prepared state
            st = binding.MDState(R=snap[0].clone(), V=snap[1].clone(), A=snap[2].clone(), X=Xsnap.clone(),
                                 Y=snap[4].clone(), head=snap[5], mu=snap[6])
            reps = hnd.step(st, args.drift_steps, report=True)
            E = np.array([r["E_tot"] for r in reps])
            tfs = w["dt"] * np.arange(1, len(E) + 1)
            drift = float(np.polyfit(tfs, E, 1)[0]) * 1000.0 / sys_.n_atoms
            torch.cuda.synchronize()
            cmp[pr] = dict(P=P.cpu().numpy(), P1=P1.cpu().numpy(), Y=Y.cpu().numpy(), f=f.cpu().numpy(), U=U,
                           drift=drift)
            if hh is None:
                hnd.close()
        a_, b_ = cmp["split"], cmp["fp64"]
        fro = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
        W0 = float(np.linalg.norm(b_["P"] - Xc.cpu().numpy()))
        ferr = float(np.abs(a_["f"] - b_["f"]).max())
        out["force_err_vs_fp64_eV_per_A"] = ferr
        out["density_err_vs_fp64"] = float(np.abs(a_["P"] - b_["P"]).max())
        out["force_err_ok"] = ferr <= 1e-4
        out["split_vs_fp64"] = {
            "D0_maxabs": float(np.abs(a_["P"] - b_["P"]).max()) / 2.0, "D0_rel_fro": fro(a_["P"], b_["P"]),
            "D1_rel_fro": fro(a_["P1"], b_["P1"]), "Y_rel_W0": float(np.linalg.norm(a_["Y"] - b_["Y"]) / W0),
            "forces_maxabs_eV_per_A": ferr, "U_eV_per_atom": abs(a_["U"] - b_["U"]) / sys_.n_atoms,
            "drift_eV_per_ps_per_atom": {"split": a_["drift"], "fp64": b_["drift"],
                                         "steps": args.drift_steps, "trajectory": "free NVE from the prepared state"}}

    if not args.no_cpu_baseline:
        log("timing the oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(sys_, w, state.x_current().cpu().numpy(), args.cpu_threads)
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
