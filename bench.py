"""Benchmark of the MSC-LBM dual-time march on one MI355X.

Workload (default): D3Q19, N = 128, FP64 populations and arithmetic (the
paper's precision), 3D Taylor-Green vortex plus a seeded divergence-free
perturbation (|k| <= 8, amplitude 1e-2 U), Re = 1 at nu = 1/6, BDF2 dt =
63.83 (154 physical steps to the horizon 0.1 N^2/nu = 9830 lattice steps),
n_min = 2, linear trial.  A "step" is one physical BDF step: setup, the
corrected inner iterations (sweep, residual, shadow correction) and
acceptance.  The tolerance is chosen by the paper's protocol: every candidate
eps runs the full horizon, and the fastest passing both accuracy gates (the
matched gate against the linear Stokes decay, and the 1% engineering gate
against the FP64 explicit endpoint) is the one timed.

Printed: one JSON line with wall-seconds per viscous time (N^2/nu lattice
steps) of the timed corrected march, the full-horizon speedup over the
explicit TRT march (the library's in-place AA march, same GPU) under the
gate that passed,
the dominant kernel's achieved bandwidth from per-launch HIP events against
the MI355X HBM peak, the FP64 CPU oracle timed on a bounded sample on the
host, and the other workloads (FP32 3D, the 2D random fields at N = 256 and
1024 in FP32 and FP16-deviation storage, the differentiable march, the
paper's 2D Taylor-Green matched-gate cells at N = 256 ... 1024).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rms(a):
    return math.sqrt(float((a ** 2).sum(0).mean()))


def stokes_decay(u0, t, nu):
    """Linear Stokes decay of a periodic field: each Fourier mode times
    exp(-nu |k|^2 t) with the continuous wavenumbers."""
    shape = u0.shape[1:]
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n for n in shape], indexing="ij")
    k2 = sum(k ** 2 for k in ks)
    out = np.empty_like(u0)
    for a in range(u0.shape[0]):
        out[a] = np.real(np.fft.ifftn(np.fft.fftn(u0[a]) * np.exp(-nu * k2 * t)))
    return out


def sweep_beyond_cache(msc, stream, torch, NL=4096):
    """Sweep kernel bandwidth beyond the 256 MB last-level cache: D2Q9 at
    N = 4096 (two 604 MB FP32 population arrays), explicit and dual-time
    modes of the tiled sweep and the in-place AA march; D3Q19 at N = 256^3
    (two 1.27 GB arrays), the explicit tiled sweep and the AA march; and a
    plain device copy of 1.2 GB (torch) as a reference ceiling."""
    pz = np.zeros((NL, NL))
    uz = np.zeros((2, NL, NL))
    uz[0] = 1e-4 * np.sin(2 * np.pi * np.arange(NL) / NL)[None, :]
    p = msc.make_params(2, NL, dt=256.0, eps=1e-30, storage="fp32", corrector="picard", k_max=4)
    big = msc.Solver(p, pz, uz, stream=stream)
    big.set_tuning(10, 0)
    big.explicit_step(4)
    big.set_kernel_timing(True)
    big.explicit_step(20)
    xs, xn, xb = big.kernel_time(1)
    big.set_tuning(10, 1)
    big.explicit_step(4)
    big.set_kernel_timing(True)
    big.explicit_step(20)
    as_, an, ab = big.kernel_time(1)
    big.set_kernel_timing(True)
    big.bdf2_step(1, raise_on_fail=False)
    ds, dn, db = big.kernel_time(0)
    big.close()
    # D3Q19 N = 256^3: two 1.27 GB FP32 population arrays, explicit sweep
    N3 = 256
    p3 = msc.make_params(3, N3, dt=64.0, eps=1e-30, storage="fp32", corrector="picard", k_max=4)
    z3 = torch.zeros((N3, N3, N3), dtype=torch.float64, device="cuda")
    u3 = torch.zeros((3, N3, N3, N3), dtype=torch.float64, device="cuda")
    u3[0] = 1e-4 * torch.sin(2 * math.pi * torch.arange(N3, dtype=torch.float64, device="cuda") / N3)[None, None, :]
    big3 = msc.Solver(p3, z3, u3, stream=stream)
    big3.set_tuning(10, 0)
    big3.explicit_step(2)
    big3.set_kernel_timing(True)
    big3.explicit_step(10)
    ys, yn, yb = big3.kernel_time(1)
    big3.set_tuning(10, 1)
    big3.explicit_step(2)
    big3.set_kernel_timing(True)
    big3.explicit_step(10)
    zs, zn, zb = big3.kernel_time(1)
    big3.close()
    del z3, u3
    a = torch.empty(150 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(10):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    copy_s = ev0.elapsed_time(ev1) / 1e3 / 10
    copy_bytes = 2 * a.numel() * 4
    del a, b
    return {
        "N": NL, "storage": "fp32",
        "explicit": {"avg_launch_us": xs / xn * 1e6, "bytes_per_launch": xb, "achieved_GBs": xb / (xs / xn) / 1e9,
                     "frac": xb / (xs / xn) / 1e9 / HBM_PEAK_GBS},
        "dts": {"avg_launch_us": ds / dn * 1e6, "bytes_per_launch": db, "achieved_GBs": db / (ds / dn) / 1e9,
                "frac": db / (ds / dn) / 1e9 / HBM_PEAK_GBS, "launches": dn},
        "explicit_aa": {"avg_launch_us": as_ / an * 1e6, "bytes_per_launch": ab,
                        "achieved_GBs": ab / (as_ / an) / 1e9, "frac": ab / (as_ / an) / 1e9 / HBM_PEAK_GBS},
        "d3q19_n256_explicit": {"avg_launch_us": ys / yn * 1e6, "bytes_per_launch": yb,
                                "achieved_GBs": yb / (ys / yn) / 1e9, "frac": yb / (ys / yn) / 1e9 / HBM_PEAK_GBS},
        "d3q19_n256_explicit_aa": {"avg_launch_us": zs / zn * 1e6, "bytes_per_launch": zb,
                                   "achieved_GBs": zb / (zs / zn) / 1e9, "frac": zb / (zs / zn) / 1e9 / HBM_PEAK_GBS},
        "device_copy": {"bytes": copy_bytes, "avg_us": copy_s * 1e6, "achieved_GBs": copy_bytes / copy_s / 1e9,
                        "frac": copy_bytes / copy_s / 1e9 / HBM_PEAK_GBS},
    }


def traffic_profile(workload):
    """Committed counter summary of the dual-time sweep for a workload."""
    name = {"tgv3d_n128_fp64": "hbm_traffic_sweep_d3q19_n128_fp64.md",
            "rand2d_n256_fp32": "hbm_traffic_sweep_d2q9_n256_fp32.md"}.get(workload)
    return os.path.join(ROOT, "profiles", name) if name else None


def counter_traffic(path):
    """HBM bytes per sweep launch from a committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the sweep kernel's sources have changed since those
    counters were taken (or the summary is absent)."""
    if path is None:
        return None
    import hashlib
    try:
        fields = {}
        for line in open(path):
            line = line.strip().lstrip("- ")
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in fields["kernel_sources"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def calibration_copies(torch):
    """Five elementwise kernels b = 2 a over 64 MiB (a kernel of known
    traffic: 64 MiB read, 64 MiB written)."""
    a = torch.ones(16 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    return a.numel() * 4


def extra_workload(msc, W, stream, torch, name, storage, extrap=2, ref_cache=None, dt=None):
    """Corrected march against the explicit march (in-place AA, same storage)
    over the workload's whole horizon, both timed; accuracy against an FP64
    explicit endpoint (cached per workload) and against the linear Stokes
    decay of the initial field (matched gate); the speedup is reported under
    the gate that passed, or null."""
    cfg = W.config(name)
    N, nu, d = cfg["N"], cfg["nu"], cfg["d"]
    p0, u0 = W.initial_fields(cfg)
    T_end = cfg["T_end"]
    if dt is None:
        S, dt = cfg["S"], cfg["dt"]
    else:
        S = int(round(T_end / dt))
    tnu = N * N / nu

    def solver(st, corrector, eps=cfg["eps"], ex=extrap):
        p = msc.make_params(d, N, dt=dt, eps=eps, storage=st, corrector=corrector, n_min=cfg["nmin"],
                            extrap_states=ex)
        return msc.Solver(p, p0, u0, stream=stream)

    if ref_cache is not None and name in ref_cache:
        u_ref = ref_cache[name]
    else:
        r = solver("fp64", "picard")
        r.explicit_step(int(round(T_end)))
        u_ref = r.moments()[1:]
        r.close()
        if ref_cache is not None:
            ref_cache[name] = u_ref
    e = solver(storage, "picard")
    e.explicit_step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.explicit_step(int(T_end) - 64)
    torch.cuda.synchronize()
    t_exp = (time.perf_counter() - t0) * T_end / (T_end - 64)
    u_exp = e.moments()[1:]
    e.close()
    s = solver(storage, "shadow")
    s.bdf2_step(2)
    s.close()
    s = solver(storage, "shadow")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, stats = s.bdf2_step(S, raise_on_fail=False)
    torch.cuda.synchronize()
    t_msc = time.perf_counter() - t0
    u_msc = s.moments()[1:]
    s.close()
    iters = [x["iters"] for x in stats]
    e_msc = rms(u_msc - u_ref) / max(rms(u_ref), 1e-300)
    e_exp = rms(u_exp - u_ref) / max(rms(u_ref), 1e-300)
    # the same march with the paper's trial rule (up to cubic), for reference
    u_st0 = stokes_decay(u0, float(T_end), nu)
    paper_rule = None
    if extrap != 0:
        s = solver(storage, "shadow", ex=0)
        s.bdf2_step(2, raise_on_fail=False)
        s.close()
        s = solver(storage, "shadow", ex=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc0, st0 = s.bdf2_step(S, raise_on_fail=False)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        u_p = s.moments()[1:] if rc0 == 0 else None
        s.close()
        done0 = sum(1 for x in st0 if x["converged"])
        paper_rule = {"status": int(rc0), "steps_accepted": done0, "steps_requested": S, "seconds": t_p,
                      "mean_inner": float(np.mean([x["iters"] for x in st0[:max(done0, 1)]])) if st0 else None}
        if u_p is not None:
            e_p = rms(u_p - u_ref) / max(rms(u_ref), 1e-300)
            e_pst = rms(u_p - u_st0)
            paper_rule.update({"msc_rel_vs_fp64_explicit": e_p, "msc_abs_vs_stokes": e_pst,
                               "gate_1pct": e_p <= 1e-2, "gate_matched": e_pst <= 3.0 * rms(u_ref - u_st0)})
        log(f"[bench] {name} {storage} paper trial rule: status {rc0}, {done0}/{S} steps, "
            f"inner {paper_rule['mean_inner']}, {t_p:.3f} s")
    u_st = stokes_decay(u0, float(T_end), nu)
    e_st, e_ref_st = rms(u_msc - u_st), rms(u_ref - u_st)
    matched = rc == 0 and e_st <= 3.0 * e_ref_st
    eng1 = rc == 0 and e_msc <= 1e-2
    gate = "matched and 1%" if (matched and eng1) else ("1%" if eng1 else ("matched" if matched else None))
    Q = 9 if d == 2 else 19
    bsite = {"fp64": 16 * Q, "fp32": 8 * Q, "fp16dev": 4 * Q + 8 * (d + 1)}[storage]
    log(f"[bench] {name} {storage}: MSC {t_msc:.3f} s ({S} steps, inner {np.mean(iters):.2f}), explicit "
        f"{t_exp:.2f} s, speedup {t_exp / t_msc:.1f}; errors MSC {e_msc:.3e} explicit {e_exp:.3e}")
    return {
        "lattice": "D2Q9" if d == 2 else "D3Q19", "N": N, "Re": cfg["Re"], "storage": storage, "dt": dt,
        "eps": cfg["eps"], "n_min": cfg["nmin"], "extrap_states": extrap, "physical_steps": S,
        "horizon_lattice_steps": T_end, "status": int(rc),
        "msc_wall_s_per_viscous_time": t_msc * tnu / T_end, "explicit_wall_s_per_viscous_time": t_exp * tnu / T_end,
        "speedup_vs_explicit": (t_exp / t_msc) if gate else None, "speedup_gate": gate,
        "mean_inner": float(np.mean(iters)), "max_inner": int(max(iters)),
        "msc_rel_vs_fp64_explicit": e_msc, "explicit_rel_vs_fp64_explicit": e_exp,
        "msc_abs_vs_stokes": e_st, "fp64_explicit_abs_vs_stokes": e_ref_st,
        "gate_1pct": eng1, "gate_matched": matched, "msc_not_less_accurate_than_explicit": e_msc <= e_exp,
        "explicit_sweep_GBs": bsite * N ** d / (t_exp / T_end) / 1e9,
        "paper_trial_rule": paper_rule,
    }


def re_sweep(msc, W, stream, torch, res=(1e-4, 1e-2, 1.0, 10.0, 100.0), storages=("fp32", "fp16dev"),
             S_ladder=(64, 128, 256, 512), eps_rel=(1e-6, 1e-7, 1e-8)):
    """Reynolds sweep of the D2Q9 N = 1024 random-field workload (seeded
    |k|^-3 spectrum, |k| <= 16, nu = 1/6, Re set by U, horizon 0.1 N^2/nu).
    Per Re: the FP64 explicit endpoint as the reference; per storage the
    explicit march (timed over the whole horizon) and the corrected march
    over a ladder of physical step counts S (fewest first) and tolerances
    eps = e Re (the residual scales with U; e from eps_rel, loosest first):
    every candidate runs the whole horizon, and the fastest one passing the
    1% gate (RMS velocity difference from the FP64 explicit endpoint over its
    RMS) is reported with its speedup over the same-storage explicit march;
    the Stokes-decay error (the matched gate's reference, valid for the
    linear regime Re <= 1) is reported beside it.  The sweep kernel's
    achieved bandwidth comes from per-launch events over the first steps of
    the chosen candidate."""
    base = W.config("rand2d_n1024_fp32")
    N, nu, d = base["N"], base["nu"], 2
    T_end = base["T_end"]
    tnu = N * N / nu
    out = []
    for Re in res:
        U = Re * nu / N
        cfg = dict(base, Re=Re, U=U)
        p0, u0 = W.initial_fields(cfg)
        u_st = stokes_decay(u0, float(T_end), nu)

        def mk(st, corrector, S=64, eps=1e-8):
            p = msc.make_params(d, N, dt=T_end / S, eps=eps, storage=st, corrector=corrector, n_min=base["nmin"],
                                extrap_states=2)
            return msc.Solver(p, p0, u0, stream=stream)

        r = mk("fp64", "picard")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.explicit_step(int(T_end))
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t0
        u_ref = r.moments()[1:]
        r.close()
        nref = max(rms(u_ref), 1e-300)
        row = {"Re": Re, "U": U, "fp64_explicit_s": t_ref, "fp64_explicit_abs_vs_stokes": rms(u_ref - u_st),
               "storages": {}}
        for st in storages:
            e = mk(st, "picard")
            e.explicit_step(64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e.explicit_step(int(T_end) - 64)
            torch.cuda.synchronize()
            t_exp = (time.perf_counter() - t0) * T_end / (T_end - 64)
            u_exp = e.moments()[1:]
            e.close()
            e_exp = rms(u_exp - u_ref) / nref
            cands = []
            best = None
            for S in S_ladder:
                for er in eps_rel:
                    eps = er * Re
                    s = mk(st, "shadow", S, eps)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    rc, stats = s.bdf2_step(S, raise_on_fail=False)
                    torch.cuda.synchronize()
                    t_msc = time.perf_counter() - t0
                    done = sum(1 for x in stats if x["converged"])
                    u_msc = s.moments()[1:] if rc == 0 else None
                    s.close()
                    e_msc = rms(u_msc - u_ref) / nref if u_msc is not None else None
                    ok = rc == 0 and e_msc is not None and e_msc <= 1e-2
                    c = {"S": S, "eps": eps, "status": int(rc), "steps_accepted": done, "s": t_msc,
                         "mean_inner": float(np.mean([x["iters"] for x in stats[:max(done, 1)]])) if stats else None,
                         "rel_vs_fp64_explicit": e_msc,
                         "abs_vs_stokes": rms(u_msc - u_st) if u_msc is not None else None, "gate_1pct": ok}
                    cands.append(c)
                    if ok and (best is None or t_msc < best["s"]):
                        best = c
                if best is not None:
                    break
            res_st = {"explicit_s": t_exp, "explicit_rel_vs_fp64_explicit": e_exp,
                      "explicit_wall_s_per_viscous_time": t_exp * tnu / T_end, "candidates": cands, "best": best,
                      "speedup_vs_explicit": (t_exp / best["s"]) if best else None,
                      "speedup_gate": "1%" if best else None}
            if best is not None:
                s = mk(st, "shadow", best["S"], best["eps"])
                s.set_kernel_timing(True)
                s.bdf2_step(min(best["S"], 16), raise_on_fail=False)
                ks, kn, kb = s.kernel_time(0)
                s.close()
                res_st["msc_wall_s_per_viscous_time"] = best["s"] * tnu / T_end
                res_st["msc_not_less_accurate_than_explicit"] = best["rel_vs_fp64_explicit"] <= e_exp
                res_st["sweep"] = {"avg_launch_us": ks / max(kn, 1) * 1e6, "bytes_per_launch": kb,
                                   "achieved_GBs": kb / (ks / kn) / 1e9 if kn else None,
                                   "frac": kb / (ks / kn) / 1e9 / HBM_PEAK_GBS if kn else None}
            row["storages"][st] = res_st
            log(f"[re-sweep] Re={Re:g} {st}: explicit {t_exp:.2f} s (e {e_exp:.2e}); best "
                + (f"S={best['S']} eps={best['eps']:.1e} {best['s']:.3f} s e {best['rel_vs_fp64_explicit']:.2e} "
                   f"speedup {t_exp / best['s']:.1f}" if best else "none passed"))
        out.append(row)
    return {"workload": "rand2d_n1024 (D2Q9 N=1024, seeded |k|^-3 field, |k| <= 16, nu=1/6)",
            "horizon_lattice_steps": T_end, "gate": "1% (RMS velocity difference from the FP64 explicit endpoint "
            "over its RMS)", "rows": out}


def adjoint_workload(msc, W, stream, torch):
    """Differentiable march of the vorticity-control workload (D2Q9 N=256,
    20 steps of dt=64, FP32): forward march, forward with per-step
    checkpoints, and the backward pass (msc_bdf2_adjoint) timed on the GPU."""
    from paper_2609_39474_amd import autograd as AG

    cfg = W.config("vort2d_n256_adjoint")
    N, nsteps, dt = cfg["N"], cfg["nsteps"], cfg["dt"]
    w0 = torch.tensor(W.random_vorticity_2d(N, cfg["U"], seed=cfg["seed"]), device="cuda")
    u0 = AG.biot_savart(w0).contiguous()
    p0 = torch.zeros((N, N), dtype=torch.float64, device="cuda")

    def solver():
        p = msc.make_params(2, N, dt=dt, eps=cfg["eps"], storage=cfg["storage"], extrap_states=2)
        return msc.Solver(p, p0, u0, stream=stream)

    s = solver()
    s.bdf2_step(2)
    s.close()
    s = solver()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.bdf2_step(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s.close()
    s = solver()
    s.set_recording(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.bdf2_step(nsteps)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    lam = torch.zeros(s.state_size(), dtype=torch.float64, device="cuda")
    lam[3 * 9 * N * N + N * N:] = 1e-3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.bdf2_adjoint_device(nsteps, lam.data_ptr())
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    s.close()
    log(f"[bench] adjoint N={N}: forward {t_fwd * 1e3:.2f} ms, with checkpoints {t_rec * 1e3:.2f} ms, "
        f"backward {t_bwd * 1e3:.2f} ms")
    return {"N": N, "steps": nsteps, "dt": dt, "storage": cfg["storage"],
            "mean_inner": float(np.mean([x["iters"] for x in st])), "forward_s": t_fwd,
            "forward_with_checkpoints_s": t_rec, "backward_s": t_bwd,
            "backward_over_forward": t_bwd / t_fwd,
            "note": "backward recomputes each step's inner iterates in FP64 from its checkpoint, then "
                    "runs the FP64 transposed sweeps and corrections"}


def tgv_matched_cells(msc, W, stream, torch, cells=((256, 32, 1e-6, 0), (512, 64, 1e-6, 0), (1024, 256, 1e-8, 2)),
                      reps=3):
    """The paper's headline 2D comparison (Tab. tgv2d, matched gate) at N =
    256, 512, 1024, Re = 1, FP64: the decaying Taylor-Green vortex over
    T_end = nint(0.15 N^2); explicit march (minimum of two runs) against the
    corrected march at the fastest passing (S, eps, trial rule) of the full
    campaign (bench.py --tgv), re-timed here (minimum of reps runs) with the
    gate e_abs <= 3 e_explicit re-evaluated against the analytic field."""
    nu = 1.0 / 6.0
    out = []
    for N, S, eps, extrap in cells:
        U = nu / N
        T_end = W.nint(0.15 * N * N)
        p0, u0 = W.tgv2d(N, U, nu)
        _, u_an = W.tgv2d(N, U, nu, t=float(T_end))

        def mk(corr, dt):
            p = msc.make_params(2, N, dt=dt, eps=eps, storage="fp64", corrector=corr, n_min=2, k_max=300,
                                extrap_states=extrap)
            return msc.Solver(p, p0, u0, stream=stream)

        t_exp = math.inf
        for _ in range(2):
            e = mk("picard", float(T_end))
            e.explicit_step(64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e.explicit_step(T_end - 64)
            torch.cuda.synchronize()
            t_exp = min(t_exp, (time.perf_counter() - t0) * T_end / (T_end - 64))
            u_exp = e.moments()[1:]
            e.close()
        e_exp = rms(u_exp - u_an)
        w = mk("shadow", T_end / S)
        w.bdf2_step(2, raise_on_fail=False)
        w.close()
        t_msc, rc, e_abs, inner = math.inf, 0, None, None
        for _ in range(reps):
            s = mk("shadow", T_end / S)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = s.bdf2_step(S, raise_on_fail=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if rc == 0:
                t_msc = min(t_msc, t)
                e_abs = rms(s.moments()[1:] - u_an)
                inner = float(np.mean([x["iters"] for x in st]))
            s.close()
        passed = rc == 0 and e_abs is not None and e_abs <= 3.0 * e_exp
        row = {"N": N, "Re": 1.0, "T_end": T_end, "S": S, "eps": eps,
               "trial_rule": "paper" if extrap == 0 else f"{extrap} states", "explicit_s": t_exp, "msc_s": t_msc,
               "explicit_e_abs": e_exp, "msc_e_abs": e_abs, "gate_matched": passed, "mean_inner": inner,
               "S_wall": (t_exp / t_msc) if passed else None}
        log(f"[tgv-matched] N={N}: explicit {t_exp:.4f} s, MSC {t_msc:.4f} s, e {e_abs} vs 3x{e_exp:.3e} "
            f"-> S_wall {row['S_wall']}")
        out.append(row)
    return out


def envelope(msc, W, stream, torch, N=128):
    """Operating envelope of the corrected iteration (FP64 storage, one interior
    BDF2 step, eps = 1e-10, 2D Taylor-Green at Re = 1 unless stated):
    observed contraction rho_obs (Eq. rho-observed) along Lambda at nu = 1/6
    and along nu at Lambda = 1/4 beside the ghost-survival amplitude
    eta(nu) = |6 nu - 1| / (6 nu + 1) (Eq. eta), and the (Re, dt) stability
    cells of the step-size scan (Sec. 4.6)."""
    def one_step_rho(tau_p, tau_m, nu, dt, Re=1.0, flow="tgv", corrector="shadow"):
        U = Re * nu / N
        p0, u0 = W.tgv2d(N, U, nu) if flow == "tgv" else W.random_field_2d(N, U, seed=1)
        p = msc.make_params(2, N, dt=dt, eps=1e-10, storage="fp64", tau_plus=tau_p, tau_minus=tau_m,
                            k_max=2000, corrector=corrector)
        s = msc.Solver(p, p0, u0, stream=stream)
        rc, st = s.bdf2_step(2, raise_on_fail=False)
        s.close()
        last = st[-1]
        return {"status": int(rc), "iters": int(last["iters"]), "rho_obs": last["rho_obs"],
                "R_first": last["R_first"], "R_final": last["R_final"]}

    out = {"N": N, "dt": 64.0, "lambda_sweep_nu_1_6": [], "nu_sweep_lambda_1_4": [], "stability_re_dt": []}
    nu0 = 1.0 / 6.0
    for flow in ("tgv", "random"):
        for lam in (1 / 64, 1 / 16, 1 / 8, 3 / 16, 1 / 4, 3 / 8, 1 / 2, 1.0, 2.0, 4.0):
            tau_p = 0.5 + 3 * nu0
            tau_m = 0.5 + lam / (tau_p - 0.5)
            r = one_step_rho(tau_p, tau_m, nu0, 64.0, flow=flow)
            r.update({"flow": flow, "Lambda": lam, "tau_minus": tau_m, "odd_survival": abs(1 - 1 / tau_m)})
            r["full_symbol"] = one_step_rho(tau_p, tau_m, nu0, 64.0, flow=flow, corrector="full_symbol")
            out["lambda_sweep_nu_1_6"].append(r)
            log(f"[envelope] {flow} Lambda {lam:.4f}: rho {r['rho_obs']:.3f} iters {r['iters']} status {r['status']}; "
                f"full symbol rho {r['full_symbol']['rho_obs']:.2e} iters {r['full_symbol']['iters']}")
        for nu in (0.05, 0.06, 0.07, 0.08, 0.09, 0.1, 0.12, 0.14, 1 / 6, 0.2, 0.25, 0.35, 0.5):
            tau_p = 0.5 + 3 * nu
            tau_m = 0.5 + 1 / (12 * nu)
            r = one_step_rho(tau_p, tau_m, nu, 64.0, flow=flow)
            r.update({"flow": flow, "nu": nu, "eta": abs(6 * nu - 1) / (6 * nu + 1)})
            r["full_symbol"] = one_step_rho(tau_p, tau_m, nu, 64.0, flow=flow, corrector="full_symbol")
            out["nu_sweep_lambda_1_4"].append(r)
            log(f"[envelope] {flow} nu {nu:.4f}: eta {r['eta']:.3f} rho {r['rho_obs']:.3f} iters {r['iters']} "
                f"status {r['status']}; full symbol rho {r['full_symbol']['rho_obs']:.2e} "
                f"iters {r['full_symbol']['iters']}")
    # (Re, dt) cells at N = 128 (the paper's pair S = 32 stable, S = 16
    # divergent at Re = 100, and its scan at Re = 120, 150, 180)
    for Re in (100.0, 120.0, 150.0, 180.0):
        T_end = int(math.floor(0.15 * N * N + 0.5))
        for S in (128, 32, 16):
            dt = T_end / S
            U = Re * nu0 / N
            p0, u0 = W.tgv2d(N, U, nu0)
            p = msc.make_params(2, N, dt=dt, eps=1e-10, storage="fp64", k_max=3000)
            s = msc.Solver(p, p0, u0, stream=stream)
            rc, st = s.bdf2_step(S, raise_on_fail=False)
            m = s.moments() if rc == 0 else None
            s.close()
            ok = rc == 0 and bool(np.all(np.isfinite(m)))
            out["stability_re_dt"].append({"Re": Re, "S": S, "dt": dt, "status": int(rc), "stable": ok,
                                           "mean_inner": float(np.mean([x["iters"] for x in st]))})
            log(f"[envelope] Re {Re:.0f} dt {dt:.1f}: status {rc}")
    return out


def fullsym_cost(msc, W, stream, torch, sizes=((256, "fp32"), (256, "fp64"), (128, "fp64"))):
    """Cost of one inner iteration with the full-symbol reference corrector
    (Eq. full-symbol: every population field, every wavevector) beside the
    shadow correction (three fields, band-pruned), D2Q9 random field at the
    operating point, dt = 64: 4 timed BDF2 steps of 8 replayed iterations
    each after 2 untimed steps; plus the inner counts and seconds per step of
    both correctors run to eps = 1e-10 (FP64) at an off-design point
    (Lambda = 1/64 at nu = 1/6) and at nu = 0.1 on Lambda = 1/4."""
    out = []
    nu0 = 1.0 / 6.0
    for N, storage in sizes:
        p0, u0 = W.random_field_2d(N, nu0 / N, seed=1)
        row = {"N": N, "storage": storage}
        for corr in ("shadow", "full_symbol"):
            p = msc.make_params(2, N, dt=64.0, eps=1e-30, storage=storage, corrector=corr)
            s = msc.Solver(p, p0, u0, stream=stream)
            s.set_schedule([8] * 6)
            s.bdf2_step(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.bdf2_step(4)
            torch.cuda.synchronize()
            row[f"{corr}_us_per_iteration"] = (time.perf_counter() - t0) / 32 * 1e6
            s.close()
        row["cost_ratio"] = row["full_symbol_us_per_iteration"] / row["shadow_us_per_iteration"]
        log(f"[bench] full symbol N={N} {storage}: {row['full_symbol_us_per_iteration']:.1f} us/iteration, "
            f"shadow {row['shadow_us_per_iteration']:.1f} (x{row['cost_ratio']:.2f})")
        out.append(row)
    off = []
    N = 128
    for label, tp, tm in (("Lambda=1/64 nu=1/6", 1.0, 0.5 + (1 / 64) / 0.5),
                          ("nu=0.1 Lambda=1/4", 0.5 + 0.3, 0.5 + 1 / 1.2)):
        nu = (tp - 0.5) / 3.0
        p0, u0 = W.random_field_2d(N, nu / N, seed=1)
        row = {"point": label, "N": N, "tau_plus": tp, "tau_minus": tm}
        for corr in ("shadow", "full_symbol"):
            p = msc.make_params(2, N, dt=64.0, eps=1e-10, storage="fp64", corrector=corr, tau_plus=tp,
                                tau_minus=tm, k_max=2000)
            s = msc.Solver(p, p0, u0, stream=stream)
            s.bdf2_step(1, raise_on_fail=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = s.bdf2_step(1, raise_on_fail=False)
            torch.cuda.synchronize()
            row[corr] = {"status": int(rc), "iters": int(st[-1]["iters"]), "rho_obs": st[-1]["rho_obs"],
                         "seconds_per_step": time.perf_counter() - t0}
            s.close()
        log(f"[bench] off-design {label}: shadow {row['shadow']}, full symbol {row['full_symbol']}")
        off.append(row)
    return {"per_iteration": out, "off_design_step": off}


def tgv_campaign(msc, W, stream, torch, cells=None, storage="fp64", S_list=(4, 8, 16, 32, 64, 128, 256),
                 eps_list=(1e-6, 1e-8, 1e-10), extrap=0, reps=3):
    """The 2D periodic timing protocol of Sec. 4.1 (Tab. protocol) and its
    table of wall-clock ratios (Tab. tgv2d), on one GPU: the decaying
    Taylor-Green vortex (Eq. tgv2d, nu = 1/6, Lambda = 1/4, U = Re nu / N)
    over T_end = nint(0.15 N^2) lattice steps; every candidate (S, eps) with
    dt = T_end / S, K_max = 300, n_min = 2 and the paper's trial rule is run
    once; errors are the pointwise-vector RMS against the analytic field; the
    matched gate is e_abs <= 3 e_explicit, the engineering gate e_abs / RMS(u)
    <= 1%.  The fastest passing candidates of each gate are timed again and
    the ratio uses the minimum over reps runs (the explicit march: minimum of
    two)."""
    nu = 1.0 / 6.0
    if cells is None:
        cells = [(N, 1.0) for N in (32, 64, 128, 256, 512, 1024)] + [(N, 100.0) for N in (128, 256, 512, 1024)]
    out = []
    for N, Re in cells:
        U = Re * nu / N
        T_end = W.nint(0.15 * N * N)
        p0, u0 = W.tgv2d(N, U, nu)
        _, u_an = W.tgv2d(N, U, nu, t=float(T_end))

        def mk(corr, dt, eps):
            p = msc.make_params(2, N, dt=dt, eps=eps, storage=storage, corrector=corr, n_min=2, k_max=300,
                                extrap_states=extrap)
            return msc.Solver(p, p0, u0, stream=stream)

        t_exp = math.inf
        for _ in range(2):
            e = mk("picard", float(T_end), 1e-10)
            e.explicit_step(64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e.explicit_step(T_end - 64)
            torch.cuda.synchronize()
            t_exp = min(t_exp, (time.perf_counter() - t0) * T_end / (T_end - 64))
            u_exp = e.moments()[1:]
            e.close()
        e_exp = rms(u_exp - u_an)
        log(f"[tgv] N={N} Re={Re:g}: T_end {T_end}, explicit {t_exp:.4f} s, e_abs {e_exp:.3e}")
        w = mk("shadow", T_end / 8.0, 1e-8)  # kernels and allocator warm
        w.bdf2_step(2, raise_on_fail=False)
        w.close()

        def run(S, eps):
            s = mk("shadow", T_end / S, eps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = s.bdf2_step(S, raise_on_fail=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            u = s.moments()[1:]
            s.close()
            return int(rc), t, u, st

        cands = []
        for S in S_list:
            for eps in eps_list:
                rc, t, u, st = run(S, eps)
                e_abs = rms(u - u_an)
                e_eng = e_abs / max(rms(u), 1e-12)
                c = {"S": S, "eps": eps, "status": rc, "seconds": t, "e_abs": e_abs, "e_eng": e_eng,
                     "mean_inner": float(np.mean([x["iters"] for x in st])) if st else None,
                     "matched": rc == 0 and e_abs <= 3.0 * e_exp, "eng1": rc == 0 and e_eng <= 1e-2}
                cands.append(c)
                log(f"[tgv] N={N} Re={Re:g} S={S} eps={eps:g}: status {rc} {t:.4f} s e_abs {e_abs:.3e} "
                    f"e_eng {e_eng:.3e} inner {c['mean_inner']} matched {c['matched']} 1% {c['eng1']}")
        best = {}
        for gate in ("matched", "eng1"):
            passing = sorted([c for c in cands if c[gate]], key=lambda c: c["seconds"])[:3]
            for c in passing:
                for _ in range(reps - 1):
                    rc, t, _, _ = run(c["S"], c["eps"])
                    if rc == 0:
                        c["seconds"] = min(c["seconds"], t)
            if passing:
                b = min(passing, key=lambda c: c["seconds"])
                best[gate] = {"S": b["S"], "eps": b["eps"], "seconds": b["seconds"], "S_wall": t_exp / b["seconds"],
                              "e_abs": b["e_abs"], "e_eng": b["e_eng"], "mean_inner": b["mean_inner"]}
            else:
                best[gate] = None
            log(f"[tgv] N={N} Re={Re:g} {gate}: {best[gate]}")
        out.append({"N": N, "Re": Re, "U": U, "T_end": T_end, "storage": storage,
                    "trial_rule": "paper" if extrap == 0 else f"{extrap} states",
                    "explicit_s": t_exp, "explicit_e_abs": e_exp, "best": best, "candidates": cands})
    return out


def tgv3d_campaign(msc, W, stream, torch, cells=None, storage="fp64", S_list=(3, 4, 5, 8, 16, 32, 64),
                   eps_list=(1e-6, 1e-8, 1e-10, 1e-12), reps=3):
    """The 3D periodic timing protocol of Sec. 4.1 (Tab. protocol) and its
    table (Tab. tgv3d), on one GPU: the D3Q19 Taylor-Green field of Eq.
    tgv3d-ic (zero pressure, nu = 1/6, Lambda = 1/4) over T_end =
    nint(0.075 N^2); plain Picard and MSC over every candidate (S, eps) with
    n_min = 1 and K_max = 300.  Engineering error: RMS velocity difference
    from the same-grid FP64 explicit endpoint over U/2 (1% gate); matched
    gate (reading of the undefined 3D e_explicit): both endpoints against the
    linear Stokes decay of the initial field, e_DTS <= 3 e_explicit."""
    nu = 1.0 / 6.0
    if cells is None:
        cells = [(32, 1.0), (64, 1.0), (128, 1.0), (64, 100.0), (128, 100.0)]
    out = []
    for N, Re in cells:
        U = Re * nu / N
        T_end = W.nint(0.075 * N * N)
        p0, u0 = W.tgv3d(N, U)
        u_st = stokes_decay(u0, float(T_end), nu)

        def mk(corr, dt, eps, st=storage):
            p = msc.make_params(3, N, dt=dt, eps=eps, storage=st, corrector=corr, n_min=1, k_max=300)
            return msc.Solver(p, p0, u0, stream=stream)

        r = mk("picard", float(T_end), 1e-10, "fp64")
        r.explicit_step(T_end)
        u_ref = r.moments()[1:]
        r.close()
        t_exp = math.inf
        for _ in range(2):
            e = mk("picard", float(T_end), 1e-10)
            e.explicit_step(16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e.explicit_step(T_end - 16)
            torch.cuda.synchronize()
            t_exp = min(t_exp, (time.perf_counter() - t0) * T_end / (T_end - 16))
            u_exp = e.moments()[1:]
            e.close()
        e_exp_st = rms(u_exp - u_st)
        log(f"[tgv3d] N={N} Re={Re:g}: T_end {T_end}, explicit {t_exp:.4f} s, e vs Stokes {e_exp_st:.3e}")
        w = mk("shadow", T_end / 8.0, 1e-8)
        w.bdf2_step(2, raise_on_fail=False)
        w.close()

        def run(corr, S, eps):
            s = mk(corr, T_end / S, eps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = s.bdf2_step(S, raise_on_fail=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            u = s.moments()[1:]
            s.close()
            return int(rc), t, u, st

        cells_out = {}
        for corr in ("picard", "shadow"):
            cands = []
            for S in S_list:
                for eps in eps_list:
                    rc, t, u, st = run(corr, S, eps)
                    e_st = rms(u - u_st)
                    e_eng = rms(u - u_ref) / (U / 2)
                    c = {"S": S, "eps": eps, "status": rc, "seconds": t, "e_stokes": e_st, "e_eng": e_eng,
                         "mean_inner": float(np.mean([x["iters"] for x in st])) if st else None,
                         "matched": rc == 0 and e_st <= 3.0 * e_exp_st, "eng1": rc == 0 and e_eng <= 1e-2}
                    cands.append(c)
                    log(f"[tgv3d] N={N} Re={Re:g} {corr} S={S} eps={eps:g}: status {rc} {t:.4f} s e_st {e_st:.3e} "
                        f"e_eng {e_eng:.3e} inner {c['mean_inner']} matched {c['matched']} 1% {c['eng1']}")
            best = {}
            for gate in ("matched", "eng1"):
                passing = sorted([c for c in cands if c[gate]], key=lambda c: c["seconds"])[:3]
                for c in passing:
                    for _ in range(reps - 1):
                        rc, t, _, _ = run(corr, c["S"], c["eps"])
                        if rc == 0:
                            c["seconds"] = min(c["seconds"], t)
                if passing:
                    b = min(passing, key=lambda c: c["seconds"])
                    best[gate] = {"S": b["S"], "eps": b["eps"], "seconds": b["seconds"],
                                  "S_wall": t_exp / b["seconds"], "e_stokes": b["e_stokes"], "e_eng": b["e_eng"],
                                  "mean_inner": b["mean_inner"]}
                else:
                    best[gate] = None
                log(f"[tgv3d] N={N} Re={Re:g} {corr} {gate}: {best[gate]}")
            cells_out[corr] = {"best": best, "candidates": cands}
        out.append({"N": N, "Re": Re, "U": U, "T_end": T_end, "storage": storage, "explicit_s": t_exp,
                    "explicit_e_stokes": e_exp_st, "picard": cells_out["picard"], "msc": cells_out["shadow"]})
    return out


def cavity_campaign(msc, stream, torch, cells=((64, 10.0), (128, 10.0), (256, 10.0), (64, 100.0), (128, 100.0),
                                                (256, 100.0)),
                    S_list=(16, 32, 64), tol_list=(1e-2, 1e-4)):
    """D2Q9 lid-driven cavity (Sec. 3.3, Sec. 4.5): impulsive lid from rest,
    T_end = 1.5 N^2 lattice steps, FP64.  The explicit march with the same
    wall rows is the reference and the baseline; the Picard DTS march and
    Algorithm 2 (frozen and adaptive operator) run S physical steps each
    (dt = T_end / S, eps = 1e-10, K_max 4000 for Picard, 300 for Algorithm 2,
    n_min = 1 as printed in Algorithm 2) with the wall corrector's
    GMRES tolerance from tol_list.  Error: RMS velocity error against the
    explicit endpoint over the lid speed (lid-normalised); march ratio =
    explicit seconds / scheme seconds (both on this GPU)."""
    nu = 1.0 / 6.0
    out = []
    for N, Re in cells:
        ulid = Re * nu / N
        T_end = int(round(1.5 * N * N))
        z0, z1 = np.zeros((N, N)), np.zeros((2, N, N))

        def mk(corr, dt, op="frozen", tol=0.0):
            kmax = 4000 if corr == "picard" else 300
            p = msc.make_params(2, N, dt=dt, eps=1e-10, storage="fp64", corrector=corr, n_min=1, k_max=kmax,
                                boundary="cavity", u_lid=ulid, wall_operator=op, krylov_tol=tol)
            return msc.Solver(p, z0, z1, stream=stream)

        e = mk("picard", 1.0)
        e.explicit_step(64)
        e.close()
        e = mk("picard", 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.explicit_step(T_end)
        torch.cuda.synchronize()
        t_exp = time.perf_counter() - t0
        u_ref = e.moments()[1:]
        e.close()
        cell = {"N": N, "Re": Re, "u_lid": ulid, "T_end": T_end, "explicit_s": t_exp, "runs": []}
        log(f"[cavity] N={N} Re={Re:g}: explicit {t_exp:.3f} s for {T_end} steps")
        for S in S_list:
            dt = T_end / S
            variants = [("picard", "frozen", 0.0)]
            for tol in tol_list:
                variants += [("wall_kinetic", "frozen", tol), ("wall_kinetic", "adaptive", tol)]
            for corr, op, tol in variants:
                s = mk(corr, dt, op, tol)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, st = s.bdf2_step(S, raise_on_fail=False)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                err = float("nan")
                if rc == 0:
                    u = s.moments()[1:]
                    err = float(np.sqrt(((u - u_ref) ** 2).sum(0).mean()) / ulid)
                ks = s.krylov_stats()
                s.close()
                name = corr if corr == "picard" else f"{op}"
                run = {"S": S, "dt": dt, "scheme": name, "krylov_tol": tol, "status": int(rc), "seconds": t,
                       "march_ratio": t_exp / t if rc == 0 else None, "err_lid": err,
                       "mean_inner": float(np.mean([x["iters"] for x in st])) if st else None,
                       "refreshes": int(sum(x["refreshes"] for x in st)),
                       "krylov_iters_per_solve": (ks[1] / ks[0]) if ks[0] else None}
                cell["runs"].append(run)
                log(f"[cavity] N={N} Re={Re:g} S={S} {name:8s} tol {tol:g}: status {rc} {t:.3f} s ratio "
                    f"{(t_exp / t) if rc == 0 else 0:.2f} err {err:.2e} inner {run['mean_inner']} "
                    f"krylov/solve {run['krylov_iters_per_solve']}")
        out.append(cell)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="physical steps timed (0: the whole horizon)")
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="tgv3d_n128_fp64")
    ap.add_argument("--dt", type=float, default=0.0, help="BDF step (0: the workload's)")
    ap.add_argument("--eps-candidates", default="1e-6,1e-8,1e-10",
                    help="candidate tolerances; the fastest passing both accuracy gates is timed")
    ap.add_argument("--extrap", type=int, default=2,
                    help="population states in the initial-trial extrapolation (0: paper rule, up to cubic)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the beyond-cache sweep measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (FP32 3D, 2D N=256 and N=1024, adjoint, 2D matched-gate cells)")
    ap.add_argument("--march-only", action="store_true",
                    help="only the timed corrected march and its sweep timing pass (counter runs)")
    ap.add_argument("--re-sweep", action="store_true",
                    help="only the D2Q9 N=1024 Reynolds sweep (FP32 and FP16-deviation storage, 1%% gate)")
    ap.add_argument("--re-list", default="", help="Reynolds numbers of --re-sweep, comma separated")
    ap.add_argument("--envelope", action="store_true",
                    help="only the operating-envelope measurements (rho_obs along Lambda and nu, (Re, dt) cells)")
    ap.add_argument("--cavity", action="store_true",
                    help="only the lid-driven cavity campaign (explicit, Picard, Algorithm 2 frozen/adaptive)")
    ap.add_argument("--tgv", action="store_true",
                    help="only the 2D Taylor-Green timing campaign (explicit against MSC, matched and 1%% gates)")
    ap.add_argument("--tgv3d", action="store_true",
                    help="only the D3Q19 Taylor-Green timing campaign (explicit against Picard and MSC)")
    ap.add_argument("--tgv-cells", default="", help="campaign cells as N:Re,N:Re (default: the paper's set)")
    ap.add_argument("--tgv-storage", default="fp64", help="population storage of the campaign")
    ap.add_argument("--tgv-extrap", type=int, default=0, help="trial extrapolation cap (0 = the paper's rule)")
    ap.add_argument("--cavity-cells", default="", help="cavity cells as N:Re,N:Re (default: the full set)")
    ap.add_argument("--cavity-steps", default="", help="cavity physical step counts S, comma separated")
    ap.add_argument("--cavity-tols", default="", help="wall corrector GMRES tolerances, comma separated")
    ap.add_argument("--fullsym", action="store_true",
                    help="only the full-symbol reference corrector: cost per iteration and off-design steps")
    ap.add_argument("--calib", action="store_true",
                    help="end with five 64 MiB device copies (a known-size kernel for counter calibration)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the beyond-cache sweep measurement and a plain-copy calibration (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_39474_amd import msc, workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if args.sweep_only:
        r = sweep_beyond_cache(msc, stream, torch)
        print(json.dumps({"sweep_beyond_cache": r}), flush=True)
        return
    if args.envelope:
        print(json.dumps({"envelope": envelope(msc, W, stream, torch)}), flush=True)
        return
    if args.re_sweep:
        kw = {}
        if args.re_list:
            kw["res"] = tuple(float(v) for v in args.re_list.split(","))
        print(json.dumps({"re_sweep": re_sweep(msc, W, stream, torch, **kw)}), flush=True)
        return
    if args.fullsym:
        print(json.dumps({"full_symbol": fullsym_cost(msc, W, stream, torch)}), flush=True)
        return
    if args.tgv3d:
        kw = {}
        if args.tgv_cells:
            kw["cells"] = [(int(c.split(":")[0]), float(c.split(":")[1])) for c in args.tgv_cells.split(",")]
        print(json.dumps({"tgv3d_campaign": tgv3d_campaign(msc, W, stream, torch, storage=args.tgv_storage, **kw)}),
              flush=True)
        return
    if args.tgv:
        kw = {}
        if args.tgv_cells:
            kw["cells"] = [(int(c.split(":")[0]), float(c.split(":")[1])) for c in args.tgv_cells.split(",")]
        print(json.dumps({"tgv2d_campaign": tgv_campaign(msc, W, stream, torch, storage=args.tgv_storage,
                                                          extrap=args.tgv_extrap, **kw)}), flush=True)
        return
    if args.cavity:
        kw = {}
        if args.cavity_cells:
            kw["cells"] = tuple((int(c.split(":")[0]), float(c.split(":")[1])) for c in args.cavity_cells.split(","))
        if args.cavity_steps:
            kw["S_list"] = tuple(int(v) for v in args.cavity_steps.split(","))
        if args.cavity_tols:
            kw["tol_list"] = tuple(float(v) for v in args.cavity_tols.split(","))
        print(json.dumps({"cavity": cavity_campaign(msc, stream, torch, **kw)}), flush=True)
        return
    cfg = W.config(args.workload)
    N, nu, d = cfg["N"], cfg["nu"], cfg["d"]
    dt = args.dt if args.dt > 0 else cfg["dt"]
    T_end = cfg["T_end"]
    S_full = int(round(T_end / dt))
    T_full = S_full * dt
    K = args.steps if args.steps > 0 else S_full
    tnu = N * N / nu  # lattice steps per viscous time
    p0, u0 = W.initial_fields(cfg)
    storage = cfg["storage"]
    U = cfg["U"]
    dtype = {"fp64": "f64", "fp32": "f32", "fp16dev": "f16dev"}[storage]
    eps_list = [float(v) for v in args.eps_candidates.split(",")] if args.eps_candidates else [cfg["eps"]]

    def solver(eps, st=storage, corrector="shadow", extrap=args.extrap):
        p = msc.make_params(d, N, dt=dt, eps=eps, storage=st, corrector=corrector, n_min=cfg["nmin"],
                            extrap_states=extrap)
        return msc.Solver(p, p0, u0, stream=stream)

    def march(eps, steps, st=storage, extrap=args.extrap):
        s = solver(eps, st, extrap=extrap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, stats = s.bdf2_step(steps, raise_on_fail=False)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        u = s.moments()[1:] if rc == 0 else None
        s.close()
        return int(rc), t, u, stats

    log(f"[bench] workload {args.workload} N={N} dt={dt:.4f} S={S_full} steps={K} warmup={args.warmup} "
        f"eps candidates {eps_list}")
    if args.march_only:
        # profiling runs: only the corrected march (first candidate eps), then
        # the same steps with per-launch sweep timing
        eps = eps_list[0]
        s = solver(eps)
        s.bdf2_step(max(1, args.warmup), raise_on_fail=False)
        s.close()
        rc, t_msc, _, stats = march(eps, K)
        s = solver(eps)
        s.set_kernel_timing(True)
        s.bdf2_step(K, raise_on_fail=False)
        sec, launches, bytes_per = s.kernel_time(0)
        s.close()
        part = {"workload": args.workload, "steps": K, "eps": eps, "status": rc, "msc_s": t_msc,
                "mean_inner": float(np.mean([x["iters"] for x in stats])), "sweep_launches": launches,
                "sweep_avg_us": sec / max(launches, 1) * 1e6, "sweep_bytes_per_launch": bytes_per}
        if args.calib:
            part["calibration_copy_bytes_each_way"] = calibration_copies(torch)
        print(json.dumps(part), flush=True)
        return
    # ---- explicit march over the full horizon: the speedup baseline (same
    # kernel, same storage) and, in FP64, the reference endpoint of the
    # engineering gate
    nexp = int(round(T_full))
    t_exp = math.inf
    for _ in range(2):
        e = solver(cfg["eps"], corrector="picard")
        e.explicit_step(64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.explicit_step(nexp - 64)
        torch.cuda.synchronize()
        t_exp = min(t_exp, (time.perf_counter() - t0) * nexp / (nexp - 64))
        u_exp = e.moments()[1:]
        e.close()
    if storage == "fp64":
        u_ref = u_exp
    else:
        r = solver(cfg["eps"], st="fp64", corrector="picard")
        r.explicit_step(nexp)
        u_ref = r.moments()[1:]
        r.close()
    u_stokes = stokes_decay(u0, T_full, nu)
    e_exp_st = rms(u_ref - u_stokes)

    def eng_err(u):
        # 3D: RMS difference over U/2 (the paper's 3D engineering error);
        # 2D: relative to the reference RMS
        return rms(u - u_ref) / (U / 2) if d == 3 else rms(u - u_ref) / max(rms(u_ref), 1e-300)

    log(f"[bench] explicit: {t_exp:.3f} s for {nexp} lattice steps; FP64 explicit vs Stokes {e_exp_st:.3e}")

    # ---- tolerance by the paper's protocol (Sec. 4.1): every candidate eps
    # over the full horizon, gates against the Stokes decay (matched) and the
    # FP64 explicit endpoint (1%); the fastest candidate passing both is timed
    w = solver(eps_list[0])
    w.bdf2_step(2, raise_on_fail=False)
    w.close()
    cands = []
    for eps in eps_list:
        rc, t, u, st = march(eps, S_full)
        c = {"eps": eps, "status": rc, "seconds": t,
             "mean_inner": float(np.mean([x["iters"] for x in st])) if st else None}
        if rc == 0:
            c["e_vs_stokes"] = rms(u - u_stokes)
            c["e_eng"] = eng_err(u)
            c["gate_matched"] = c["e_vs_stokes"] <= 3.0 * e_exp_st
            c["gate_1pct"] = c["e_eng"] <= 1e-2
        else:
            c.update({"gate_matched": False, "gate_1pct": False})
        cands.append(c)
        log(f"[bench] eps {eps:g}: status {rc} {t:.3f} s inner {c['mean_inner']} e_stokes "
            f"{c.get('e_vs_stokes', float('nan')):.3e} e_eng {c.get('e_eng', float('nan')):.3e} "
            f"matched {c['gate_matched']} 1% {c['gate_1pct']}")
    passing = [c for c in cands if c["gate_matched"] and c["gate_1pct"]]
    chosen = min(passing, key=lambda c: c["seconds"]) if passing else min(cands, key=lambda c: c["eps"])
    eps = chosen["eps"]
    rc, t2, _, _ = march(eps, S_full)
    if rc == 0:
        chosen["seconds"] = min(chosen["seconds"], t2)
    gate = "matched and 1%" if passing else None

    # ---- timed region: K physical steps from t = 0 after W warmup steps on
    # a separate context
    s = solver(eps)
    s.bdf2_step(max(1, args.warmup), raise_on_fail=False)
    s.close()
    rc, t_msc, _, stats = march(eps, K)
    assert rc == 0, f"march failed: {rc}"
    iters = [x["iters"] for x in stats]
    rhos = [x["rho_obs"] for x in stats if x["rho_obs"] == x["rho_obs"]]
    log(f"[bench] timed MSC: {t_msc:.3f} s for {K} steps, mean inner {np.mean(iters):.2f}")

    # ---- roofline pass: the same K steps with every sweep launch carrying
    # its own start/stop events on the library's stream
    s = solver(eps)
    s.set_kernel_timing(True)
    s.bdf2_step(K, raise_on_fail=False)
    sec, launches, bytes_per = s.kernel_time(0)
    s.close()
    sweep_avg = sec / max(launches, 1)
    sweep_gbs = bytes_per / sweep_avg / 1e9 if launches else float("nan")
    log(f"[bench] sweep: {launches} launches, avg {sweep_avg * 1e6:.2f} us, {bytes_per / 1e6:.2f} MB -> "
        f"{sweep_gbs:.0f} GB/s")
    e = solver(eps, corrector="picard")
    e.set_kernel_timing(True)
    e.explicit_step(64)
    xsec, xl, xbytes = e.kernel_time(1)
    e.close()

    # ---- the paper's trial rule (up to cubic) on the same workload
    rc0, t_paper, u_p, st0 = march(eps, S_full, extrap=0)
    done0 = sum(1 for x in st0 if x["converged"])
    paper_rule = {"status": rc0, "steps_accepted": done0, "steps_requested": S_full, "seconds": t_paper,
                  "mean_inner": float(np.mean([x["iters"] for x in st0[:max(done0, 1)]]))}
    if rc0 == 0:
        paper_rule.update({"e_vs_stokes": rms(u_p - u_stokes), "e_eng": eng_err(u_p)})
        paper_rule.update({"gate_matched": paper_rule["e_vs_stokes"] <= 3.0 * e_exp_st,
                           "gate_1pct": paper_rule["e_eng"] <= 1e-2})
    log(f"[bench] paper trial rule: status {rc0}, {done0}/{S_full} steps, {t_paper:.3f} s")

    value = t_msc * tnu / (K * dt)
    out = {
        "metric": "wall-s per viscous time + speedup vs explicit TRT at matched err; HBM GB/s",
        "value": value,
        "unit": "s per viscous time (N^2/nu lattice steps), corrected BDF2 march",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_msc / K,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": "D2Q9" if d == 2 else "D3Q19", "N": N, "Re": cfg["Re"],
                   "nu": nu, "dt": dt, "eps": eps, "physical_steps_timed": K, "physical_steps_horizon": S_full,
                   "horizon_lattice_steps": T_full, "storage": storage, "n_min": cfg["nmin"], "K_max": 300,
                   "extrap_states": args.extrap, "initial_field": cfg["kind"]},
        "tolerance_selection": {"rule": "fastest candidate eps passing the matched and 1% gates over the full "
                                        "horizon (Sec. 4.1 protocol)", "candidates": cands, "chosen": eps},
        "full_horizon": {"msc_s": chosen["seconds"], "explicit_s": t_exp,
                         "msc_wall_s_per_viscous_time": chosen["seconds"] * tnu / T_full,
                         "explicit_wall_s_per_viscous_time": t_exp * tnu / T_full,
                         "speedup_vs_explicit": (t_exp / chosen["seconds"]) if gate else None,
                         "speedup_gate": gate, "mean_inner": chosen["mean_inner"],
                         "msc_abs_vs_stokes": chosen.get("e_vs_stokes"), "fp64_explicit_abs_vs_stokes": e_exp_st,
                         "msc_eng_err": chosen.get("e_eng"),
                         "eng_err_definition": "RMS velocity difference from the FP64 explicit endpoint over U/2"
                         if d == 3 else "RMS velocity difference from the FP64 explicit endpoint over its RMS"},
        "paper_trial_rule": paper_rule,
        "inner_iterations_timed": {"mean": float(np.mean(iters)), "max": int(max(iters)), "min": int(min(iters)),
                                   "rho_obs_median": float(np.median(rhos)) if rhos else None},
        "roofline": {"bound": "hbm", "achieved": sweep_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sweep_gbs / HBM_PEAK_GBS,
                     "traffic": counter_traffic(traffic_profile(args.workload)),
                     "kernel": "k_sweep (fused dual-time sweep: setup or lift, collision, streaming, residual, P r)",
                     "bytes_per_launch": bytes_per, "avg_launch_us": sweep_avg * 1e6, "launches": launches},
        "explicit_march": {"kernels": "k_aa_even / k_aa_odd (in-place AA march, one step each)",
                           "avg_launch_us": xsec / max(xl, 1) * 1e6, "bytes_per_launch": xbytes,
                           "achieved_GBs": xbytes / (xsec / max(xl, 1)) / 1e9 if xl else None},
    }

    # ---- beyond-cache bandwidth of the sweep kernel
    if not args.no_large:
        out["sweep_beyond_cache"] = sweep_beyond_cache(msc, stream, torch)
        sb = out["sweep_beyond_cache"]
        log(f"[bench] N=4096 sweep: explicit {sb['explicit']['achieved_GBs']:.0f} GB/s (AA "
            f"{sb['explicit_aa']['achieved_GBs']:.0f}), dts {sb['dts']['achieved_GBs']:.0f} GB/s; D3Q19 N=256 explicit "
            f"{sb['d3q19_n256_explicit']['achieved_GBs']:.0f} GB/s (AA {sb['d3q19_n256_explicit_aa']['achieved_GBs']:.0f});"
            f" device copy {sb['device_copy']['achieved_GBs']:.0f} GB/s")

    # ---- the other workloads: the precision-policy lines, the paper's 2D
    # matched-gate cells, and the differentiable march
    if not args.no_extras:
        cache = {}
        out["workloads"] = {}
        if args.workload != "tgv3d_n128_fp32":
            out["workloads"]["tgv3d_n128_fp32"] = extra_workload(msc, W, stream, torch, "tgv3d_n128_fp32", "fp32")
        out["workloads"]["rand2d_n256_fp32_dt256"] = extra_workload(msc, W, stream, torch, "rand2d_n256_fp32",
                                                                    "fp32", ref_cache=cache)
        out["workloads"]["rand2d_n256_fp32_dt64"] = extra_workload(msc, W, stream, torch, "rand2d_n256_fp32", "fp32",
                                                                   ref_cache=cache, dt=64.0)
        out["workloads"]["rand2d_n1024_fp32"] = extra_workload(msc, W, stream, torch, "rand2d_n1024_fp32", "fp32",
                                                               ref_cache=cache)
        out["workloads"]["rand2d_n1024_fp16dev"] = extra_workload(msc, W, stream, torch, "rand2d_n1024_fp32",
                                                                  "fp16dev", ref_cache=cache)
        out["workloads"]["adjoint_vort2d_n256_fp32"] = adjoint_workload(msc, W, stream, torch)
        out["tgv2d_matched_gate"] = tgv_matched_cells(msc, W, stream, torch)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    if not args.no_cpu_baseline:
        from oracle import oracle as orc  # the bench's CPU-baseline leg only

        shape = (N,) * d
        st_, bc_ = orc.initial_state(p0, u0), 0
        its = []
        nsamp = 0
        t0 = time.perf_counter()
        while nsamp < 1 or (time.perf_counter() - t0 < 12.0 and nsamp < K):
            rc_, st_, bc_, sst = orc.march_state(st_, bc_, shape, dt=dt, nsteps=1, eps=eps, nmin=cfg["nmin"],
                                                 extrap_states=args.extrap)
            its.append(sst[0]["iters"])
            nsamp += 1
        t_cpu = time.perf_counter() - t0
        per_step = t_cpu / nsamp
        out["cpu_baseline"] = {
            "value": per_step * tnu / dt, "unit": out["unit"].replace("corrected BDF2 march", "FP64 oracle march"),
            "cores": 1, "kind": "oracle",
            "sample": f"{nsamp} physical BDF step(s) (dt={dt:.3f}, eps={eps:g}) of the same N={N} workload from "
                      f"t=0, {t_cpu:.1f} s, scaled per step to one viscous time",
            "host": platform.processor() or platform.machine(), "host_nproc": os.cpu_count(),
            "mean_inner_iterations": float(np.mean(its)),
        }
        log(f"[bench] oracle: {t_cpu:.2f} s for {nsamp} steps")

    if args.calib:
        out["calibration_copy_bytes_each_way"] = calibration_copies(torch)

    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
