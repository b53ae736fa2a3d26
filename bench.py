"""Benchmark of the explicit HOPU convection substep on one MI355X.

Workload: 3D periodic unit cube [0, 2 pi]^3, 32^3 cubes x 6 tets
(196,608 tets), BDM velocity order k = 3 (7,864,320 DoFs), 3D Taylor-Green
field interpolated by the library plus seeded N(0, 1e-3^2) coefficient
noise, HOPU projection degree l = 2, dt = 5e-4.  One step = one explicit
substep u <- u - dt M^-1 r(u): the convection apply (dual->modal transform,
fused element kernel, facet-row assembly), the PCG mass solve (warm-started,
preconditioned residual 1e-13) and the update, all on the GPU.

Prints one JSON line (metric in DoF-updates/s: n_dof x steps / time).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "convection DoF-updates/s, FP64 vs mixed at ≤1e-6 rel err; % HBM/MFMA roofline"
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after the run, copy a 1 GiB device buffer (reference for HBM counters)")
    return ap.parse_args()


def flops_model(sz, E, F):
    """Algorithmic FP64 flops of one convection apply (modal formulation,
    contract quadrature): per element 4n^2 + 2 nq n (1 + d) + 30 nq, per
    interior facet 8 nqf n + 8 d nqf dimP^{k-1}(F) + 40 nqf."""
    d, k, n, nq, nqf = sz["dim"], sz["k"], sz["n"], sz["nqv"], sz["nqf"]
    dimPf = k * (k + 1) // 2 if d == 3 else k  # dim P^{k-1} on a facet
    fv = 4 * n * n + 2 * nq * n * (1 + d) + 30 * nq
    ff = 8 * nqf * n + 8 * d * nqf * dimPf + 40 * nqf
    return E * fv + F * ff, fv, ff


def traffic_from_profiles(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    src = os.path.join(ROOT, "paper_2408_06698_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    text = open(src).read()
    body = text[text.index("namespace hopu {"):text.index("// " + "-" * 66 + " launchers")]
    sha = hashlib.sha256(body.encode()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            vals[a.strip()] = b.strip()
    if vals.get("kernels_sha") != sha or kernel_key + "_bytes_per_launch" not in vals:
        return None
    return float(vals[kernel_key + "_bytes_per_launch"])


def cpu_baseline():
    """The FP64 oracle as it stands, on a bounded sample: the same recipe on
    5^3 x 6 = 750 tets (30,000 DoFs), one substep = residual + sparse-LU mass
    solve + update; 1 warm-up (includes the LU factorisation), median of 5
    (about 15 s of single-threaded work on an EPYC host)."""
    import numpy as np
    import synth
    from oracle import space as S, operator as O
    import contextlib
    try:
        # one thread for every BLAS/OpenMP pool, so that `cores` is what ran
        from threadpoolctl import threadpool_limits, threadpool_info
        limit = threadpool_limits(limits=1)
    except Exception:
        limit, threadpool_info = contextlib.nullcontext(), lambda: []
    with limit:
        blas = [(i.get("internal_api"), i.get("num_threads")) for i in threadpool_info()]
        mesh, field, cfg = synth.make_config(2, n_override=(5, 5, 5))
        sp = S.Space(mesh.elem_vid, mesh.elem_xyz, 3)
        x = sp.interpolate(field, nq1d=5)
        x = x + 1e-3 * np.random.default_rng(6698 + 2).standard_normal(sp.n_dof)
        O.substep(sp, x, 5e-4, 2)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            x = O.substep(sp, x, 5e-4, 2)
            ts.append(time.perf_counter() - t0)
    t = sorted(ts)[2]
    return {"value": sp.n_dof / t, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"C2 recipe on 5^3x6=750 tets, k=3, {sp.n_dof} DoFs; one substep "
                      f"(numpy einsum + SuperLU, single-threaded; BLAS pools {blas}); median of 5 "
                      f"= {t:.2f} s per substep",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    from synth.configs import coefficient_noise
    from paper_2408_06698_amd.hopu import Hopu
    from paper_2408_06698_amd import FP64, FP32_MFMA, BF16X2, BF16X3

    mesh, field, cfg = synth.make_config(2)
    k, l, dt = cfg["k"], cfg["l"], cfg["dt"]
    h = Hopu(3, k, mesh.elem_vid, mesh.elem_xyz)
    h.set_upwind(l)
    h.set_solver(rtol=1e-13, max_it=1000, check_every=2)
    u0 = h.interpolate(field, n1d=k + 2)
    u0 += torch.tensor(coefficient_noise(2, h.n_dof, cfg["noise"]), device=u0.device)
    ndof = h.n_dof
    sz = dict(dim=3, k=k, n=h.n_loc, nqv=((3 * k + 1) // 2) ** 3, nqf=((3 * k + 2) // 2) ** 2)
    stream = torch.cuda.current_stream()

    # the library's per-launch timing events go on every PROF_STRIDE-th launch
    # of each kernel kind (a dispatch with events is a few microseconds
    # slower; every launch instrumented would cost the timed run 3%)
    PROF_STRIDE = 8

    def run(prec, steps, warm, profile=False):
        u = u0.clone()
        if warm:
            h.substeps(u, dt, warm, prec)
        u = u0.clone()
        torch.cuda.synchronize()
        h.profile(PROF_STRIDE if profile else 0)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        h.substeps(u, dt, steps, prec, diag=False)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        prof = {kk: h.profile_read(kk) for kk in ("elem", "mass", "prec", "modal", "plain")} if profile else None
        h.profile(False)
        return u, ms, prof

    u64, ms64, prof64 = run(FP64, args.steps, args.warmup, profile=True)
    value = ndof * args.steps / (ms64 * 1e-3)
    # PCG iterations per substep, from an untimed run with diagnostics
    ud = u0.clone()
    diag = h.substeps(ud, dt, args.steps, FP64, diag=True).cpu()
    pcg_its = float(diag[1:, 3].mean())

    # apply-only timings (FP64 and FP32 MFMA), 20 launches each
    def apply_ms(prec, reps=20):
        r = h.zeros()
        h.apply(u0, r, prec=prec)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            h.apply(u0, r, prec=prec)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps
    apply64 = apply_ms(FP64)
    apply32 = apply_ms(FP32_MFMA)
    apply_bf = {p: apply_ms(p) for p in (BF16X2, BF16X3)}

    # residual error of each reduced-precision form against the FP64 apply,
    # in the M^-1 norm (the dual norm of a residual)
    def apply_err(prec):
        r64, rp = h.apply(u0, prec=FP64), h.apply(u0, prec=prec)
        d = rp - r64
        wd, _ = h.mass_solve(d, rtol=1e-12)
        w64, _ = h.mass_solve(r64, rtol=1e-12)
        return float(torch.sqrt(torch.dot(d, wd) / torch.dot(r64, w64)))

    # dominant kernel over the timed region
    tot = {kk: v[1] for kk, v in prof64.items()}
    dom = max(tot, key=tot.get)
    E, F = mesh.n_elems, h.n_facets
    F_apply, fv, ff = flops_model(sz, E, F)
    n = h.n_loc
    if dom == "elem":
        launches, ms = prof64["elem"]
        avg = ms / max(launches, 1) * 1e-3
        # element kernel: everything of the apply except the dual->modal GEMM (2n^2) and assembly
        algo = F_apply - E * 2 * n * n
        roof = {"kernel": "k_elem (volume + HOPU facet + dual transform)", "bound": "mfma",
                "achieved": algo / avg / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s"}
    else:
        launches, ms = prof64[dom]
        avg = ms / max(launches, 1) * 1e-3
        algo = 4.0 * n * n * E + 2.0 * 9 * (n // 3) * E  # two n x n contractions + G mixing
        roof = {"kernel": f"k_mass ({'mass apply' if dom == 'mass' else 'preconditioner'} sandwich)",
                "bound": "mfma", "achieved": algo / avg / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # what this GPU sustains for register-only FP64 MFMA chains, by waves per
    # SIMD (the FP64 kernels run one or two)
    from paper_2408_06698_amd.hopu import mfma_f64_rate
    sustained = {str(w): mfma_f64_rate(w) for w in (1, 2, 8)}
    roof["avg_launch_us"] = avg * 1e6
    roof["launches"] = launches
    roof["launches_timed_every"] = PROF_STRIDE
    tr = traffic_from_profiles(dom)
    roof["traffic"] = tr
    out = {
        "metric": METRIC, "value": value, "unit": "DoF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms64 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded Taylor-Green + noise)",
        "config": {"workload": "3d_periodic_tg_k3: [0,2pi]^3 periodic, 32^3x6=196608 tets, BDM k=3, "
                               "7,864,320 DoFs, TG + N(0,1e-3^2) noise, l=2, dt=5e-4, one substep per step",
                   "n_dof": ndof, "elements": E, "facets": F},
        "roofline": roof,
        "mfma_f64_sustained_tflops_by_waves_per_simd": sustained,
        "apply_ms_fp64": apply64, "apply_ms_fp32_mfma": apply32,
        "apply_rate_fp64": ndof / (apply64 * 1e-3), "apply_rate_fp32_mfma": ndof / (apply32 * 1e-3),
        "apply_frac_fp64_flops": F_apply / (apply64 * 1e-3) / PEAK_FP64,
        "pcg_iters_per_step": pcg_its,
        "kernel_stats_stride": PROF_STRIDE,
        "kernel_ms_sampled": {kk: v[1] for kk, v in prof64.items()},
        "kernel_launches_sampled": {kk: v[0] for kk, v in prof64.items()},
    }
    if not args.no_projection:
        # projection step (paper section 2.3, eq. (MCS_step2)) of the state
        # after the timed substeps, whose divergence the convection broke
        un = h.zeros()
        h.project(u64, un, rtol=1e-13)            # set-up (A^-1) and warm-up
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _, its = h.project(u64, un, rtol=1e-13)
        b.record(stream)
        torch.cuda.synchronize()
        _, div0, _ = h.diagnostics(u64)
        _, div1, _ = h.diagnostics(un)
        out_proj = {"ms": a.elapsed_time(b), "cg_iters": its, "rtol": 1e-13,
                    "div_l2_before": div0, "div_l2_after": div1,
                    "note": "condensed facet-multiplier system, unpreconditioned CG"}
    if not args.no_mixed:
        u32, ms32, prof32 = run(FP32_MFMA, args.steps, 1)
        d = u32 - u64
        err = float(torch.sqrt(torch.dot(d, h.mass_apply(d)) / torch.dot(u64, h.mass_apply(u64))))
        out["mixed"] = {"value": ndof * args.steps / (ms32 * 1e-3), "ms_per_step": ms32 / args.steps,
                        "rel_err_vs_fp64_M_norm": err, "dtype": "fp32-mfma contractions, f64 state/PCG",
                        "speedup_substep": ms64 / ms32, "speedup_apply": apply64 / apply32}
        # split-BF16 forms (hi/lo, hi/mid/lo) of the same contractions
        for prec, name in ((BF16X2, "bf16x2"), (BF16X3, "bf16x3")):
            ub, msb, _ = run(prec, args.steps, 1)
            d = ub - u64
            errb = float(torch.sqrt(torch.dot(d, h.mass_apply(d)) / torch.dot(u64, h.mass_apply(u64))))
            out["mixed_" + name] = {
                "value": ndof * args.steps / (msb * 1e-3), "ms_per_step": msb / args.steps,
                "rel_err_vs_fp64_M_norm": errb,
                "dtype": f"split-bf16 ({'hi/lo' if prec == BF16X2 else 'hi/mid/lo'}) mfma contractions, "
                         "f64 state/PCG",
                "speedup_substep": ms64 / msb, "apply_ms": apply_bf[prec], "speedup_apply": apply64 / apply_bf[prec]}
        out["apply_rel_err_vs_fp64_Minv_norm"] = {"fp32_mfma": apply_err(FP32_MFMA), "bf16x2": apply_err(BF16X2),
                                                  "bf16x3": apply_err(BF16X3)}
    if not args.no_projection:
        out["projection"] = out_proj
    if args.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device=u0.device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
