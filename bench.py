"""Benchmark of the explicit HOPU convection substep on one MI355X.

Main workload (the largest one-GPU configuration): the channel-like box
[0,4]x[0,1]x[0,2], x and z periodic, walls at y = 0 and 1, 96x64x48 cubes x
6 tets (1,769,472 tets), symmetric geometric y-grading to a wall aspect ratio
of 50, BDM velocity order k = 5 (168 DoFs per element, 222,759,936 DoFs), a
seeded turbulent-like field (random Fourier modes with a -5/3 spectrum, unit
RMS) interpolated by the library, HOPU projection degree l = 4, dt = 1e-4.
One step = one explicit substep u <- u - dt M^-1 r(u): the convection apply
(dual->modal transform, fused element kernel, facet-row assembly), the PCG
mass solve (warm-started, preconditioned residual 1e-13) and the update,
all on the GPU, inputs resident in HBM.

Also reported: the same substeps with FP32-MFMA and split-BF16 contractions
(rate, speed-up and the state's error against the FP64 path), the
checkpointed mixed-precision adjoint chain, apply-only rates, the roofline of
the dominant kernel, the 3D periodic Taylor-Green workload (32^3 x 6 tets,
k = 3) as a secondary line, the projection step on it, and the FP64 oracle
on the host cores as the CPU baseline.

Prints one JSON line (metric in DoF-updates/s: n_dof x steps / time).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "convection DoF-updates/s, FP64 vs mixed at ≤1e-6 rel err; % HBM/MFMA roofline"
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12

WORKLOADS = {
    5: "3d_channel_spectral_k5: [0,4]x[0,1]x[0,2], x/z periodic, walls y=0,1, 96x64x48x6=1,769,472 tets, "
       "y-grading to wall aspect 50, BDM k=5, 222,759,936 DoFs, -5/3-spectrum curl field (RMS 1), l=4, dt=1e-4, "
       "one substep per step",
    2: "3d_periodic_tg_k3: [0,2pi]^3 periodic, 32^3x6=196,608 tets, BDM k=3, 7,864,320 DoFs, "
       "Taylor-Green + N(0,1e-3^2) coefficient noise, l=2, dt=5e-4, one substep per step",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=5, choices=(2, 5),
                    help="main line: 5 (channel, k=5) or 2 (periodic Taylor-Green, k=3)")
    ap.add_argument("--adjoint-steps", type=int, default=10,
                    help="substeps of the timed mixed-precision adjoint chain (checkpoint every 5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the Taylor-Green line")
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


def mass_flops(n, d, E):
    """Algorithmic flops of one mass or preconditioner apply: the two n x n
    contractions of the sandwich (2 n^2 each per element) and the G mixing
    (d^2 multiply-adds per modal row, n/d rows per component)."""
    return 4.0 * n * n * E + 2.0 * d * d * (n // d) * E


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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(workload):
    """The FP64 oracle as it stands on the host cores, on a bounded sample:
    the same recipe on a 4 x 4 x 4 x 6 = 384-tet mesh (k and l of the
    workload); one substep = residual + mass solve (the oracle's CG) +
    update, timed once with every BLAS/OpenMP pool at its default (all host
    cores) and once with one thread.  Set-up (space, interpolation, mass
    matrix) is not timed."""
    import numpy as np
    import synth
    from oracle import space as S, operator as O
    try:
        from threadpoolctl import threadpool_limits, threadpool_info
    except Exception:  # pragma: no cover
        threadpool_limits, threadpool_info = None, lambda: []
    mesh, field, cfg = synth.make_config(workload, n_override=(4, 4, 4))
    k, l, dt = cfg["k"], cfg["l"], cfg["dt"]
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    x = sp.interpolate(field, nq1d=k + 1)
    if cfg["noise"]:
        x = x + cfg["noise"] * np.random.default_rng(6698 + workload).standard_normal(sp.n_dof)
    O.mass_matrix(sp)

    def substep(x):
        t0 = time.perf_counter()
        w = O.mass_solve(sp, O.residual(sp, x, l), method="cg")
        x = x - dt * w
        return x, time.perf_counter() - t0

    pools = [(i.get("internal_api"), i.get("num_threads")) for i in threadpool_info()]
    x, t_all = substep(x)
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            x, t_one = substep(x)
    else:
        t_one = None
    threads = max([p[1] for p in pools if p[1]] or [1])
    return {"value": sp.n_dof / t_all, "unit": "DoF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"workload recipe on 4x4x4x6=384 tets, k={k}, {sp.n_dof} DoFs; one substep (numpy einsum "
                      f"residual + CG mass solve + update) = {t_all:.2f} s with the BLAS/OpenMP pools at their "
                      f"defaults {pools}" + (f", {t_one:.2f} s with one thread" if t_one else ""),
            "value_1_thread": sp.n_dof / t_one if t_one else None,
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


class Ctx:
    """A workload on the GPU: context, initial state and timing helpers."""

    def __init__(self, workload, torch):
        import synth
        from synth.configs import coefficient_noise
        from paper_2408_06698_amd.hopu import Hopu
        self.torch = torch
        t0 = time.time()
        mesh, field, cfg = synth.make_config(workload)
        self.cfg, self.mesh = cfg, mesh
        self.k, self.l, self.dt = cfg["k"], cfg["l"], cfg["dt"]
        h = Hopu(3, self.k, mesh.elem_vid, mesh.elem_xyz)
        h.set_upwind(self.l)
        h.set_solver(rtol=1e-13, max_it=2000, check_every=2)
        self.h = h
        # the field is sampled on the GPU in chunks of points (the random
        # Fourier fields evaluate every mode at every point)
        n1d = self.k + 1

        def chunked(p):
            flat = p.reshape(-1, 3)
            out = torch.empty_like(flat)
            for s in range(0, flat.shape[0], 1 << 21):
                out[s:s + (1 << 21)] = field(flat[s:s + (1 << 21)])
            return out.reshape(p.shape)
        self.u0 = h.interpolate(chunked, n1d=n1d)
        if cfg["noise"]:
            self.u0 += torch.tensor(coefficient_noise(workload, h.n_dof, cfg["noise"]), device=self.u0.device)
        torch.cuda.synchronize()
        self.setup_s = time.time() - t0
        self.stream = torch.cuda.current_stream()
        self.sz = dict(dim=3, k=self.k, n=h.n_loc, nqv=((3 * self.k + 1) // 2) ** 3,
                       nqf=((3 * self.k + 2) // 2) ** 2)

    def ev(self):
        return self.torch.cuda.Event(enable_timing=True)

    def substeps(self, prec, steps, warm, profile=0):
        torch, h = self.torch, self.h
        if warm:
            u = self.u0.clone()
            h.substeps(u, self.dt, warm, prec)
        u = self.u0.clone()
        torch.cuda.synchronize()
        h.profile(profile)
        a, b = self.ev(), self.ev()
        a.record(self.stream)
        h.substeps(u, self.dt, steps, prec, diag=False)
        b.record(self.stream)
        torch.cuda.synchronize()
        prof = {kk: h.profile_read(kk) for kk in ("elem", "mass", "prec", "modal", "plain")} if profile else None
        h.profile(False)
        return u, a.elapsed_time(b), prof

    def apply_ms(self, prec, reps=5):
        h, r = self.h, self.h.zeros()
        h.apply(self.u0, r, prec=prec)
        self.torch.cuda.synchronize()
        a, b = self.ev(), self.ev()
        a.record(self.stream)
        for _ in range(reps):
            h.apply(self.u0, r, prec=prec)
        b.record(self.stream)
        self.torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def mnorm_rel(self, v, ref):
        torch, h = self.torch, self.h
        d = v - ref
        return float(torch.sqrt(torch.dot(d, h.mass_apply(d)) / torch.dot(ref, h.mass_apply(ref))))

    def apply_err(self, prec):
        """Residual error of a reduced-precision apply against the FP64 one
        in the M^-1 norm (the dual norm of a residual)."""
        torch, h = self.torch, self.h
        r64, rp = h.apply(self.u0), h.apply(self.u0, prec=prec)
        d = rp - r64
        wd, _ = h.mass_solve(d, rtol=1e-12)
        w64, _ = h.mass_solve(r64, rtol=1e-12)
        return float(torch.sqrt(torch.dot(d, wd) / torch.dot(r64, w64)))


def roofline(c, prof, pcg_its_per_step, steps):
    """Roofline of the kernel with the largest summed time in the timed
    region: algorithmic flops per launch / average launch duration (the
    library's HIP events on the launches themselves)."""
    E, F, n = c.mesh.n_elems, c.h.n_facets, c.h.n_loc
    tot = {kk: v[1] for kk, v in prof.items()}
    dom = max(tot, key=tot.get)
    launches, ms = prof[dom]
    avg = ms / max(launches, 1) * 1e-3
    F_apply, fv, ff = flops_model(c.sz, E, F)
    if dom == "elem":
        # the element kernel: everything of the apply but the dual->modal GEMM
        algo = F_apply - E * 2 * n * n
        name = f"k_elem<double,3,{c.k},0> (volume + HOPU facets + dual transform)"
    elif dom in ("mass", "prec"):
        algo = mass_flops(n, 3, E)
        name = f"mass kernel, k={c.k} ({'M p' if dom == 'mass' else 'preconditioner P r'} sandwich)"
    else:
        algo = 2.0 * n * n * E
        name = f"{dom} kernel"
    key = {"elem": "elem", "mass": "mass", "prec": "prec"}.get(dom, dom) + f"_k{c.k}"
    roof = {"kernel": name, "bound": "mfma", "achieved": algo / avg / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": algo / avg / PEAK_FP64, "traffic": traffic_from_profiles(key),
            "avg_launch_us": avg * 1e6, "launches_timed": launches, "flops_per_launch": algo}
    return roof, dom


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(this build targets a single MI355X)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2408_06698_amd import FP64, FP32_MFMA, BF16X2, BF16X3
    from paper_2408_06698_amd.hopu import mfma_f64_rate

    # the library's per-launch timing events go on every PROF_STRIDE-th
    # launch of each kernel kind (a dispatch with events starts a few
    # microseconds later)
    PROF_STRIDE = 4
    c = Ctx(args.workload, torch)
    h, ndof = c.h, c.h.n_dof
    print(f"# workload {args.workload}: {c.mesh.n_elems} elements, {ndof} DoFs, set-up {c.setup_s:.1f} s",
          file=sys.stderr, flush=True)
    u64, ms64, prof64 = c.substeps(FP64, args.steps, args.warmup, profile=PROF_STRIDE)
    value = ndof * args.steps / (ms64 * 1e-3)
    print(f"# fp64 substeps: {ms64 / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
    diag = h.substeps(c.u0.clone(), c.dt, 2, FP64, diag=True).cpu()
    pcg_its = float(diag[1:, 3].mean())
    roof, dom = roofline(c, prof64, pcg_its, args.steps)
    apply64 = c.apply_ms(FP64)
    F_apply, _, _ = flops_model(c.sz, c.mesh.n_elems, h.n_facets)
    out = {
        "metric": METRIC, "value": value, "unit": "DoF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms64 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded, see config.workload)",
        "config": {"workload": WORKLOADS[args.workload], "n_dof": ndof, "elements": c.mesh.n_elems,
                   "facets": h.n_facets, "wall_facets": h.n_wall, "k": c.k, "l": c.l, "dt": c.dt},
        "roofline": roof,
        "pcg_iters_per_step": pcg_its,
        "apply_ms_fp64": apply64, "apply_rate_fp64": ndof / (apply64 * 1e-3),
        "apply_frac_fp64_flops": F_apply / (apply64 * 1e-3) / PEAK_FP64,
        "apply_flops": F_apply,
        "kernel_stats_stride": PROF_STRIDE,
        "kernel_ms_sampled": {kk: v[1] for kk, v in prof64.items()},
        "kernel_launches_sampled": {kk: v[0] for kk, v in prof64.items()},
        "mfma_f64_sustained_tflops_by_waves_per_simd": {str(w): mfma_f64_rate(w) for w in (1, 2, 8)},
        "setup_s": c.setup_s,
    }
    if not args.no_mixed:
        mixed = {}
        for prec, name, dtype in ((FP32_MFMA, "fp32_mfma", "fp32-mfma"), (BF16X3, "bf16x3", "split-bf16 hi/mid/lo"),
                                  (BF16X2, "bf16x2", "split-bf16 hi/lo")):
            up, msp, _ = c.substeps(prec, args.steps, 1)
            ap = c.apply_ms(prec)
            mixed[name] = {"value": ndof * args.steps / (msp * 1e-3), "ms_per_step": msp / args.steps,
                           "speedup_substep": ms64 / msp, "apply_ms": ap, "speedup_apply": apply64 / ap,
                           "state_rel_err_vs_fp64_M_norm": c.mnorm_rel(up, u64),
                           "apply_rel_err_vs_fp64_Minv_norm": c.apply_err(prec),
                           "dtype": dtype + " contractions, FP32 accumulation in a tile, FP64 across tiles; "
                                            "FP64 state, transforms, mass solve and diagnostics"}
            del up
            print(f"# {name}: {msp / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
        out["mixed"] = mixed
    if not args.no_adjoint:
        # checkpointed reverse chain of L = 1/2 u_N.M u_N in the reduced
        # forms (and FP64), checkpoint every 5 substeps: forward with
        # checkpoints, then the segments' recomputation and the reverse steps
        n_adj = args.adjoint_steps
        uN = c.u0.clone()
        h.substeps(uN, c.dt, n_adj, FP64)
        lamN = h.mass_apply(uN)
        del uN
        adj = {"substeps": n_adj, "ckpt_every": 5}
        lam_ref = None
        for prec, name in ((FP64, "fp64"), (FP32_MFMA, "fp32_mfma"), (BF16X3, "bf16x3")):
            torch.cuda.synchronize()
            a, b = c.ev(), c.ev()
            a.record(c.stream)
            lam0 = h.substeps_vjp(c.u0, c.dt, n_adj, lamN, ckpt_every=5, prec=prec)
            b.record(c.stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            adj[name] = {"ms": ms, "dof_updates_per_s": ndof * n_adj / (ms * 1e-3)}
            if lam_ref is None:
                lam_ref = lam0
            else:
                d = lam0 - lam_ref
                wd, _ = h.mass_solve(d, rtol=1e-12)
                wr, _ = h.mass_solve(lam_ref.clone(), rtol=1e-12)
                adj[name]["rel_err_vs_fp64_Minv_norm"] = float(torch.sqrt(torch.dot(d, wd) / torch.dot(lam_ref, wr)))
            print(f"# adjoint {name}: {ms:.0f} ms", file=sys.stderr, flush=True)
        del lam_ref, lamN
        out["adjoint_chain"] = adj
    if args.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device=c.u0.device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = src.numel() * 8
        del src, dst
    del u64
    h.close()
    del c
    torch.cuda.empty_cache()
    if not args.no_secondary and args.workload != 2:
        # the 3D periodic Taylor-Green workload, FP64 and FP32-MFMA substeps
        c2 = Ctx(2, torch)
        steps2 = 50
        u2, ms2, prof2 = c2.substeps(FP64, steps2, 3, profile=PROF_STRIDE)
        roof2, _ = roofline(c2, prof2, None, steps2)
        sec = {"workload": WORKLOADS[2], "value": c2.h.n_dof * steps2 / (ms2 * 1e-3),
               "ms_per_step": ms2 / steps2, "steps": steps2, "roofline": roof2,
               "apply_ms_fp64": c2.apply_ms(FP64, 20)}
        if not args.no_mixed:
            u32, ms32, _ = c2.substeps(FP32_MFMA, steps2, 1)
            sec["fp32_mfma"] = {"ms_per_step": ms32 / steps2, "speedup_substep": ms2 / ms32,
                                "state_rel_err_vs_fp64_M_norm": c2.mnorm_rel(u32, u2)}
        if not args.no_projection:
            # projection step (section 2.3, eq. (MCS_step2)) of the state
            # after the substeps, whose divergence the convection broke
            un = c2.h.zeros()
            c2.h.project(u2, un, rtol=1e-13)        # set-up (A^-1) and warm-up
            torch.cuda.synchronize()
            a, b = c2.ev(), c2.ev()
            a.record(c2.stream)
            _, its = c2.h.project(u2, un, rtol=1e-13)
            b.record(c2.stream)
            torch.cuda.synchronize()
            sec["projection"] = {"ms": a.elapsed_time(b), "cg_iters": its, "rtol": 1e-13,
                                 "div_l2_before": c2.h.diagnostics(u2)[1], "div_l2_after": c2.h.diagnostics(un)[1]}
        out["secondary"] = sec
        c2.h.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
