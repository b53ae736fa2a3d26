"""Benchmark of the explicit HOPU convection substep on one MI355X.

Main workload (the largest one-GPU configuration): the channel-like box
[0,4]x[0,1]x[0,2], x and z periodic, walls at y = 0 and 1, 96x64x48 cubes x
6 tets (1,769,472 tets), symmetric geometric y-grading to a wall aspect ratio
of 50, BDM velocity order k = 5 (168 DoFs per element, 222,759,936 DoFs), a
seeded turbulent-like field (random Fourier modes with a -5/3 spectrum, unit
RMS) interpolated by the library, HOPU projection degree l = 4, dt = 1e-4.
One step = one explicit substep u <- u - dt M^-1 r(u): the convection apply
(dual->modal transform, fused element kernel, facet-row assembly), the PCG
mass solve (preconditioned residual 1e-13, initial guess extrapolated from
the previous substeps' solutions) and the update, all on the GPU, inputs
resident in HBM.  The W warm-up substeps and the K timed ones are one
trajectory: the timed substeps continue the warm-up's (hopu_set_warm_start),
as in a long run; the first, cold substep's PCG count is reported apart.

Also reported: the PCG iteration counts (cold and warm), one substep from
u0 with FP32-MFMA and split-BF16 contractions (rate, speed-up, the state's
error against the FP64 substep and the apply's error against the FP64
apply), the checkpointed FP64 and hi/mid/lo adjoint of one substep,
apply-only rates, the roofline of the dominant kernel, the 3D periodic
Taylor-Green workload (32^3 x 6 tets, k = 3) as a secondary line with the
projection step and the implicit Stokes step (element Schur complements,
PCG with the element-wise BDDC; --only-stokes runs that section alone), and
the FP64 oracle on the host cores as the CPU baseline.  The sections after the timed substeps and the CPU baseline run
only while they fit in --budget-s; a skipped one is named under "skipped".

Prints one JSON line (metric in DoF-updates/s: n_dof x steps / time).
"""
import argparse
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
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", type=int, default=5, choices=(2, 5),
                    help="main line: 5 (channel, k=5) or 2 (periodic Taylor-Green, k=3)")
    ap.add_argument("--adjoint-steps", type=int, default=1,
                    help="substeps of the timed adjoint chain (FP64 and hi/mid/lo)")
    ap.add_argument("--adjoint-ckpt", type=int, default=1, help="checkpoint interval of the adjoint chain")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget of the whole run: the sections after the timed substeps and the "
                         "CPU baseline (mixed forms, adjoint, secondary workload) run only while they fit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the Taylor-Green line")
    ap.add_argument("--no-projection", action="store_true")
    ap.add_argument("--no-stokes", action="store_true", help="skip the implicit Stokes step section")
    ap.add_argument("--only-stokes", action="store_true",
                    help="run only the implicit Stokes step section and print it as the JSON line")
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


def traffic_from_profiles(kernel_key, source="kernels.hip"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summaries (profiles/*traffic*.txt), if one was taken on the current
    kernel source; else None."""
    from paper_2408_06698_amd.rocpd_summary import source_sha
    sha = source_sha(open(os.path.join(ROOT, "paper_2408_06698_amd", "csrc", source)).read())
    pdir = os.path.join(ROOT, "profiles")
    for fn in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        if "traffic" not in fn or not fn.endswith(".txt"):
            continue
        vals = {}
        for line in open(os.path.join(pdir, fn)):
            if "=" in line and not line.startswith("#"):
                a, b = line.split("=", 1)
                vals[a.strip()] = b.strip()
        if vals.get("kernels_sha") == sha and kernel_key + "_bytes_per_launch" in vals:
            return float(vals[kernel_key + "_bytes_per_launch"])
    return None


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
    the same recipe on a 3 x 3 x 3 x 6 = 162-tet mesh (k and l of the
    workload).  One substep = the oracle's residual + mass solve + update,
    timed once with every BLAS/OpenMP pool at its default (all host cores)
    and once with one thread.  Set-up (space, interpolation, mass matrix and
    its sparse LU factorisation) is not timed, as the GPU's is not."""
    import numpy as np
    import synth
    from oracle import space as S, operator as O
    try:
        from threadpoolctl import threadpool_limits, threadpool_info
    except Exception:  # pragma: no cover
        threadpool_limits, threadpool_info = None, lambda: []
    mesh, field, cfg = synth.make_config(workload, n_override=(3, 3, 3))
    k, l, dt = cfg["k"], cfg["l"], cfg["dt"]
    t_set = time.perf_counter()
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    x = sp.interpolate(field, nq1d=k + 1)
    if cfg["noise"]:
        x = x + cfg["noise"] * np.random.default_rng(6698 + workload).standard_normal(sp.n_dof)
    O.mass_solve(sp, np.zeros(sp.n_dof))   # assembles M and factors it
    t_set = time.perf_counter() - t_set

    def substep(x):
        t0 = time.perf_counter()
        w = O.mass_solve(sp, O.residual(sp, x, l))
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
            "sample": f"workload recipe on 3x3x3x6=162 tets, k={k}, {sp.n_dof} DoFs; one substep (numpy einsum "
                      f"residual + sparse-LU mass solve + update) = {t_all:.2f} s with the BLAS/OpenMP pools at "
                      f"their defaults {pools}" + (f", {t_one:.2f} s with one thread" if t_one else "") +
                      f"; untimed set-up (space, interpolation, mass matrix, LU) {t_set:.1f} s",
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
        # convergence checked every 16 iterations (a C5 solve takes
        # hundreds; iterations queued past convergence return at once)
        h.set_solver(rtol=1e-13, max_it=3000, check_every=16)
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

    def timed(self, fn):
        """fn() between two events on the stream; (result, ms)."""
        torch = self.torch
        torch.cuda.synchronize()
        a, b = self.ev(), self.ev()
        a.record(self.stream)
        out = fn()
        b.record(self.stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b)

    def apply_ms(self, prec, reps=5):
        h, r = self.h, self.h.zeros()
        h.apply(self.u0, r, prec=prec)

        def run():
            for _ in range(reps):
                h.apply(self.u0, r, prec=prec)
        return self.timed(run)[1] / reps

    def mnorm_rel(self, v, ref):
        torch, h = self.torch, self.h
        d = v - ref
        return float(torch.sqrt(torch.dot(d, h.mass_apply(d)) / torch.dot(ref, h.mass_apply(ref))))

    def minv_norm2(self, d):
        """d.M^-1 d (a residual's squared dual norm).  CG's d.w_i approaches
        d.M^-1 d from below with error ||w - w_i||_M^2, so a solve to a
        relative residual of 1e-4 gives it to far better than the digits
        reported."""
        w, _ = self.h.mass_solve(d, rtol=1e-4, max_it=3000)
        return float(self.torch.dot(d, w))


STOKES_NU = 1.0 / 1600.0   # Taylor-Green at Re = 1600 on [0, 2 pi]^3
STOKES_STEPS = 3


def stokes_section(torch, log):
    """The splitting step of section 2.3 on the 3D periodic Taylor-Green
    workload (32^3 x 6 tets, k = 3, dt = 5e-4, nu = 1/1600): the implicit
    Stokes step (eq. (MCS_step1), convection of u^n on the right-hand side)
    and the projection (eq. (MCS_step2)) of its u*, which gives the next
    state.  Set-up of the element Schur complements and their inverses
    (timed), one warm-up step from u0 with a zero PCG guess, then
    STOKES_STEPS timed steps of the trajectory, each Stokes PCG started from
    [u^n; u^ of the previous step] and run to 1e-10 of the right-hand side's
    C^-1 norm.  The element products read the packed upper triangle of S_T
    or S_T^-1 once per launch, so their roofline is HBM: bytes =
    E nx (nx + 1)/2 8 per launch (the matrix; vectors add < 1%) over the
    launch's average duration from the library's events."""
    import synth
    from paper_2408_06698_amd.hopu import Hopu
    mesh, field, cfg = synth.make_config(2)
    h = Hopu(3, cfg["k"], mesh.elem_vid, mesh.elem_xyz)
    h.set_upwind(cfg["l"])
    u = h.interpolate(field, n1d=cfg["k"] + 1)
    nt, nh, nx = h.stokes_sizes()
    torch.cuda.synchronize()
    t0 = time.time()
    h.stokes_setup(STOKES_NU, cfg["dt"])
    setup_s = time.time() - t0
    log(f"stokes set-up {setup_s:.1f} s ({mesh.n_elems} elements, {nx} unknowns each)")
    x, its0 = h.stokes_step(u, with_convection=True, rtol=1e-10)
    u0 = h.project(x[:h.n_dof], rtol=1e-13)[0]
    x0 = x.clone()

    def trajectory(fp32):
        """STOKES_STEPS timed splitting steps from u0 (PCG guess [u^n; u^ of
        the previous step], the first from the warm-up step's solution)."""
        u, x = u0.clone(), x0.clone()
        h.profile(1)
        its, pits, ms_st, ms_pr, div = [], [], [], [], []
        for _ in range(STOKES_STEPS):
            x[:h.n_dof].copy_(u)
            torch.cuda.synchronize()
            t1 = time.time()
            its.append(h.stokes_step(u, with_convection=True, out=x, rtol=1e-10, guess=True)[1])
            t2 = time.time()
            div_star = h.diagnostics(x[:h.n_dof].contiguous())[1]
            torch.cuda.synchronize()
            t3 = time.time()
            u, pit = h.project(x[:h.n_dof], rtol=1e-13)
            torch.cuda.synchronize()
            t4 = time.time()
            pits.append(pit)
            ms_st.append((t2 - t1) * 1e3)
            ms_pr.append((t4 - t3) * 1e3)
            div.append((div_star, h.diagnostics(u)[1]))
        prof = {kk: h.profile_read(kk) for kk in ("stokes_S", "stokes_C")}
        h.profile(False)
        return u, its, pits, ms_st, ms_pr, div, prof

    u64, its, pits, ms_st, ms_pr, div, prof = trajectory(False)
    (nS, msS), (nC, msC) = prof["stokes_S"], prof["stokes_C"]
    ms = sum(ms_st) / len(ms_st)
    # the packed upper triangle of S_T^-1 (padded to 8 entries per element)
    packed = mesh.n_elems * ((nx * (nx + 1) // 2 + 7) // 8 * 8)
    mat_bytes = packed * 8
    avg_S, avg_C = msS / max(nS, 1), msC / max(nC, 1)
    ach = mat_bytes / (avg_C * 1e-3)
    # the same trajectory with S_T^-1 in FP32
    t0 = time.time()
    h.stokes_setup(STOKES_NU, cfg["dt"], fp32_precond=True)
    setup32 = time.time() - t0
    u32, its32, _, ms_st32, _, _, prof32 = trajectory(True)
    d = u32 - u64
    rel32 = float(torch.sqrt(torch.dot(d, h.mass_apply(d)) / torch.dot(u64, h.mass_apply(u64))))
    avg_C32 = prof32["stokes_C"][1] / max(prof32["stokes_C"][0], 1)
    ms32 = sum(ms_st32) / len(ms_st32)
    out = {
        "workload": WORKLOADS[2].replace("one substep per step", "one splitting step (implicit Stokes step + "
                                         "projection) per step") + f", nu={STOKES_NU}",
        "n_unknowns": nt, "n_uhat": nh, "unknowns_per_element": nx,
        "setup_s": setup_s, "pcg_iterations": its, "pcg_iterations_first_zero_guess": its0, "rtol": 1e-10,
        "ms_per_stokes_step": ms, "ms_per_pcg_iteration": ms / max(1.0, sum(its) / len(its)),
        "stokes_dof_updates_per_s": h.n_dof / (ms * 1e-3),
        "projection_ms": sum(ms_pr) / len(ms_pr), "projection_cg_iterations": pits,
        "ms_per_splitting_step": (sum(ms_st) + sum(ms_pr)) / len(ms_st),
        "div_l2_before_after_projection": div,
        "kernel_avg_ms": {"stokes_S": avg_S, "stokes_C": avg_C},
        "kernel_launches": {"stokes_S": nS, "stokes_C": nC},
        "roofline": {"kernel": "k_stokes_gemv (S_T^-1, the preconditioner)", "bound": "hbm",
                     "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": ach / PEAK_HBM, "traffic": traffic_from_profiles("stokes_gemv", "stokes_kernels.hip"),
                     "algorithmic_bytes_per_launch": mat_bytes},
        "fp32_preconditioner": {
            "setup_s": setup32, "pcg_iterations": its32, "ms_per_stokes_step": ms32,
            "speedup_stokes_step": ms / ms32, "kernel_avg_ms_stokes_C": avg_C32,
            "hbm_frac_stokes_C": packed * 4 / (avg_C32 * 1e-3) / PEAK_HBM,
            "state_rel_err_vs_fp64_M_norm": rel32,
            "protocol": f"S_T^-1 in FP32, S and the vectors FP64; the same {STOKES_STEPS}-step trajectory from "
                        "the same state, final states compared"},
        "timing": "host clock around each hopu_stokes_step and hopu_project call (both synchronise); kernel "
                  "averages from the library's HIP events on every element-product launch",
    }
    out["cpu_oracle"] = stokes_cpu_oracle()
    log(f"stokes: {ms:.1f} ms per step, {its} PCG iterations, element product {avg_S:.2f} / {avg_C:.2f} ms; "
        f"projection {out['projection_ms']:.1f} ms; FP32 preconditioner {ms32:.1f} ms per step, {its32}")
    h.close()
    return out


def secondary_cpu_oracle(what):
    """The oracle as it stands on a 3^3 x 6 = 162-tet sample of the 3D
    Taylor-Green recipe (k = 3), on the host: the projection step (its
    hybrid-mixed system assembled and solved by sparse LU) of the state after
    one substep, or 10 substeps with the adaptive order re-selected before
    the first (residuals in numpy, mass solves by a factored sparse LU)."""
    import numpy as np
    import synth
    from oracle import operator as O, projection as P
    from oracle.space import Space
    mesh, field, cfg = synth.make_config(2, n_override=(3, 3, 3))
    sp = Space(mesh.elem_vid, mesh.elem_xyz, cfg["k"])
    x = sp.interpolate(field) + 1e-3 * np.random.default_rng(0).standard_normal(sp.n_dof)
    O.mass_solve(sp, x)  # factor M (untimed, as the GPU's set-up)
    from threadpoolctl import threadpool_limits
    if what == "projection":
        xs = O.substep(sp, x, cfg["dt"], cfg["l"])
        with threadpool_limits(1):
            t0 = time.perf_counter()
            P.project(sp, xs)
            t = time.perf_counter() - t0
        return {"value_ms": t * 1e3, "kind": "oracle", "cores": 1,
                "sample": f"3^3 x 6 = 162 tets ({sp.n_dof} DoFs): one projection = {t:.2f} s, one thread"}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.substeps_adaptive(sp, x, cfg["dt"], 10, [0.1, 0.2, 0.3, 0.4], every=10)
        t = time.perf_counter() - t0
    return {"value": sp.n_dof * 10 / t, "unit": "DoF-updates/s", "kind": "oracle", "cores": 1,
            "sample": f"3^3 x 6 = 162 tets ({sp.n_dof} DoFs): 10 adaptive substeps = {t:.2f} s, one thread"}


def stokes_cpu_oracle():
    """The oracle's implicit Stokes step as it stands, timed on the host: the
    same recipe (3D Taylor-Green, k = 3, nu = 1/1600, dt = 5e-4, convection
    with l = 2) on 3^3 x 6 = 162 tets; element blocks (the stress space's
    basis and the forms), the condensed system and its sparse direct solve,
    all timed (the oracle forms them per step)."""
    import numpy as np
    import synth
    from oracle import operator as O, stokes as OST
    from oracle.space import Space
    mesh, field, cfg = synth.make_config(2, n_override=(3, 3, 3))
    sp = Space(mesh.elem_vid, mesh.elem_xyz, cfg["k"])
    un = sp.interpolate(field)
    r = O.residual(sp, un, cfg["l"])
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        OST.step1_condensed(sp, un, STOKES_NU, cfg["dt"], r)
        t = time.perf_counter() - t0
    return {"value": sp.n_dof / t, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the recipe on 3^3 x 6 = 162 tets ({sp.n_dof} velocity DoFs): one Stokes step by the "
                      f"oracle's condensed route = {t:.1f} s, one thread (element blocks, condensed system, sparse LU)",
            "seconds": t}


def small_latency(torch):
    """Launch-bound latency on the 2D periodic Taylor-Green workload (16x16x2
    = 512 triangles, k = 2, 3,840 DoFs): one convection apply (averaged over
    200 back to back) and one substep (50 substeps in one call, so the PCG's
    host checks are included)."""
    import numpy as np
    import synth
    from synth.configs import coefficient_noise
    from paper_2408_06698_amd.hopu import Hopu
    mesh, field, cfg = synth.make_config(1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        h = Hopu(2, cfg["k"], mesh.elem_vid, mesh.elem_xyz, stream=st)
        h.set_upwind(cfg["l"])
        h.set_solver(rtol=1e-13, max_it=500, check_every=4)
        u = h.interpolate(field, n1d=cfg["k"] + 1)
        u += torch.tensor(coefficient_noise(1, h.n_dof, cfg["noise"]), device=u.device)
        r = h.zeros()
        h.apply(u, r)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    with torch.cuda.stream(st):
        ev[0].record(st)
        for _ in range(200):
            h.apply(u, r)
        ev[1].record(st)
        h.substeps(u, cfg["dt"], 5)
        torch.cuda.synchronize()
        ev[2].record(st)
        h.substeps(u, cfg["dt"], 50)
        ev[3].record(st)
    torch.cuda.synchronize()
    # the apply captured into a HIP graph (10 applies per graph, 20 replays)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        for _ in range(10):
            h.apply(u, r)
    torch.cuda.synchronize()
    ev[4].record()
    for _ in range(20):
        g.replay()
    ev[5].record()
    torch.cuda.synchronize()
    out = {"workload": "2d_periodic_tg_k2: [0,1]^2 periodic, 16x16x2=512 triangles, BDM k=2, "
                       f"{h.n_dof} DoFs, l=1, dt=1e-3",
           "apply_us": ev[0].elapsed_time(ev[1]) / 200 * 1e3,
           "apply_us_hip_graph": ev[4].elapsed_time(ev[5]) / 200 * 1e3,
           "substep_us": ev[2].elapsed_time(ev[3]) / 50 * 1e3,
           "note": "launch-bound: each apply is 3 launches, each PCG iteration 4 plus a host check every 4; "
                   "the graph replays 10 captured applies per launch"}
    del g
    h.close()
    return out


def roofline(c, prof):
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
        kern = "k_mass_tiled" if c.k >= 4 else "k_mass_lds"
        name = f"{kern}, k={c.k} ({'M p' if dom == 'mass' else 'preconditioner P r'} sandwich)"
    else:
        algo = 2.0 * n * n * E
        name = f"{dom} kernel"
    key = f"{dom}_k{c.k}"
    roof = {"kernel": name, "bound": "mfma", "achieved": algo / avg / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": algo / avg / PEAK_FP64, "traffic": traffic_from_profiles(key),
            "traffic_key": key, "avg_launch_us": avg * 1e6, "launches_timed": launches, "flops_per_launch": algo}
    return roof, dom


def main():
    t_start = time.time()
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the library and its benchmark target a single MI355X)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2408_06698_amd import FP64, FP32_MFMA, BF16X2, BF16X3
    from paper_2408_06698_amd.hopu import mfma_f64_rate

    def log(msg):
        print(f"# [{time.time() - t_start:6.1f} s] {msg}", file=sys.stderr, flush=True)

    if args.only_stokes:
        line = {"stokes_step": stokes_section(torch, log)}
        if args.copy_calib:
            src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            line["copy_calib_bytes"] = src.numel() * 8
        line["wall_s"] = time.time() - t_start
        print(json.dumps(line))
        return

    # the library's per-launch timing events go on every PROF_STRIDE-th
    # launch of each kernel kind (a dispatch with events starts a few
    # microseconds later)
    PROF_STRIDE = 4
    c = Ctx(args.workload, torch)
    h, ndof = c.h, c.h.n_dof
    log(f"workload {args.workload}: {c.mesh.n_elems} elements, {ndof} DoFs, set-up {c.setup_s:.1f} s")

    # warm-up: the first substep from u0 cold (its state and time are also
    # the FP64 reference of the mixed forms), then the rest continuing it
    W = max(args.warmup, 1)
    u = c.u0.clone()
    h.set_warm_start(False)
    diag1, ms_first = c.timed(lambda: h.substeps(u, c.dt, 1, FP64, diag=True))
    diag1 = diag1.cpu()
    u1 = u.clone()
    h.set_warm_start(True)
    diagw = h.substeps(u, c.dt, W - 1, FP64, diag=True).cpu() if W > 1 else None
    log(f"warm-up: {W} substeps, first (cold) {ms_first:.0f} ms, {int(diag1[1, 3])} PCG iterations")
    # timed: K substeps continuing the warm-up's trajectory and extrapolation
    h.profile(PROF_STRIDE)
    _, ms64 = c.timed(lambda: h.substeps(u, c.dt, args.steps, FP64, diag=False))
    prof64 = {kk: h.profile_read(kk) for kk in ("elem", "mass", "prec", "modal", "plain")}
    h.profile(False)
    t_sub = ms64 / args.steps * 1e-3
    value = ndof * args.steps / (ms64 * 1e-3)
    log(f"fp64 substeps: {ms64 / args.steps:.1f} ms/step")
    roof, dom = roofline(c, prof64)
    apply64 = c.apply_ms(FP64)
    F_apply, _, _ = flops_model(c.sz, c.mesh.n_elems, h.n_facets)
    pcg = {"cold_first_substep": float(diag1[1, 3]), "rtol": 1e-13,
           "preconditioner": "element-wise BDDC without primal constraints (local mass inverses, plain average)"}
    if diagw is not None:
        pcg["warm_mean_warmup_substeps"] = float(diagw[1:, 3].mean())
    # launches of the preconditioner kernel in the timed region (every
    # PROF_STRIDE-th is timed; each solve adds two set-up launches)
    pcg["timed_mean_estimate"] = prof64["prec"][0] * PROF_STRIDE / args.steps - 2
    out = {
        "metric": METRIC, "value": value, "unit": "DoF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms64 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded, see config.workload)",
        "config": {"workload": WORKLOADS[args.workload], "n_dof": ndof, "elements": c.mesh.n_elems,
                   "facets": h.n_facets, "wall_facets": h.n_wall, "k": c.k, "l": c.l, "dt": c.dt,
                   "warmup_substeps_run": W},
        "roofline": roof,
        "pcg_iterations_per_substep": pcg,
        "apply_ms_fp64": apply64, "apply_rate_fp64": ndof / (apply64 * 1e-3),
        "apply_frac_fp64_flops": F_apply / (apply64 * 1e-3) / PEAK_FP64,
        "apply_flops": F_apply,
        "kernel_stats_stride": PROF_STRIDE,
        "kernel_ms_sampled": {kk: v[1] for kk, v in prof64.items()},
        "kernel_launches_sampled": {kk: v[0] for kk, v in prof64.items()},
        "mfma_f64_sustained_tflops_by_waves_per_simd": {str(w): mfma_f64_rate(w) for w in (1, 2, 8)},
        "setup_s": c.setup_s,
        "skipped": {},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
        log("cpu baseline done")

    def fits(name, est_s):
        """Whether a further section of about est_s seconds keeps the whole
        run inside --budget-s; records the skip otherwise."""
        left = args.budget_s - (time.time() - t_start)
        if est_s <= left - 30:
            return True
        out["skipped"][name] = f"time budget: needs about {est_s:.0f} s, {left:.0f} s of {args.budget_s:.0f} s left"
        log(f"skipping {name}: {out['skipped'][name]}")
        return False

    # the mixed forms: each one cold substep from u0, against the FP64
    # state after the same substep (the warm-up's first); apply error in the
    # M^-1 norm against the FP64 apply
    if not args.no_mixed:
        mixed = {"protocol": "one cold substep from u0 per form (timed), state error against the FP64 "
                             "substep from u0 in the M norm; apply error against the FP64 apply in the "
                             "M^-1 norm", "fp64_ms_per_step": ms_first}
        r64 = None
        for prec, name, dtype in ((FP32_MFMA, "fp32_mfma", "fp32-mfma"), (BF16X3, "bf16x3", "split-bf16 hi/mid/lo"),
                                  (BF16X2, "bf16x2", "split-bf16 hi/lo")):
            if not fits(f"mixed_{name}", 1.5 * ms_first * 1e-3 + (0.7 if r64 is None else 0.35) * t_sub):
                continue
            if r64 is None:
                r64 = h.apply(c.u0)
                r64_n2 = c.minv_norm2(r64)
            up = c.u0.clone()
            h.set_warm_start(False)
            dp, msp = c.timed(lambda: h.substeps(up, c.dt, 1, prec, diag=True))
            ap = c.apply_ms(prec)
            d = h.apply(c.u0, prec=prec) - r64
            mixed[name] = {"ms_per_step": msp, "value": ndof / (msp * 1e-3), "speedup_substep": ms_first / msp,
                           "pcg_iterations": float(dp.cpu()[1, 3]), "apply_ms": ap, "speedup_apply": apply64 / ap,
                           "state_rel_err_vs_fp64_M_norm": c.mnorm_rel(up, u1),
                           "apply_rel_err_vs_fp64_Minv_norm": math.sqrt(c.minv_norm2(d) / r64_n2),
                           "dtype": dtype + " contractions, FP32 accumulation in a tile, FP64 across tiles; "
                                            "FP64 state, transforms, mass solve and diagnostics"}
            del up, d
            log(f"{name}: {msp:.0f} ms/step")
        out["mixed"] = mixed
        del r64
    # the checkpointed reverse chain of L = 1/2 u_1.M u_1 after one
    # substep, FP64 and hi/mid/lo: the forward recomputation, then the
    # reverse step (a mass solve and a transpose Jacobian)
    if not args.no_adjoint:
        n_adj, ck = args.adjoint_steps, args.adjoint_ckpt
        adj = {"substeps": n_adj, "ckpt_every": ck, "loss": "1/2 u_N.M u_N"}
        lamN = None
        lam_ref = None
        for prec, name in ((FP64, "fp64"), (BF16X3, "bf16x3")):
            if not fits(f"adjoint_{name}", (2.5 * n_adj + 0.4) * t_sub):
                continue
            if lamN is None:
                uN = u1.clone() if n_adj == 1 else c.u0.clone()
                if n_adj != 1:
                    h.set_warm_start(False)
                    h.substeps(uN, c.dt, n_adj, FP64)
                lamN = h.mass_apply(uN)
                del uN
            h.set_warm_start(False)
            lam0, ms = c.timed(lambda: h.substeps_vjp(c.u0, c.dt, n_adj, lamN, ckpt_every=ck, prec=prec))
            adj[name] = {"ms": ms, "dof_updates_per_s": ndof * n_adj / (ms * 1e-3)}
            if lam_ref is None:
                lam_ref = lam0
            else:
                adj[name]["rel_err_vs_fp64_Minv_norm"] = math.sqrt(c.minv_norm2(lam0 - lam_ref) /
                                                                   c.minv_norm2(lam_ref))
            log(f"adjoint {name}: {ms:.0f} ms")
        del lam_ref, lamN
        out["adjoint_chain"] = adj
    if args.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device=c.u0.device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = src.numel() * 8
        del src, dst
    del u, u1
    h.close()
    del c
    torch.cuda.empty_cache()
    if not args.no_secondary and args.workload != 2 and fits("secondary", 40):
        # the 3D periodic Taylor-Green workload, FP64 and FP32-MFMA substeps
        c2 = Ctx(2, torch)
        steps2 = 50
        h2 = c2.h
        u2 = c2.u0.clone()
        h2.set_warm_start(False)
        h2.substeps(u2, c2.dt, 3, FP64)
        h2.set_warm_start(True)
        h2.profile(PROF_STRIDE)
        _, ms2 = c2.timed(lambda: h2.substeps(u2, c2.dt, steps2, FP64))
        prof2 = {kk: h2.profile_read(kk) for kk in ("elem", "mass", "prec", "modal", "plain")}
        h2.profile(False)
        roof2, _ = roofline(c2, prof2)
        sec = {"workload": WORKLOADS[2], "value": h2.n_dof * steps2 / (ms2 * 1e-3),
               "ms_per_step": ms2 / steps2, "steps": steps2, "roofline": roof2,
               "apply_ms_fp64": c2.apply_ms(FP64, 20)}
        if not args.no_mixed:
            u2r = c2.u0.clone()
            h2.set_warm_start(False)
            h2.substeps(u2r, c2.dt, 1, FP64)
            h2.set_warm_start(True)
            _, ms2r = c2.timed(lambda: h2.substeps(u2r, c2.dt, steps2, FP64))
            u32 = c2.u0.clone()
            h2.set_warm_start(False)
            h2.substeps(u32, c2.dt, 1, FP32_MFMA)
            h2.set_warm_start(True)
            _, ms32 = c2.timed(lambda: h2.substeps(u32, c2.dt, steps2, FP32_MFMA))
            sec["fp32_mfma"] = {"ms_per_step": ms32 / steps2, "speedup_substep": ms2r / ms32,
                                "apply_ms": c2.apply_ms(FP32_MFMA, 20),
                                "state_rel_err_vs_fp64_M_norm": c2.mnorm_rel(u32, u2r),
                                "protocol": f"1 untimed + {steps2} timed substeps from u0, FP64 on the same"}
            del u2r, u32
        if not args.no_projection:
            # projection step (section 2.3, eq. (MCS_step2)) of the state
            # after the substeps, whose divergence the convection broke
            un = h2.zeros()
            h2.project(u2, un, rtol=1e-13)        # set-up (A^-1) and warm-up
            (_, its), ms = c2.timed(lambda: h2.project(u2, un, rtol=1e-13))
            sec["projection"] = {"ms": ms, "cg_iters": its, "rtol": 1e-13,
                                 "div_l2_before": h2.diagnostics(u2)[1], "div_l2_after": h2.diagnostics(un)[1],
                                 "cpu_oracle": secondary_cpu_oracle("projection")}
        if fits("adaptive", 20):
            # the adaptive HOPU order (end of section 3.2): orders from the
            # jump indicator before every 10th substep, the paper's k = 3
            # thresholds, against the same substeps at the fixed order
            ua = c2.u0.clone()
            h2.set_warm_start(False)
            h2.set_adaptive(10, [0.1, 0.2, 0.3, 0.4], -1)
            h2.substeps(ua, c2.dt, 1, FP64)
            h2.set_warm_start(True)
            _, msa = c2.timed(lambda: h2.substeps(ua, c2.dt, steps2, FP64))
            orders = h2.facet_orders().to(torch.int64) + 1
            hist = torch.bincount(orders, minlength=c2.k + 2).cpu().tolist()
            h2.set_upwind(c2.l)
            sec["adaptive"] = {"ms_per_step": msa / steps2, "value": h2.n_dof * steps2 / (msa * 1e-3),
                               "overhead_vs_fixed_l": msa / ms2 - 1.0,
                               "facet_orders_histogram_from_l=-1": hist,
                               "protocol": f"1 untimed + {steps2} timed substeps from u0 (orders re-selected "
                                           "before substeps 0, 10, 20, ...), thresholds 0.1..0.4",
                               "cpu_oracle": secondary_cpu_oracle("adaptive")}
        out["secondary"] = sec
        h2.close()
        log("secondary done")
    if not args.no_stokes and fits("stokes_step", 90):
        out["stokes_step"] = stokes_section(torch, log)
        torch.cuda.empty_cache()
    if not args.no_secondary and fits("small_latency", 15):
        out["small_latency"] = small_latency(torch)
        log("small-workload latency done")
    out["wall_s"] = time.time() - t_start
    print(json.dumps(out))


if __name__ == "__main__":
    main()
