#!/usr/bin/env python3
"""Benchmark of the APR-SPH hot path on one MI355X.

Metric: SPH pair interactions per second (density + force), FP32 form vs FP64
form.  Workload: the 64^3 = 262144-particle periodic box (jittered lattice,
left/right states rho/P = 1/1 and 0.125/0.1 carried by masses of levels 0 and
3, adiabatic gamma = 5/3, artificial viscosity alpha = 1, beta = 2), stepped
with the kick-drift-kick leapfrog at the fixed dt = 0.3 min(h / vsig) of t = 0.

A step is one full pass of the library's step: kick, drift, cell build
(Morton sort + cells + tree), density with its h-rho Newton iteration, EOS,
forces, kick.  The box has no refinement zone, so its step contains no
split/merge pass.  Interactions per step = sum_a |{b != a: r < 2 h_a}|
(density) + sum_a |{b != a: r < 2 max(h_a, h_b)}| (force), counted with the
library's exact neighbour export before and after the timed steps (mean).
value = interactions per step * steps / wall time of the timed steps.

The same run times the rest of the path on the other workloads ("legs"): the
refined box (one split pass over 262144 particles, then density + forces +
adjoint on the 362k-particle result, both forms), the same box and step with
the Wendland C2 kernel (h_fact 1.3, FP32 form), the sound-wave box of the
paper's appendix A (run to t = 2 with and without its refinement zone; the
density blip at the zone boundary), relaxing after that box's split, the
1M-particle planet disc
stepped with its refinement zone (every step: cells, density, split/merge,
forces, sink gravity, leapfrog) and the 8M-particle circumbinary disc (FP32
density + forces + adjoint).

The FP64 form runs twice: at its own Newton tolerance 1e-12 and at the FP32
form's 1e-6 (the like-for-like comparison of the precisions); each form
reports its Newton passes per step.

The CPU baseline (the FP64 oracle on a bounded ball sample) is taken on the
FP32 form's state after its timed steps, so that it also states that form's
error: the oracle's h, rho, a and du/dt at the GPU's positions against the
GPU's own ("error_vs_oracle").

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-legs]
       [--no-cpu-baseline] [--fp32-only] [--only-leg circumbinary]
Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPH pair interactions/s (density+force), FP32 vs FP64 form, at stated error"
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)
# Algorithmic floating-point operations per pair, as the hot-path scope
# counts them: the density pair about 30 (the kernel, its h-derivative and
# the second derivative for the h-rho Newton step, one sqrt) plus about 8 for
# the compensated (Kahan) sums, 38 in all; the force pair about 70 (both
# supports' kernel gradients, one sqrt and one reciprocal, the viscosity, the
# acceleration and du/dt) plus about 16 of compensation, 86.  Each counts
# once per pair at the converged h, however many Newton passes run.  The
# leaner counts of the formulas alone, without compensation or the second
# derivative (22 and 59), are reported beside them.
FLOP_DENSITY_PAIR = 38
FLOP_FORCE_PAIR = 86
FLOP_DENSITY_PAIR_MIN = 22
FLOP_FORCE_PAIR_MIN = 59
# Algorithmic HBM bytes per particle (the hot-path scope's count): density
# reads x (24), level (1), h (8) and writes h, rho, Omega, n_neigh (8 + 4 +
# 4 + 4), 53 in all; forces read x, v, level, h, rho, Omega, u (24 + 24 + 1
# + 8 + 4 + 4 + 8) and write a, du/dt, vsig (12 + 4 + 4), 93.
BYTES_DENSITY = 53
BYTES_FORCES = 93
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE over the 20 timed launches, each scaled by what the
# counter reads for a plain 1 GiB device copy: fetch x2.000, write x1.000),
# with the digest of the kernel's sources at the time; reported only while the
# sources are unchanged.
MEASURED_TRAFFIC = {
    "k_density<float, 0, false, false>": dict(
        bytes_per_launch=47788638,
        sources=("paper_2409_11470_amd/csrc/density.hip", "paper_2409_11470_amd/csrc/search.hpp",
                 "paper_2409_11470_amd/csrc/common.hpp"),
        sha256="690bd1dfbd34921a3971ecb54f2eba317f14a71a36ae924ddbb1ca3688a69651"),
}


def measured_traffic(kernel):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return m["bytes_per_launch"] if h.hexdigest() == m["sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_ctx(A, p, precision, seed=7, tol=None):
    """A context for a workload's parameter dict p in the given form (Newton
    tolerance 1e-6 for FP32, 1e-12 for FP64, unless tol is given)."""
    if tol is None:
        tol = 1e-6 if precision == "fp32" else 1e-12
    return A.Context(A.make_params(
        precision=A.APR_FP32 if precision == "fp32" else A.APR_FP64, eos=int(p["eos"]),
        periodic=int(p["periodic"]), box_lo=p["lo"], box_hi=p["hi"], m0=p["m0"],
        hfact=p["hfact"], kernel=int(p.get("kernel", 0)), gamma=p["gamma"], cs0=p["cs0"],
        q_cs=p.get("q_cs", 0.25),
        r_ref=p.get("r_ref", 1.0), av_alpha=p["alpha"], av_beta=p["beta"],
        tol_h=tol, max_iter=60,
        r_sep_factor=p.get("r_sep_factor", 0.2), nn_cap=p.get("nn_cap", 0.0),
        split_mode=int(p.get("split_mode", 0)), seed=seed, G=p.get("G", 1.0)))


def count_interactions(A, ctx, ds):
    h = ds["h"].contiguous()
    return (A.apr_neighbours(ctx, ds, h, 0, count_only=True),
            A.apr_neighbours(ctx, ds, h, 1, count_only=True))


def final_values(A, torch, ctx, ds):
    """Density and hydro forces on a copy of the state as it stands (cells
    rebuilt): per-id numpy arrays of x, y, z, h, rho, ax, ay, az, dudt, and the
    other state arrays the oracle needs."""
    import numpy as np
    w = ds.clone()
    A.apr_build_cells(ctx, w)
    n = w.n
    dt = ctx.dtype
    rho = torch.zeros(n, dtype=dt, device="cuda")
    om = torch.zeros_like(rho)
    A.apr_density(ctx, w, rho, om)
    acc = [torch.zeros_like(rho) for _ in range(4)]
    A.apr_forces(ctx, w, rho, om, *acc)
    A.apr_sync_status(ctx)
    g = w.to_numpy()
    ids = g["id"]
    out = {}
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "level"):
        v = np.empty_like(g[k])
        v[ids] = g[k]
        out[k] = v
    for k, t in (("rho", rho), ("ax", acc[0]), ("ay", acc[1]), ("az", acc[2]),
                 ("dudt", acc[3])):
        v = np.empty(n)
        v[ids] = t.double().cpu().numpy()
        out[k] = v
    return out


def run_form(A, torch, st, p, precision, steps, warmup, tol=None, keep_final=False):
    ctx = make_ctx(A, p, precision, tol=tol)
    ds = A.DeviceState.from_numpy(st)
    A.apr_accel(ctx, ds)
    dt = A.apr_timestep(ctx, ds, 0.3)
    A.apr_sync_status(ctx)
    for k in range(warmup):
        A.apr_step(ctx, ds, [], [], dt, k)
    A.apr_sync_status(ctx)
    d0, f0 = count_interactions(A, ctx, ds)
    torch.cuda.synchronize()
    # inside the timed steps only the roofline kernel is bracketed by events:
    # every event record waits for the work before it, and timing all the
    # kernel groups costs the step about 5 %
    A.apr_profile_enable(ctx, True)
    A.apr_profile_select(ctx, [A.APR_PROF_DENSITY])
    A.apr_profile_read(ctx, reset=True)
    A.apr_counters(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        A.apr_step(ctx, ds, [], [], dt, warmup + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = A.apr_profile_read(ctx, reset=True)
    A.apr_profile_enable(ctx, False)
    counters = A.apr_counters(ctx, reset=True)
    fails = A.apr_sync_status(ctx)
    d1, f1 = count_interactions(A, ctx, ds)
    n = ds.n
    idens = 0.5 * (d0 + d1)
    iforce = 0.5 * (f0 + f1)
    wall = t1 - t0
    per_step = idens + iforce
    ms_d, cnt_d = prof[A.APR_PROF_DENSITY]
    res = dict(n=n, dt=dt, wall_s=wall, ms_per_step=1e3 * wall / steps,
               interactions_per_step=per_step, density_pairs=idens, force_pairs=iforce,
               value=per_step * steps / wall, failures=fails,
               density_ms=ms_d / max(cnt_d, 1),
               newton_passes_per_step=counters["density_passes"] / steps,
               counters=counters, newton_tol=ctx.params.tol_h)
    if keep_final:
        res["final"] = final_values(A, torch, ctx, ds)
    ctx.close()
    # every kernel group's time over the same steps: the run again from the
    # same start (the steps are deterministic), all groups timed, outside the
    # wall time above
    ctx = make_ctx(A, p, precision, tol=tol)
    ds = A.DeviceState.from_numpy(st)
    A.apr_accel(ctx, ds)
    for k in range(warmup):
        A.apr_step(ctx, ds, [], [], dt, k)
    A.apr_sync_status(ctx)
    A.apr_profile_enable(ctx, True)
    A.apr_profile_read(ctx, reset=True)
    for k in range(steps):
        A.apr_step(ctx, ds, [], [], dt, warmup + k)
    prof2 = A.apr_profile_read(ctx, reset=True)
    A.apr_profile_enable(ctx, False)
    A.apr_sync_status(ctx)
    ms_f, cnt_f = prof2[A.APR_PROF_FORCES]
    ms_c, cnt_c = prof2[A.APR_PROF_CELLS]
    ms_p, cnt_p = prof2[A.APR_PROF_CAND]
    ms_d2, cnt_d2 = prof2[A.APR_PROF_DENSITY]
    res.update(forces_ms=ms_f / max(cnt_f, 1), cells_ms=ms_c / max(cnt_c, 1),
               cand_ms_per_step=ms_p / max(steps, 1), launches=(cnt_d, cnt_f, cnt_c),
               density_ms_all_timed=ms_d2 / max(cnt_d2, 1),
               group_timing="density_ms from events on the timed steps (the only kernel "
                            "timed there); forces_ms, cells_ms, cand_ms_per_step from the "
                            "same steps run again with every group timed")
    # density + forces pass: both kernels and the candidate walks ahead of them
    res["density_force_rate"] = per_step / (1e-3 * (res["density_ms"] + res["forces_ms"] +
                                                    res["cand_ms_per_step"]))
    ctx.close()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(st, p, nballs=64, gpu=None, h_guess=None):
    """The FP64 oracle (brute force, OpenMP) on a bounded sample of the same
    workload: the density (h-rho Newton) of every particle within reach of
    nballs balls of 48 targets, then the forces on the targets (about 15 s on
    16 host threads).

    With gpu (the GPU form's per-id values on the state st, final_values),
    the sample is also the stated error of that form: the oracle's h, rho
    and forces at the same positions against the GPU's, at the targets.  The
    oracle's Newton starts from h_guess (the workload's initial h), not from
    the GPU's h."""
    import numpy as np
    import oracle
    n = st["x"].shape[0]
    h0 = st["h"] if h_guess is None else h_guess
    pos = np.stack([st["x"], st["y"], st["z"]], 1)
    hs = 1.2 / 64
    rng = np.random.default_rng(99)
    tg, sh = [], []
    for c in rng.choice(n, nballs, replace=False):
        d = pos - pos[c]
        d -= np.round(d)
        r = np.sqrt((d * d).sum(1))
        order = np.argsort(r, kind="stable")[:48]
        tg.append(order)
        sh.append(np.nonzero(r < r[order[-1]] + 4.5 * hs)[0])
    tg = np.unique(np.concatenate(tg))
    sh = np.unique(np.concatenate(sh))
    kw = dict(m0=p["m0"], periodic=True, lo=p["lo"], hi=p["hi"])
    t0 = time.perf_counter()
    o = oracle.density(st["x"], st["y"], st["z"], st["level"], h0[sh], tol=1e-12,
                       max_iter=60, targets=sh, **kw)
    h, rho, om = np.full(n, 1e-9), np.ones(n), np.ones(n)
    h[sh], rho[sh], om[sh] = o["h"], o["rho"], o["omega"]
    f = oracle.forces(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"],
                      st["level"], h, rho, om, eos=int(p["eos"]), gamma=p["gamma"],
                      alpha=p["alpha"], beta=p["beta"], targets=tg, **kw)
    t1 = time.perf_counter()
    err = None
    if gpu is not None:
        ga = np.sqrt(sum((gpu[k][tg] - f[k]) ** 2 for k in ("ax", "ay", "az")))
        err = dict(targets=int(tg.shape[0]),
                   h_max_rel=float(np.max(np.abs(gpu["h"][tg] / h[tg] - 1))),
                   rho_max_rel=float(np.max(np.abs(gpu["rho"][tg] / rho[tg] - 1))),
                   a_max_rel_l1=float(np.max(ga / f["anorm"])),
                   dudt_max_rel_l1=float(np.max(np.abs(gpu["dudt"][tg] - f["dudt"])
                                                / np.maximum(f["unorm"], 1e-300))),
                   gates=dict(rho=1e-3, a=1e-3),
                   definition="at the sampled targets, GPU FP32 form vs the FP64 oracle at "
                              "the same positions: max |h/h_o - 1|, |rho/rho_o - 1|, "
                              "|a - a_o| / sum_b |pair term| (the L1 pair sum), |du/dt - "
                              "du/dt_o| / L1 sum")
    nb = oracle.neighbours(st["x"], st["y"], st["z"], h, symmetric=True, periodic=True,
                           lo=p["lo"], hi=p["hi"], targets=tg)
    inter = float(np.sum(o["nneigh"] - 1)) + float(sum(len(a) for a in nb))
    return dict(value=inter / (t1 - t0), unit="interactions/s", cores=oracle.num_threads(),
                cpu=_cpu_model(), kind="oracle",
                sample="FP64 oracle: h-rho Newton for %d particles (within reach of %d balls "
                       "of 48 targets) over all %d sources, then forces on %d targets; %.1f s"
                       % (sh.shape[0], nballs, n, tg.shape[0], t1 - t0),
                seconds=t1 - t0, error=err)


def _cot(torch, n, dt, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return [torch.randn(n, dtype=dt, device="cuda", generator=g) for _ in range(5)]


def forward_adjoint(A, torch, ctx, ds, reps):
    """Density + forces + adjoint (apr_vjp with seeded N(0,1) cotangents on rho,
    a and du/dt) on the state's current cells, reps times; kernel times from
    the library's stream events."""
    n = ds.n
    dt = ctx.dtype
    rho = torch.empty(n, dtype=dt, device="cuda")
    om = torch.empty_like(rho)
    acc = [torch.empty_like(rho) for _ in range(4)]
    rb, ab0, ab1, ab2, ub = _cot(torch, n, dt, 17)
    A.apr_build_cells(ctx, ds)
    A.apr_density(ctx, ds, rho, om)
    A.apr_forces(ctx, ds, rho, om, *acc)
    A.apr_vjp(ctx, ds, rho, om, rb, None, ab0, ab1, ab2, ub)
    A.apr_sync_status(ctx)
    A.apr_profile_enable(ctx, True)
    A.apr_profile_read(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        A.apr_density(ctx, ds, rho, om)
        A.apr_forces(ctx, ds, rho, om, *acc)
        A.apr_vjp(ctx, ds, rho, om, rb, None, ab0, ab1, ab2, ub)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = A.apr_profile_read(ctx, reset=True)
    A.apr_profile_enable(ctx, False)
    fails = A.apr_sync_status(ctx)
    d, f = count_interactions(A, ctx, ds)
    ms = {k: prof[i][0] / max(prof[i][1], 1) for k, i in
          (("density_ms", A.APR_PROF_DENSITY), ("forces_ms", A.APR_PROF_FORCES),
           ("vjp_ms", A.APR_PROF_VJP))}
    ms["cand_ms_per_rep"] = prof[A.APR_PROF_CAND][0] / reps
    inter = d + f
    out = dict(n=n, interactions=inter, density_pairs=d, force_pairs=f, failures=fails,
               reps=reps, wall_ms_per_rep=1e3 * wall / reps, **ms)
    # each of density, forces and the adjoint has one candidate walk ahead of it
    cw = ms["cand_ms_per_rep"] / 3.0
    out["forward_rate"] = inter / (1e-3 * (ms["density_ms"] + ms["forces_ms"] + 2 * cw))
    out["adjoint_rate"] = inter / (1e-3 * (ms["vjp_ms"] + cw))
    out["forward_adjoint_rate"] = inter * reps / wall
    return out


def leg_refine_box(A, torch, W, reps):
    """The refined box: one split pass over 262144 particles (about 1e5 split),
    then forward + adjoint on the 362k-particle result in both forms."""
    st, p = W.refine_box()
    n = st["x"].shape[0]
    times = []
    for k in range(reps + 1):
        ctx = make_ctx(A, p, "fp64")
        ds = A.DeviceState.from_numpy(st, capacity=2 * n + 8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ns, nm, nsp = A.apr_split_merge(ctx, ds, p["zones"], 3, 1)
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t0)
        ctx.close()
    times.sort()
    out = dict(workload="refined box: 64^3 periodic shock box, split sphere r = 0.45 at the "
                        "centre (level 4), tangential split, r_sep = 0.2 h",
               n_before=n, n_split=ns, split_pass_ms=1e3 * times[len(times) // 2],
               split_particles_per_s=n / times[len(times) // 2])
    for prec in ("fp32", "fp64"):
        ctx = make_ctx(A, p, prec)
        out[prec] = forward_adjoint(A, torch, ctx, ds.clone(), reps)
        ctx.close()
    return out


def leg_wendland_box(A, torch, W, steps, warmup):
    """The benchmarked box and step with the Wendland C2 kernel at h_fact 1.3
    (the kernel of the paper's example applications), FP32 form."""
    st, p = W.shock_box()
    p = dict(p, kernel=1, hfact=1.3)
    r = run_form(A, torch, st, p, "fp32", steps, warmup)
    out = dict(workload="periodic shock box, 64^3 = 262144 particles, as the headline, "
                        "Wendland C2 kernel, h_fact 1.3", form="fp32", steps=steps)
    out.update({k: r[k] for k in ("value", "ms_per_step", "density_ms", "forces_ms",
                                  "cells_ms", "interactions_per_step", "density_pairs",
                                  "force_pairs", "density_force_rate", "failures")})
    return out


def _wave_run(A, torch, st, p, zones_on, t_split=0.5, t_end=2.0):
    """The sound-wave box stepped to t_end (dt = 0.3 min(h / vsig), taken again
    after the split), zone active from t_split; returns the final state with
    its density, the step count and the wall time of the steps."""
    ctx = make_ctx(A, p, "fp32", seed=5)
    ds = A.DeviceState.from_numpy(st, capacity=2 * st["x"].shape[0])
    A.apr_accel(ctx, ds)
    dt = A.apr_timestep(ctx, ds, 0.3)
    torch.cuda.synchronize()
    t, k, split_done, t0 = 0.0, 0, False, time.perf_counter()
    while t < t_end - 1e-12:
        zones = p["zones"] if (zones_on and t >= t_split) else []
        step = min(dt, t_end - t)
        A.apr_step(ctx, ds, zones, [], step, k)
        t += step
        k += 1
        if zones and not split_done:
            split_done = True
            dt = A.apr_timestep(ctx, ds, 0.3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    A.apr_sync_status(ctx)
    A.apr_build_cells(ctx, ds)
    rho = torch.zeros(ds.n, dtype=torch.float32, device="cuda")
    om = torch.zeros_like(rho)
    A.apr_density(ctx, ds, rho, om)
    A.apr_sync_status(ctx)
    out = ds.to_numpy()
    out["rho"] = rho.double().cpu().numpy()
    ctx.close()
    return out, k, wall


def _blip(a, b, nbins=50):
    import numpy as np

    def prof(r):
        sel = (r["y"] > 0.4) & (r["y"] < 0.6)
        i = np.minimum((r["x"][sel] * nbins).astype(int), nbins - 1)
        return (np.bincount(i, weights=r["rho"][sel], minlength=nbins)
                / np.maximum(np.bincount(i, minlength=nbins), 1))
    return float(np.max(np.abs(prof(a) - prof(b))))


def leg_wave_box(A, torch, W):
    """The sound-wave box of the paper's appendix A (56832 particles, cylinder
    zone r = 0.1 at level 1 from t = 0.5, to t = 2), FP32 form, with and
    without the zone, for the M4 and the Wendland C2 kernel: wall time per
    step of the refined run and the density blip (largest difference of the
    binned 0.4 < y < 0.6 cross-section density, over the initial mean 1)."""
    out = dict(workload="sound-wave box, 64 x 74 x 12 hcp lattice, A = 0.02, cylinder zone "
                        "r = 0.1, level 1 from t = 0.5 to t = 2, FP32 form")
    for name, kw in (("m4", dict(kernel=0, hfact=1.2)), ("wc2", dict(kernel=1, hfact=1.3))):
        st, p = W.wave_box(hfact=kw["hfact"])
        p = dict(p, **kw)
        ref, _, _ = _wave_run(A, torch, st, p, False)
        apr, steps, wall = _wave_run(A, torch, st, p, True)
        out[name] = dict(steps=steps, ms_per_step=1e3 * wall / steps, n_final=int(apr["x"].shape[0]),
                         blip=_blip(apr, ref))
    return out


def leg_relax(A, torch, W):
    """Relaxing (Sec. 2.4) after the sound-wave box's split at t = 0 (56832
    particles, 1758 split), FP32 form: the paper's limits (50 shuffles, KE
    down to 0.5 %); wall time per shuffle (cells, density, forces,
    interpolation from the reference set, shift)."""
    st, p = W.wave_box()
    p = dict(p, nn_cap=0.0)  # the split context has no density pass of its own
    par = make_ctx(A, p, "fp32", seed=5).params
    rctx, ctx = A.Context(par), A.Context(par)
    dr = A.DeviceState.from_numpy(st)
    A.apr_build_cells(rctx, dr)
    n = dr.n
    rho, om = (torch.zeros(n, device="cuda") for _ in range(2))
    A.apr_density(rctx, dr, rho, om)
    a = [torch.zeros(n, device="cuda") for _ in range(4)]
    A.apr_forces(rctx, dr, rho, om, *a)
    A.apr_sync_status(rctx)
    ds = dr.clone()
    ds.grow(2 * n)
    ns, _, _ = A.apr_split_merge(ctx, ds, p["zones"], 1, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, ke0, ke1 = A.apr_relax(ctx, ds, rctx, dr, rho, a[0], a[1], a[2], 50, 0.005)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    A.apr_sync_status(ctx)
    rctx.close()
    ctx.close()
    return dict(workload="sound-wave box, 56832 particles, relaxing after its split at t = 0",
                n_split=ns, shuffles=k, ke_ratio=ke1 / ke0 if ke0 > 0 else 0.0,
                ms_per_shuffle=1e3 * wall / max(k, 1))


def leg_circumbinary(A, torch, W, reps):
    """The 8M-particle circumbinary disc (three masses): FP32 forward + adjoint,
    and the roofline of its density + force pass against both HBM (the
    algorithmic bytes per particle) and the FP32 VALU (the algorithmic FLOPs
    per pair)."""
    st, p = W.circumbinary_disc()
    ctx = make_ctx(A, p, "fp32")
    ds = A.DeviceState.from_numpy(st)
    del st
    fa = forward_adjoint(A, torch, ctx, ds, reps)
    n = fa["n"]
    sec = 1e-3 * (fa["density_ms"] + fa["forces_ms"])
    flops = FLOP_DENSITY_PAIR * (fa["density_pairs"] + n) + FLOP_FORCE_PAIR * fa["force_pairs"]
    hbm = (BYTES_DENSITY + BYTES_FORCES) * n
    fa["density_force_roofline"] = dict(
        pass_ms=1e3 * sec,
        valu=dict(achieved=flops / sec / 1e12, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                  frac=flops / sec / 1e12 / PEAK_FP32_TFLOPS, flop=flops),
        hbm=dict(achieved=hbm / sec / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                 frac=hbm / sec / 1e9 / PEAK_HBM_GBS, bytes=hbm),
        binding="valu")
    out = dict(workload="circumbinary disc, 8.0M particles (levels 0, 1, 2), locally "
                        "isothermal", fp32=fa)
    ctx.close()
    return out


def leg_planet_disc(A, torch, W, steps):
    """The 1M-particle planet disc stepped with its refinement zone: every step
    runs kick, drift, cells, density, split/merge, cells and density again,
    forces, sink gravity, kick."""
    st, p = W.planet_disc()
    ctx = make_ctx(A, p, "fp32", seed=3)
    ds = A.DeviceState.from_numpy(st, capacity=st["x"].shape[0] * 5 // 4)
    A.apr_accel(ctx, ds, p["sinks"])
    dt = 2e-3
    A.apr_step(ctx, ds, p["zones"], p["sinks"], dt, 0)
    A.apr_sync_status(ctx)
    n0 = ds.n
    d0, f0 = count_interactions(A, ctx, ds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        A.apr_step(ctx, ds, p["zones"], p["sinks"], dt, 1 + k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fails = A.apr_sync_status(ctx)
    d1, f1 = count_interactions(A, ctx, ds)
    inter = 0.5 * (d0 + d1 + f0 + f1)
    ctx.close()
    return dict(workload="planet disc, 1M particles, refinement sphere r = 1 at (5, 0, 0), "
                         "random split r_sep = 0.5 h, sink at the origin, dt = 2e-3",
                form="fp32", steps=steps, n_first=n0, n_last=ds.n, failures=fails,
                ms_per_step=1e3 * wall / steps, interactions_per_step=inter,
                value=inter * steps / wall)


def leg_planet_disc_bins(A, torch, W, nsub=64, max_bin=6):
    """Individual timesteps (Sec. 2.5) on the 1M-particle planet disc with its
    refinement zone and sink: the same time advanced twice, by `nsub` global
    steps of the smallest Courant step dt_g, and by one step of dt_max =
    nsub dt_g with per-particle bins (2^K substeps, K <= max_bin).  Each run
    starts from the same state, after one untimed step of its own kind."""
    import numpy as np
    st, p = W.planet_disc()
    n = st["x"].shape[0]
    out = dict(workload="planet disc, 1M particles, refinement sphere r = 1 at (5, 0, 0), "
                        "random split r_sep = 0.5 h, sink at the origin",
               form="fp32", n=n)
    ctx = make_ctx(A, p, "fp32", seed=3)
    ds = A.DeviceState.from_numpy(st, capacity=3 * n + 64)
    A.apr_accel(ctx, ds, p["sinks"])
    dtg = A.apr_timestep(ctx, ds)
    dt_max = nsub * dtg
    A.apr_step(ctx, ds, p["zones"], p["sinks"], dtg, 0)
    A.apr_sync_status(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsub):
        A.apr_step(ctx, ds, p["zones"], p["sinks"], dtg, 1 + k)
    torch.cuda.synchronize()
    wall_g = time.perf_counter() - t0
    A.apr_sync_status(ctx)
    ctx.close()
    del ds
    ctx = make_ctx(A, p, "fp32", seed=3)
    ds = A.DeviceState.from_numpy(st, capacity=3 * n + 64)
    A.apr_bins_init(ctx, ds, dt_max, 0.3, max_bin, p["sinks"])
    A.apr_step_bins(ctx, ds, p["zones"], p["sinks"], dt_max, 0, 0.3, max_bin)
    A.apr_sync_status(ctx)
    hist = np.bincount(ds["bin"].cpu().numpy().astype(np.int64), minlength=max_bin + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ns = A.apr_step_bins(ctx, ds, p["zones"], p["sinks"], dt_max, 1, 0.3, max_bin)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    A.apr_sync_status(ctx)
    # particle updates: every particle is active 2^bin times per dt_max
    upd = float(np.sum(hist * (2.0 ** np.arange(hist.size))))
    ctx.close()
    out.update(dt_global=dtg, dt_max=dt_max, substeps=ns, bins=hist.tolist(),
               active_fraction=float(upd / (hist.sum() * ns)), global_ms=1e3 * wall_g,
               bins_ms=1e3 * wall_b, speedup=wall_g / wall_b)
    return out


def form_summary(r):
    return {k: r[k] for k in ("value", "ms_per_step", "density_ms", "density_ms_all_timed",
                              "forces_ms", "cells_ms", "cand_ms_per_step", "group_timing",
                              "interactions_per_step",
                              "density_force_rate", "newton_tol", "newton_passes_per_step",
                              "failures", "counters")}


def density_roofline(r32):
    """Roofline of the dominant kernel of the FP32 form, the h-rho Newton density
    kernel (the longest of the step in every trace; plain VALU arithmetic):
    algorithmic FLOPs per launch over its mean launch time (HIP events on the
    library's stream, around it alone during the timed steps)."""
    n = r32["n"]
    kern, ms = "k_density<float, 0, false, false>", r32["density_ms"]
    pairs = r32["density_pairs"] + n
    flops, flops_min = FLOP_DENSITY_PAIR * pairs, FLOP_DENSITY_PAIR_MIN * pairs
    achieved = flops / (ms * 1e-3) / 1e12
    traffic = measured_traffic(kern)
    roof = dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=achieved / PEAK_FP32_TFLOPS, traffic=traffic, kernel=kern,
                flop_per_launch=flops, ms_per_launch=ms,
                frac_lean_flops=flops_min / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS)
    if traffic is not None:
        roof["traffic_unit"] = "bytes per launch (HBM, counters)"
        roof["traffic_gbs"] = traffic / (ms * 1e-3) / 1e9
    return roof


def copy_probe(torch):
    """Three plain device copies of 1 GiB: what the HBM byte counters read for a
    known transfer (their scale factors)."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 8


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the disc and refined-box legs")
    ap.add_argument("--only-leg", default=None, choices=("circumbinary", "bins"),
                    help="run only this leg, for profiling")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2409_11470_amd as A
    import workloads as W
    torch.cuda.set_device(0)
    st, p = W.shock_box()
    log("workload: %d particles" % st["x"].shape[0])
    only = args.only_leg
    r32 = r64 = r64t = roof = None
    if only is None:
        r32 = run_form(A, torch, st, p, "fp32", args.steps, args.warmup, keep_final=True)
        log("fp32: %.3e interactions/s, %.3f ms/step" % (r32["value"], r32["ms_per_step"]))
        if not args.fp32_only:
            r64 = run_form(A, torch, st, p, "fp64", args.steps, args.warmup)
            log("fp64: %.3e interactions/s, %.3f ms/step" % (r64["value"], r64["ms_per_step"]))
            # the FP64 form at the FP32 form's Newton tolerance: the like-for-like
            # comparison of the two precisions
            r64t = run_form(A, torch, st, p, "fp64", args.steps, args.warmup, tol=1e-6)
            log("fp64 at tol 1e-6: %.3e interactions/s, %.3f ms/step"
                % (r64t["value"], r64t["ms_per_step"]))
        roof = density_roofline(r32)
    legs = None
    if only is not None:
        legs = {}
        if only == "circumbinary":
            legs["circumbinary_forward_adjoint"] = leg_circumbinary(A, torch, W, 3)
        else:
            legs["planet_disc_bins"] = leg_planet_disc_bins(A, torch, W)
    elif not args.no_legs:
        legs = {}
        legs["refine_box_split_adjoint"] = leg_refine_box(A, torch, W, 5)
        log("refined box: split %.2f ms, fp32 adjoint %.3e interactions/s"
            % (legs["refine_box_split_adjoint"]["split_pass_ms"],
               legs["refine_box_split_adjoint"]["fp32"]["adjoint_rate"]))
        legs["wendland_c2_box"] = leg_wendland_box(A, torch, W, 10, 3)
        log("wendland c2 box: %.3e interactions/s, %.3f ms/step"
            % (legs["wendland_c2_box"]["value"], legs["wendland_c2_box"]["ms_per_step"]))
        legs["wave_box_blip"] = leg_wave_box(A, torch, W)
        log("wave box: blip %.4f (M4), %.4f (Wendland C2), %.3f ms/step"
            % (legs["wave_box_blip"]["m4"]["blip"], legs["wave_box_blip"]["wc2"]["blip"],
               legs["wave_box_blip"]["m4"]["ms_per_step"]))
        legs["relax_wave_box"] = leg_relax(A, torch, W)
        log("relax: %d shuffles, KE ratio %.3f, %.3f ms per shuffle"
            % (legs["relax_wave_box"]["shuffles"], legs["relax_wave_box"]["ke_ratio"],
               legs["relax_wave_box"]["ms_per_shuffle"]))
        legs["planet_disc_steps"] = leg_planet_disc(A, torch, W, 10)
        log("planet disc: %.3e interactions/s, %.2f ms/step"
            % (legs["planet_disc_steps"]["value"], legs["planet_disc_steps"]["ms_per_step"]))
        torch.cuda.empty_cache()
        legs["planet_disc_bins"] = leg_planet_disc_bins(A, torch, W)
        log("planet disc over %d dt_g: global %.1f ms, bins %.1f ms (x%.2f), bins %s"
            % (legs["planet_disc_bins"]["substeps"], legs["planet_disc_bins"]["global_ms"],
               legs["planet_disc_bins"]["bins_ms"], legs["planet_disc_bins"]["speedup"],
               legs["planet_disc_bins"]["bins"]))
        legs["circumbinary_forward_adjoint"] = leg_circumbinary(A, torch, W, 3)
        log("circumbinary: fp32 forward+adjoint %.3e interactions/s"
            % legs["circumbinary_forward_adjoint"]["fp32"]["forward_adjoint_rate"])
        torch.cuda.empty_cache()
    cpu = err = None
    if not args.no_cpu_baseline and r32 is not None:
        cpu = cpu_baseline(r32["final"], p, gpu=r32["final"], h_guess=st["h"])
        log("cpu baseline: %.3e interactions/s on %d threads" % (cpu["value"], cpu["cores"]))
        err = cpu.pop("error")
        err["state"] = "the FP32 form's state after its %d timed steps" % args.steps
        log("fp32 error vs oracle at the final state: rho %.2e, a %.2e (of the L1 pair sum)"
            % (err["rho_max_rel"], err["a_max_rel_l1"]))
        cpu.pop("seconds")
    if r32 is None:
        out = {"legs": legs}
        if args.copy_probe:
            out["copy_probe_bytes"] = copy_probe(torch)
        print(json.dumps(out), flush=True)
        return
    out = {
        "metric": METRIC, "value": r32["value"], "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "periodic shock box, 64^3 = 262144 particles, jittered lattice, "
                               "mixed mass (levels 0 and 3), adiabatic, KDK leapfrog",
                   "n_particles": r32["n"], "precision_form": "fp32 (cell-relative, "
                   "compensated sums; FP64 positions, leapfrog, Newton test)",
                   "newton_tol": 1e-6},
        "roofline": roof, "cpu_baseline": cpu, "error_vs_oracle": err,
        "fp32_form": form_summary(r32),
        "fp64_form": None if r64 is None else form_summary(r64),
        "fp64_form_at_fp32_tol": None if r64t is None else form_summary(r64t),
    }
    out["legs"] = legs
    if r64 is not None:
        out["fp32_over_fp64"] = r32["value"] / r64["value"]
        out["fp32_over_fp64_same_tol"] = r32["value"] / r64t["value"]
    if args.copy_probe:
        out["copy_probe_bytes"] = copy_probe(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
