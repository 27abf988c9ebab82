"""Benchmark of the hot path: voxel energy+gradient evaluations per second.

A step is one mass-projected descent step of the whole field: the fused HIP
sweep evaluates F_h and dF_h/du at every voxel, writes u - tau dF_h/du and the
per-block sums, then the per-instance mass shift is formed (every row of the
hot path). K steps run as one fe_step call, i.e. as replays of a captured HIP
graph, with the field resident in HBM. Before the K timed steps come the W
warmup steps and then CLOCK_SETTLE_S seconds more of the same steps, untimed,
in which the GPU reaches its steady clocks (it raises them over the first tens
of milliseconds of load); every other timed loop settles the same way. Each
workload is also timed as repeated samples (calls of 1 + 2 x 16 graph-replayed
steps, or repeated launches), reported as median and min-max.

Workload (value): a single 256^3 periodic grid, FP32, u0 ~ U(-1,1) (seed 1005),
eps = 1.5h, p = (k1 + k2 - 2)^2 + 0.5 k1 k2, target mean 0, tau = 1e-3.
Also reported, per workload of the method's five configurations:
  * 16 independent 128^3 textures with their own coefficients and target
    means, eps = 2h, mass-projected Adam with lr 1e-3, one launch per step,
    with its own roofline, against 16 sequential single-instance calls;
  * the energy+gradient sweep without the update and the energy-only sweep
    (the autograd forward), each with its roofline;
  * the 256^3 field with a general p (S terms on): its sweep and Adam steps;
  * 32^3 FP64 (200 steps), 64^3 FP32 and FP64 (noisy ball), 128^3 FP32
    (asymmetric p: Adam steps and autograd-driven steps, eager and captured
    in a CUDA graph);
  * Algorithm 1 (the H^-1 flow on a vector field with the Gaussian blur and
    Adam) at the paper's 100^3 simulation size, the coefficient-field
    workloads and Algorithm 2 (Willmore flow, Clifford torus);
  * the FP64 NumPy oracle on the host: one core on the 256^3 field, and all
    cores (a process pool over the 16 instances) on the batched workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--gpus 1]
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2103_04856_amd import fe, inputs  # noqa: E402

HELFRICH_SC = (1.0, 2.5, 1.0, -4.0, -4.0, 4.0)   # (k1 + k2 - 2)^2 + 0.5 k1 k2
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic work of one voxel update, counted on the method's formulas (each
# +, -, x, /, sqrt, exp, log counts one): stencils and M with its invariants and
# the density 97, the reverse sweep 89, the transposed stencils 41, the step 3.
FLOPS_PER_VOXEL = 230
# Of these, the S~ terms take 45: forward 18 (X~ = 2 N2 - T^2: 3; the smoothed
# positive part: 8; S~ = sqrt: 1; c3 T S~ and c5 rho S~ into f: 6) and reverse
# 27 (df/dS~: 3; the logistic: 3; dS~/dX~: 2; kappa and 2 kappa: 2; the three
# 2 m_aa - T~ and their 2 kappa terms: 12; C1 + 2 kappa: 1; the S~ parts of
# df/dT~ and df/drho~: 4). Their coefficients c3 = (a20 - a02)/(2 eps) and
# c5 = (a10 - a01)/2 vanish for p symmetric in k1, k2, and then the method
# needs none of them.
FLOPS_S_TERMS = 45


def flops_per_voxel(a):
    """Algorithmic operations per voxel update for p coefficients a = (a20, a11, a02, a10, a01, a00)."""
    return FLOPS_PER_VOXEL - (FLOPS_S_TERMS if a[0] == a[2] and a[3] == a[4] else 0)
# The forward alone (the energy-only sweep): stencils, M with its invariants
# and the density, 97 operations, of which 18 are the S~ terms.
FLOPS_FORWARD, FLOPS_FORWARD_S_TERMS = 97, 18
# Adam on one voxel: both moments (5), the bias-corrected update (7), replacing
# the plain step's 3.
FLOPS_ADAM_EXTRA = 12 - 3


def forward_flops_per_voxel(a):
    return FLOPS_FORWARD - (FLOPS_FORWARD_S_TERMS if a[0] == a[2] and a[3] == a[4] else 0)


# Algorithmic HBM bytes per voxel, FP32: a step reads u and writes the new u;
# energy + gradient reads u and writes g; the energy alone reads u; an Adam
# step also reads and writes both moments.
BYTES_PER_VOXEL_STEP = 8
BYTES_PER_VOXEL_GRAD = 8
BYTES_PER_VOXEL_ENERGY = 4
BYTES_PER_VOXEL_ADAM = 24
# The batched workload states no step rule. Its coefficients have a20 != a02,
# where the plain gradient step diverges near umbilic voxels at any useful step
# size, so it runs the paper's optimiser: mass-projected Adam, lr 1e-3.
ADAM_LR = 1e-3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# The sources that define the sweep kernels (their per-voxel arithmetic, tiling
# and memory access); the counter record holds only while these are unchanged.
KERNEL_SOURCES = ("fe_voxel.hpp", "fe_kernels.hpp")


def kernel_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2103_04856_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, z_chunk):
    """HBM bytes per launch from the committed counter runs, if they were taken on
    this kernel, launch shape and kernel sources (else None)."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256_prefix") != kernel_hash():
        return None
    for r in t.get("records", []):
        if r.get("kernel") == kernel and r.get("z_chunk") == z_chunk:
            return r.get("traffic_bytes")
    return None


# After its warmup steps, every timed loop first runs the same work untimed for
# this long: the GPU raises its clocks over the first tens of milliseconds of
# sustained load (256^3 step: 117 us per step in the first 2 ms, 94.5 us from
# about 30 ms on), and the timed steps are meant to see the steady state.
CLOCK_SETTLE_S = 0.2


def settle(fn, min_s=CLOCK_SETTLE_S):
    """Run fn() (a short piece of the workload about to be timed) until min_s seconds have passed."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s:
        fn()
        torch.cuda.synchronize()


def samples(fn, reps):
    """fn() timed reps times, each between its own pair of HIP events on the current
    stream; returns the list of ms."""
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def spread(ms, per=1.0):
    """Median and min-max of timed samples, each covering `per` units, in us per unit."""
    us = sorted(1e3 * m / per for m in ms)
    return {"median_us": us[len(us) // 2] if len(us) % 2 else 0.5 * (us[len(us) // 2 - 1] + us[len(us) // 2]),
            "min_us": us[0], "max_us": us[-1], "samples": len(us)}


# A sample of a step loop: the first step launched directly, then two replays of
# the captured 16-step graph.
SAMPLE_STEPS = 33


def time_region(fn, reps=1):
    """Run fn() reps times between HIP events on the current stream; returns ms per rep."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_single(n, steps, warmup, tune):
    h = 1.0 / n
    u = torch.from_numpy(inputs.uniform_noise(n, 1005)).float().cuda()
    ctx = fe.FeContext(u.shape, h, 1.5 * h, HELFRICH_SC, dtype=torch.float32)
    if tune:
        v, z, us, _ = ctx.autotune(u, kind="step", iters=5)
        log(f"autotune 256: variant {v} {fe.variants()[v][:3]} z_chunk {z}: {us:.1f} us")
    mass = [float(u.double().mean().item())]
    # warm-up also captures the step graph that the timed call replays
    ctx.step(u, mass, 1e-3, max(warmup, 17))
    settle(lambda: ctx.step(u, mass, 1e-3, SAMPLE_STEPS))
    ms = time_region(lambda: ctx.step(u, mass, 1e-3, steps))
    step_spread = spread(samples(lambda: ctx.step(u, mass, 1e-3, SAMPLE_STEPS), 10), SAMPLE_STEPS)
    out = {"ms_step": ms / steps, "step_spread": step_spread}
    # the energy+gradient sweep alone (no update, no projection), and the energy alone
    g = torch.empty_like(u)
    E = torch.empty(1, dtype=torch.float64, device=u.device)
    for with_grad, key in ((True, "grad"), (False, "energy")):
        def one():
            ctx.energy_grad_async(u, g if with_grad else None, E, with_grad=with_grad)
        for _ in range(3):
            one()
        settle(one)
        out[key] = spread(samples(one, max(steps, 30)))
    # the diagnostics sweep: curvature fields, a 64 x 64 histogram and the summary
    curv = torch.empty((1, 4) + u.shape, dtype=u.dtype, device=u.device)
    hist = torch.empty((1, 64, 64), dtype=torch.float64, device=u.device)

    def diag():
        ctx.diagnostics_async(u, curv, hist, kmax=100.0)

    diag()
    settle(diag)
    out["diag"] = spread(samples(diag, 10))
    del curv, hist
    return ctx, u, out


# A general p, with the S terms (a20 != a02): the 128^3 configuration's coefficients.
GENERAL_P = (1.0, 0.0, 0.2, -4.0, -4.0, 0.0)


def bench_general(n, steps):
    """The 256^3 field of the step workload with the general p: the energy+gradient sweep
    and mass-projected Adam steps (the plain step diverges near umbilic voxels for such p),
    both with the full per-voxel body."""
    h = 1.0 / n
    u = torch.from_numpy(inputs.uniform_noise(n, 1005)).float().cuda()
    ctx = fe.FeContext(u.shape, h, 1.5 * h, GENERAL_P, dtype=torch.float32)
    g = torch.empty_like(u)
    E = torch.empty(1, dtype=torch.float64, device=u.device)

    def one():
        ctx.energy_grad_async(u, g, E)

    for _ in range(3):
        one()
    settle(one)
    sw = spread(samples(one, max(steps, 30)))
    mass = [float(u.double().mean().item())]
    ctx.step_adam(u, mass, 17)
    settle(lambda: ctx.step_adam(u, mass, SAMPLE_STEPS))
    sa = spread(samples(lambda: ctx.step_adam(u, mass, SAMPLE_STEPS), 5), SAMPLE_STEPS)
    v, zc = ctx.get_launch()
    ctx.close()
    return sw, sa, v, zc


def bench_batched(n, B, warmup, tune):
    """The batched workload as calls of SAMPLE_STEPS mass-projected Adam steps (whole graph
    replays); the same 16 textures as 16 single-instance contexts called one after the other."""
    h = 1.0 / n
    coeffs, means = inputs.random_instance_table(B, 4999)
    U = torch.stack([torch.from_numpy(inputs.uniform_noise(n, 4000 + b)).float() for b in range(B)]).cuda()
    ctx = fe.FeContext(U.shape, h, 2 * h, coeffs, dtype=torch.float32)
    if tune:
        v, z, us, _ = ctx.autotune(U, kind="adam", iters=5)
        log(f"autotune batched: variant {v} {fe.variants()[v][:3]} z_chunk {z}: {us:.1f} us")
    ctx.step_adam(U, list(means), max(warmup, 17), lr=ADAM_LR)
    settle(lambda: ctx.step_adam(U, list(means), SAMPLE_STEPS, lr=ADAM_LR))
    b_spread = spread(samples(lambda: ctx.step_adam(U, list(means), SAMPLE_STEPS, lr=ADAM_LR), 6), SAMPLE_STEPS)
    # the energy+gradient sweep of the batch alone
    g = torch.empty_like(U)
    E = torch.empty(B, dtype=torch.float64, device=U.device)

    def sweep():
        ctx.energy_grad_async(U, g, E)

    sweep()
    settle(sweep)
    grad_spread = spread(samples(sweep, 20))
    del g
    # the same 16 textures, one single-instance context each, called one after the other,
    # each with the launch shape that is best for a single 128^3 grid
    singles = []
    single_launch = None
    for b in range(B):
        c1 = fe.FeContext((1, n, n, n), h, 2 * h, coeffs[b], dtype=torch.float32)
        if single_launch is None and tune:
            v1, z1, us1, _ = c1.autotune(U[0:1].contiguous(), kind="adam", iters=5)
            log(f"autotune single 128: variant {v1} {fe.variants()[v1][:3]} z_chunk {z1}: {us1:.1f} us")
            single_launch = (v1, z1)
        if single_launch is not None:
            c1.set_launch(*single_launch)
        singles.append(c1)
    views = [U[b:b + 1] for b in range(B)]
    for b in range(B):
        singles[b].step_adam(views[b], [means[b]], 17, lr=ADAM_LR)

    def run_singles():
        for b in range(B):
            singles[b].step_adam(views[b], [means[b]], SAMPLE_STEPS, lr=ADAM_LR)

    settle(lambda: singles[0].step_adam(views[0], [means[0]], SAMPLE_STEPS, lr=ADAM_LR))
    s_spread = spread(samples(run_singles, 3), SAMPLE_STEPS)
    return b_spread, grad_spread, s_spread, ctx.get_launch()


def capture_graph(fn, warm=3):
    """fn captured in a CUDA graph after `warm` eager calls on a side stream (the
    capture records the library's kernels, which take the current stream)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(warm):
            fn()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph


def replay_samples(graph, reps=5):
    """Samples of SAMPLE_STEPS replays of a captured graph, in us per replay."""
    def run():
        for _ in range(SAMPLE_STEPS):
            graph.replay()
    run()
    settle(run, 0.05)
    return spread(samples(run, reps), SAMPLE_STEPS)


def step_samples(ctx, u, mass, reps=5):
    """Graph-replayed mass-projected steps (tau = 1e-3) on a copy of u: reps samples
    of SAMPLE_STEPS steps after 17 untimed ones, in us per step. At these sizes the
    stream-ordered energy+gradient call is bound by the host's launch rate; the step
    loop shows what the device sustains."""
    u1 = u.clone()
    ctx.step(u1, mass, 1e-3, 17)
    return spread(samples(lambda: ctx.step(u1, mass, 1e-3, SAMPLE_STEPS), reps), SAMPLE_STEPS)


def bench_configs(args):
    """The method's smaller configurations: 32^3 FP64 (energy+gradient; 200 steps), 64^3
    noisy ball FP32 and FP64 (energy+gradient), 128^3 FP32 asymmetric p (energy+gradient,
    Adam steps, autograd-driven steps). Rates from timed samples (median)."""
    out = {}
    # 32^3 FP64, Willmore p, u0 ~ U(-1,1) seed 1001, eps = 2h, mean 0, tau = 1e-3
    n = 32
    h = 1.0 / n
    u = torch.from_numpy(inputs.uniform_noise(n, 1001)).double().cuda()
    ctx = fe.FeContext(u.shape, h, 2 * h, (0.25, 0.5, 0.25, 0, 0, 0), dtype=torch.float64)
    g = torch.empty_like(u)
    E = torch.empty(1, dtype=torch.float64, device=u.device)
    settle(lambda: ctx.energy_grad_async(u, g, E), 0.05)
    sw = spread(samples(lambda: ctx.energy_grad_async(u, g, E), 50))
    u1 = u.clone()
    ctx.step(u1, [0.0], 1e-3, 17)
    u1 = u.clone()
    t200 = samples(lambda: ctx.step(u1, [0.0], 1e-3, 200), 1)[0]
    ss = step_samples(ctx, u, [0.0])
    out["32cubed_fp64"] = {"energy_grad": sw, "voxels_per_s": n ** 3 / (sw["median_us"] * 1e-6),
                           "steps_200_ms": t200, "steps_per_s": 200 / (t200 * 1e-3),
                           "step": ss, "step_voxels_per_s": n ** 3 / (ss["median_us"] * 1e-6),
                           "config": "32^3 FP64, u0~U(-1,1) seed 1001, eps=2h, p=(k1+k2)^2/4, mean 0, tau=1e-3"}
    # 64^3 noisy ball, eps = 1.5h, Willmore p, FP32 and FP64
    n = 64
    h = 1.0 / n
    u0 = inputs.noisy_sphere(n, 0.3, 1.5 * h, 0.01, 1002)
    for dt, key in ((torch.float32, "64cubed_fp32"), (torch.float64, "64cubed_fp64")):
        u = torch.from_numpy(u0).to(dt).cuda()
        ctx = fe.FeContext(u.shape, h, 1.5 * h, (0.25, 0.5, 0.25, 0, 0, 0), dtype=dt)
        g = torch.empty_like(u)
        settle(lambda: ctx.energy_grad_async(u, g, E), 0.05)
        sw = spread(samples(lambda: ctx.energy_grad_async(u, g, E), 50))
        ss = step_samples(ctx, u, [u.double().mean().item()])
        out[key] = {"energy_grad": sw, "voxels_per_s": n ** 3 / (sw["median_us"] * 1e-6),
                    "step": ss, "step_voxels_per_s": n ** 3 / (ss["median_us"] * 1e-6),
                    "steps_per_s": 1e6 / ss["median_us"],
                    "config": "64^3 tanh ball R=0.3 + N(0,0.01^2) seed 1002, eps=1.5h, p=(k1+k2)^2/4, "
                              "mass-projected step tau=1e-3 at the initial mean"}
    # 128^3 FP32, asymmetric p, mean -0.3
    n = 128
    h = 1.0 / n
    a3 = (1.0, 0.0, 0.2, -4.0, -4.0, 0.0)
    u = torch.from_numpy(inputs.uniform_noise(n, 1003)).float().cuda()
    ctx = fe.FeContext(u.shape, h, 2 * h, a3, dtype=torch.float32)
    g = torch.empty_like(u)
    settle(lambda: ctx.energy_grad_async(u, g, E), 0.05)
    sw = spread(samples(lambda: ctx.energy_grad_async(u, g, E), 50))
    u1 = u.clone()
    ctx.step_adam(u1, [-0.3], 17)
    settle(lambda: ctx.step_adam(u1, [-0.3], SAMPLE_STEPS), 0.05)
    sa = spread(samples(lambda: ctx.step_adam(u1, [-0.3], SAMPLE_STEPS), 5), SAMPLE_STEPS)
    # autograd-driven steps, the paper's loop: E = FeEnergy(y) (energy-only sweep), backward
    # (the adjoint sweep), torch.optim.Adam on y (fused and capturable: one kernel, its step
    # count on the device), then the mass projection in torch; eager, and captured in a CUDA graph
    # (whose replays skip the host work of the autograd engine, about 90 us per backward
    # pass here); also the forward and backward alone, captured
    def autograd_adam(x0):
        y = x0.clone().requires_grad_(True)
        opt = torch.optim.Adam([y], lr=ADAM_LR, fused=True, capturable=True)

        def step():
            opt.zero_grad(set_to_none=True)
            fe.feps(y, ctx).sum().backward()
            opt.step()
            with torch.no_grad():
                y.add_(-0.3 - y.mean())
        return step

    autograd_step = autograd_adam(u)
    for _ in range(5):
        autograd_step()
    st = spread(samples(autograd_step, 30))
    g_st = capture_graph(autograd_adam(u))
    sgs = replay_samples(g_st)
    y = u.clone().requires_grad_(True)
    g_fb = capture_graph(lambda: torch.autograd.grad(fe.feps(y, ctx).sum(), y))
    sfb = replay_samples(g_fb)
    del g_fb, g_st
    log(f"  128^3 autograd Adam step: eager {st['median_us']:.1f} us, graph-captured {sgs['median_us']:.1f} us "
        f"(forward + backward {sfb['median_us']:.1f} us; fused Adam step {sa['median_us']:.1f} us)")
    out["128cubed_fp32"] = {"energy_grad": sw, "voxels_per_s": n ** 3 / (sw["median_us"] * 1e-6),
                            "adam_step": sa, "adam_steps_per_s": 1e6 / sa["median_us"],
                            "autograd_step": st, "autograd_steps_per_s": 1e6 / st["median_us"],
                            "autograd_step_rule": "FeEnergy forward + backward, torch.optim.Adam lr 1e-3 "
                                                  "(fused, capturable), mass projection in torch",
                            "autograd_forward_backward_graphed": sfb,
                            "autograd_step_graphed": sgs, "autograd_graphed_steps_per_s": 1e6 / sgs["median_us"],
                            "autograd_forward_backward_graphed_over_adam_step": sfb["median_us"] / sa["median_us"],
                            "config": "128^3 FP32, u0~U(-1,1) seed 1003, eps=2h, a=(1,0,0.2,-4,-4,0), mean -0.3"}
    return out


# Algorithm 1 at the paper's simulation size (Sec. 5): 100^3 pixels with dx = 0.01,
# eps = 0.02, Adam lr 1e-3, betas (0.9, 0.999), blur sigma_k = 2 pixels; the
# coefficients and mass of its convergence figure, a = (1, 2.4, 9, 30, 170, -195)
# in the (a20, a11, a02, a10, a01, a00) order, m0 = -0.66. The paper runs 8000
# iterations per shape in up to 150 s on its own GPU.
HMINUS_A = (1.0, 2.4, 9.0, 30.0, 170.0, -195.0)
HMINUS_M0 = -0.66
PAPER_HMINUS_ITERS, PAPER_HMINUS_SECONDS = 8000, 150.0


def bench_hminus(n, iters, batch=1, dtype=torch.float32):
    """Algorithm 1 on `batch` shapes of n^3 at once (each from its own A0 seed, the
    same coefficients and mass). Returns (ms per iteration, G after 16, G at the end,
    iterations done) with G of the first shape."""
    h = 1.0 / n
    A = torch.from_numpy(inputs.white_noise_vector_field(n, 2021, 0.4 * h, batch=batch)).to(dtype).cuda()
    ctx = fe.FeContext((batch, n, n, n), h, [0.02] * batch, [HMINUS_A] * batch, dtype=dtype)
    m0 = [HMINUS_M0] * batch
    G0 = ctx.hminus_step(A, m0, 16, sigma_k=2.0, lr=1e-3)[0].item()   # also captures the graph
    iters = 8 * max(1, iters // 8)
    # the clocks settle on a copy in a context of its own, so the reported
    # energies stay those of the stated iteration counts
    cs = fe.FeContext((batch, n, n, n), h, [0.02] * batch, [HMINUS_A] * batch, dtype=dtype)
    As = A.clone()
    settle(lambda: cs.hminus_step(As, m0, 8, sigma_k=2.0, lr=1e-3))
    del cs, As
    ms = time_region(lambda: ctx.hminus_step(A, m0, iters, sigma_k=2.0, lr=1e-3)) / iters
    G1 = ctx.hminus_step(A, m0, 8, sigma_k=2.0, lr=1e-3)[0].item()
    return ms, G0, G1, iters + 24


# The paper's spatialised example (Sec. 5.2): four parameter sets, interpolated
# along x over six cells (the first and last repeated), with their masses; here
# six 100^3 cells at dx = 0.01, eps = 0.02, sigma_k = 2, Adam lr 1e-3.
SPATIAL_SETS = [(2, 2, 2, 0, 0, 0), (1, 2, 6, -40, -40, 400), (2, 2, 2, -75, -75, 937.5),
                (2, 2, 11, -180, -90, 4050)]
SPATIAL_MASSES = [-0.4, -0.6, -0.7, -0.7]


def bench_spatial_flow(iters):
    nz, ny, nx = 100, 100, 600
    h = 0.01
    a_np, m_np = inputs.interpolated_parameters((nz, ny, nx), SPATIAL_SETS, SPATIAL_MASSES)
    ctx = fe.FeContext((1, nz, ny, nx), h, 0.02, SPATIAL_SETS[0], dtype=torch.float32)
    ctx.set_coeff_field(torch.from_numpy(a_np[None]).float().cuda())
    ctx.set_mass_field(torch.from_numpy(m_np[None]).float().cuda())
    del a_np, m_np
    rng = np.random.default_rng(2022)
    A = torch.from_numpy(rng.normal(0.0, 0.4 * h, size=(1, 3, nz, ny, nx))).float().cuda()
    ctx.hminus_step(A, None, 16, sigma_k=2.0)
    iters = 8 * max(1, iters // 8)
    settle(lambda: ctx.hminus_step(A, None, 8, sigma_k=2.0))
    return time_region(lambda: ctx.hminus_step(A, None, iters, sigma_k=2.0)) / iters


def bench_field_sweep(n, reps):
    """The energy+gradient sweep at n^3 with a coefficient field (random around the
    Helfrich-type vector of the main workload)."""
    h = 1.0 / n
    u = torch.from_numpy(inputs.uniform_noise(n, 1005)).float().cuda()[None].contiguous()
    ctx = fe.FeContext(u.shape, h, 1.5 * h, HELFRICH_SC, dtype=torch.float32)
    rng = np.random.default_rng(77)
    af = torch.tensor(HELFRICH_SC, dtype=torch.float32).reshape(1, 6, 1, 1, 1).cuda() * \
        (1 + 0.1 * torch.from_numpy(rng.uniform(-1, 1, size=(1, 6, n, n, n))).float().cuda())
    ctx.set_coeff_field(af)
    del af
    g = torch.empty_like(u)
    E = torch.empty(1, dtype=torch.float64, device=u.device)
    for _ in range(3):
        ctx.energy_grad_async(u, g, E)
    settle(lambda: ctx.energy_grad_async(u, g, E))
    return time_region(lambda: ctx.energy_grad_async(u, g, E), reps=reps)


def bench_clifford_torus(steps=24):
    """Algorithm 2 on the paper's genus-1 validation: the Willmore flow (p = H^2) with
    replicate boundaries and L-BFGS from a tanh torus of ratio 0.58 on 192^3, eps = 0.02,
    sigma_k = 1, FP32. Returns (seconds, F/(8 pi^2 sigma), r/R, iterations run)."""
    n, eps = 192, 0.02
    h = 1.0 / n
    u0 = torch.from_numpy(inputs.tanh_torus(n, 0.24, 0.14, eps)).float().cuda()
    flow = fe.FeL2Flow((n, n, n), h, eps, (1, 2, 1, 0, 0, 0), sigma_k=1.0, dtype=torch.float32)
    settle(lambda: flow.energy_grad(u0))      # before load, which resets the optimiser
    flow.load(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flow.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    u = flow.store()
    E, _ = flow.energy_grad(u)
    line = 0.5 * (u[n // 2 - 1, n // 2 - 1, :] + u[n // 2, n // 2, :]).double().cpu().numpy()
    xs = (np.arange(n) + 0.5) * h - 0.5
    cross = sorted(abs(xs[i] + line[i] / (line[i] - line[i + 1]) * h)
                   for i in range(n - 1) if (line[i] > 0) != (line[i + 1] > 0))
    ratio = float("nan")
    if len(cross) == 4:
        inner, outer = 0.5 * (cross[0] + cross[1]), 0.5 * (cross[2] + cross[3])
        ratio = (outer - inner) / (outer + inner)
    sigma = 4.0 / (3.0 * math.sqrt(2.0))
    return dt, E / sigma / (8 * math.pi ** 2), ratio, steps * 20


def host_cpu():
    """(CPU model, logical CPUs visible to this process)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        ncpu = os.cpu_count() or 1
    return model, ncpu


def cpu_baseline(n=256, budget_s=10.0, max_evals=3):
    """The FP64 NumPy oracle on a bounded sample of the same workload: whole 256^3
    energy + gradient evaluations, repeated until about budget_s seconds (at most
    max_evals), timed on the host; NumPy element-wise kernels use one core."""
    from oracle import fe_oracle as fo
    h = 1.0 / n
    u = inputs.uniform_noise(n, 1005)
    evals, t0 = 0, time.perf_counter()
    while evals < max_evals and (evals == 0 or time.perf_counter() - t0 < budget_s):
        fo.energy_grad(u, h, 1.5 * h, HELFRICH_SC)
        evals += 1
    dt = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return dict(value=evals * u.size / dt, unit="voxel energy+gradient evals/s", cores=1, kind="oracle",
                sample=f"{evals} FP64 energy+gradient evaluation(s) of the full 256^3 field ({dt:.1f} s)",
                cpu_model=model, nproc=ncpu)


def cpu_baseline_configs(budget_s=1.0):
    """The oracle (one core) on the smaller configurations' inputs: FP64 energy + gradient
    evaluations repeated for about budget_s seconds each (at least one)."""
    from oracle import fe_oracle as fo
    willmore_q = (0.25, 0.5, 0.25, 0.0, 0.0, 0.0)
    cases = {
        "32cubed": (inputs.uniform_noise(32, 1001), 32, 2.0, willmore_q),
        "64cubed": (inputs.noisy_sphere(64, 0.3, 1.5 / 64, 0.01, 1002), 64, 1.5, willmore_q),
        "128cubed": (inputs.uniform_noise(128, 1003), 128, 2.0, (1.0, 0.0, 0.2, -4.0, -4.0, 0.0)),
    }
    out = {}
    for key, (u, n, eps_h, a) in cases.items():
        evals, t0 = 0, time.perf_counter()
        while evals == 0 or (time.perf_counter() - t0 < budget_s and evals < 100):
            fo.energy_grad(u, 1.0 / n, eps_h / n, a)
            evals += 1
        dt = time.perf_counter() - t0
        out[key] = {"value": evals * u.size / dt, "evals": evals, "seconds": dt}
    return out


def _oracle_instance(b):
    """One instance of the batched workload through the oracle (a pool worker)."""
    from oracle import fe_oracle as fo
    n = 128
    h = 1.0 / n
    coeffs, _ = inputs.random_instance_table(16, 4999)
    u = inputs.uniform_noise(n, 4000 + b)
    fo.energy_grad(u, h, 2 * h, coeffs[b])
    return u.size


def cpu_baseline_batched(B=16):
    """The oracle on the batched workload with every host core: one FP64 energy+gradient
    evaluation of each of the 16 instances, a process pool of min(16, CPUs) workers."""
    import multiprocessing as mp
    model, ncpu = host_cpu()
    workers = max(1, min(B, ncpu))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_instance, range(min(workers, B)))     # start the workers, import numpy
        t0 = time.perf_counter()
        vox = sum(pool.map(_oracle_instance, range(B)))
        dt = time.perf_counter() - t0
    return dict(value=vox / dt, unit="voxel energy+gradient evals/s", cores=workers, kind="oracle",
                sample=f"one FP64 energy+gradient evaluation of each of the 16 instances of 128^3 ({dt:.1f} s)",
                cpu_model=model, nproc=ncpu)


def other_workloads(args, extra, n, vox):
    """Algorithm 1, the coefficient-field workloads and Algorithm 2, into `extra`."""
    log("Algorithm 1 (H^-1 flow) at 100^3 ...")
    ms_h, G0, G1, done = bench_hminus(100, max(args.steps, 64))
    extra["hminus_flow_100"] = {
        "iterations_per_s": 1e3 / ms_h, "ms_per_iteration": ms_h,
        "voxel_iterations_per_s": 100 ** 3 / (ms_h * 1e-3),
        "seconds_for_8000_iterations": PAPER_HMINUS_ITERS * ms_h * 1e-3,
        "energy_after_16": G0, f"energy_after_{done}": G1,
        "config": "100^3, dx=0.01, eps=0.02, a=(1,2.4,9,30,170,-195), m0=-0.66, sigma_k=2, Adam lr 1e-3, "
                  "A0 ~ N(0,(0.4dx)^2) seed 2021, FP32, graph-replayed",
        "paper_context": f"{PAPER_HMINUS_ITERS} iterations in up to {PAPER_HMINUS_SECONDS:.0f} s per shape "
                         f"(>= {PAPER_HMINUS_ITERS / PAPER_HMINUS_SECONDS:.0f} it/s) on the paper's GPU"}
    log(f"  {ms_h * 1e3:.1f} us/iteration ({1e3 / ms_h:.0f} it/s); G {G0:.4g} -> {G1:.4g}")
    if not args.no_batched:
        ms_h16, _, _, _ = bench_hminus(100, max(args.steps // 2, 32), batch=16)
        extra["hminus_flow_100"]["batched_16"] = {
            "shape_iterations_per_s": 16e3 / ms_h16, "ms_per_iteration": ms_h16,
            "seconds_for_8000_iterations_of_16_shapes": PAPER_HMINUS_ITERS * ms_h16 * 1e-3}
        log(f"  16 shapes at once: {ms_h16 * 1e3:.1f} us/iteration ({16e3 / ms_h16:.0f} shape-it/s)")

    log("coefficient field a(x): 256^3 sweep and the spatialised 600x100x100 flow ...")
    ms_field = bench_field_sweep(n, max(args.steps // 2, 10))
    ms_sflow = bench_spatial_flow(max(args.steps // 4, 16))
    extra["coefficient_field"] = {
        "energy_grad_sweep_256_us": ms_field * 1e3, "voxels_per_s": vox / (ms_field * 1e-3),
        "spatial_flow_600x100x100": {"ms_per_iteration": ms_sflow, "iterations_per_s": 1e3 / ms_sflow,
                                     "config": "a(x), m(x) interpolated along x from the four parameter sets "
                                               "of the paper's spatialised example, dx=0.01, eps=0.02, "
                                               "sigma_k=2, Adam lr 1e-3, FP32"}}
    log(f"  field sweep {ms_field * 1e3:.1f} us; spatialised flow {ms_sflow * 1e3:.1f} us/iteration")

    log("Algorithm 2 (L2 Willmore flow, replicate boundaries, L-BFGS): Clifford torus at 192^3 ...")
    dt_t, f_t, ratio_t, it_t = bench_clifford_torus()
    extra["l2flow_clifford_torus_192"] = {
        "seconds": dt_t, "iterations": it_t, "iterations_per_s": it_t / dt_t,
        "F_over_8pi2_sigma": f_t, "ratio_r_over_R": ratio_t, "ratio_over_clifford": ratio_t * math.sqrt(2.0),
        "config": "p=H^2 (a=(1,2,1,0,0,0)), eps=0.02, sigma_k=1, replicate boundaries, L-BFGS lr 1 history 10 "
                  "20 iterations/step x 24 steps, from a tanh torus R=0.24 r=0.14, FP32",
        "paper_context": "Sec. 4.2 reports F/sigma within 0.4% of 8 pi^2 and the ratio within 3% of 1/sqrt 2"}
    log(f"  {dt_t:.2f} s for {it_t} iterations; F/(8 pi^2 sigma) {f_t:.4f}, r/R {ratio_t:.4f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="only the 256^3 workload (step, sweep, diagnostics): for counter runs")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 256^3 step and the batched workload: for counter runs")
    ap.add_argument("--tune", action="store_true",
                    help="run the launch-shape autotuner first (default: the library's default shape)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 64 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    # the all-cores oracle baseline starts its worker processes before this process
    # touches the GPU (a process that has initialised the GPU starts no programs)
    pool_baseline = None
    if not args.no_cpu and not args.main_only and not args.batched_only and not args.no_batched:
        log("CPU oracle baseline (all cores, the 16 x 128^3 batch) ...")
        pool_baseline = cpu_baseline_batched()
    if not torch.cuda.is_available():
        print("no ROCm device visible", file=sys.stderr)
        sys.exit(1)
    fe.lib()

    if args.copy_probe:
        a = torch.empty(16 * 2 ** 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    n = 256
    vox = n ** 3
    log(f"device {torch.cuda.get_device_name(0)}; 256^3 FP32 step loop ...")
    ctx, u, single = bench_single(n, args.steps, args.warmup, args.tune)
    ms_step = single["ms_step"]
    variant, zc = ctx.get_launch()
    log(f"  {ms_step * 1e3:.1f} us/step (samples: median {single['step_spread']['median_us']:.1f}, "
        f"{single['step_spread']['min_us']:.1f}-{single['step_spread']['max_us']:.1f}), "
        f"energy+grad sweep {single['grad']['median_us']:.1f} us, energy sweep {single['energy']['median_us']:.1f} us, "
        f"diagnostics {single['diag']['median_us']:.1f} us")
    value = vox / (ms_step * 1e-3)

    extra = {}
    if not args.batched_only:
        log("256^3 with a general p (S terms): energy+gradient sweep and Adam steps ...")
        gsw, gsa, gv, gzc = bench_general(n, args.steps)
        gvi = fe.variants()[gv]
        ak = f"grad_sweep<float,{gvi[0]},{gvi[1]},{gvi[2]},2,false,false,2>"
        gk = f"grad_sweep<float,{gvi[0]},{gvi[1]},{gvi[2]},0,false,false,2>"
        aroof, _ = roofline(FLOPS_PER_VOXEL + FLOPS_ADAM_EXTRA, BYTES_PER_VOXEL_ADAM, vox, gsa["median_us"], ak,
                            measured_traffic(ak, gzc))
        sroof, _ = roofline(FLOPS_PER_VOXEL, BYTES_PER_VOXEL_GRAD, vox, gsw["median_us"], gk,
                            measured_traffic(gk, gzc))
        extra["general_p_256"] = {
            "p": list(GENERAL_P), "eps": "1.5h", "z_chunk": gzc,
            "energy_grad_sweep": {"value": vox / (gsw["median_us"] * 1e-6), "us": gsw, "roofline": sroof},
            "adam_step": {"value": vox / (gsa["median_us"] * 1e-6), "us": gsa, "roofline": aroof},
            "unit": "voxel energy+gradient evals/s"}
        log(f"  sweep {gsw['median_us']:.1f} us, Adam step {gsa['median_us']:.1f} us")
    if not args.no_batched and not args.main_only:
        log("16 x 128^3 batched vs 16 single-instance calls ...")
        b_spread, bg_spread, s_spread, (bvar, bzc) = bench_batched(128, 16, args.warmup, args.tune)
        vb = 16 * 128 ** 3
        bv = fe.variants()[bvar]
        bk = f"grad_sweep<float,{bv[0]},{bv[1]},{bv[2]},2,false,false,2>"
        broof, bother = roofline(FLOPS_PER_VOXEL + FLOPS_ADAM_EXTRA, BYTES_PER_VOXEL_ADAM, vb,
                                 b_spread["median_us"], bk, measured_traffic(bk, bzc))
        gk = f"grad_sweep<float,{bv[0]},{bv[1]},{bv[2]},0,false,false,2>"
        groof, _ = roofline(FLOPS_PER_VOXEL, BYTES_PER_VOXEL_GRAD, vb, bg_spread["median_us"], gk,
                            measured_traffic(gk, bzc))
        extra["batched_16x128"] = {
            "value": vb / (b_spread["median_us"] * 1e-6), "us_per_step": b_spread,
            "unit": "voxel energy+gradient evals/s", "step_rule": "mass-projected Adam, lr 1e-3",
            "launch_variant": list(bv[:3]), "z_chunk": bzc,
            "roofline": broof, "roofline_other": bother,
            "energy_grad_sweep": {"value": vb / (bg_spread["median_us"] * 1e-6), "us": bg_spread, "roofline": groof},
            "sequential_singles_value": vb / (s_spread["median_us"] * 1e-6), "sequential_singles_us_per_step": s_spread,
            "batched_over_singles": s_spread["median_us"] / b_spread["median_us"],
            "batched_over_256cubed_per_voxel": (vb / b_spread["median_us"]) / (vox / (ms_step * 1e3))}
        log(f"  batched {b_spread['median_us']:.1f} us/step ({b_spread['min_us']:.1f}-{b_spread['max_us']:.1f}), "
            f"its sweep {bg_spread['median_us']:.1f} us, singles {s_spread['median_us']:.1f} us/step")

    if not args.main_only and not args.batched_only:
        log("smaller configurations (32^3 FP64, 64^3 FP32/FP64, 128^3 FP32) ...")
        extra["configs"] = bench_configs(args)
        for k, v in extra["configs"].items():
            log(f"  {k}: energy+grad {v['energy_grad']['median_us']:.1f} us ({v['voxels_per_s']:.3g} voxel/s)")
        other_workloads(args, extra, n, vox)

    vinfo = fe.variants()[variant]
    kname = f"grad_sweep<float,{vinfo[0]},{vinfo[1]},{vinfo[2]},1,false,false,1>"
    roof, other = roofline(flops_per_voxel(HELFRICH_SC), BYTES_PER_VOXEL_STEP, vox, ms_step * 1e3, kname,
                           measured_traffic(kname, zc))
    ek = "energy_sweep_cols<float,2,8>"
    eroof, eother = roofline(forward_flops_per_voxel(HELFRICH_SC), BYTES_PER_VOXEL_ENERGY, vox,
                             single["energy"]["median_us"], ek, measured_traffic(ek, None))
    gk = f"grad_sweep<float,{vinfo[0]},{vinfo[1]},{vinfo[2]},0,false,false,1>"
    groof, _ = roofline(flops_per_voxel(HELFRICH_SC), BYTES_PER_VOXEL_GRAD, vox, single["grad"]["median_us"], gk,
                        measured_traffic(gk, zc))

    out = {
        "metric": "voxel energy+gradient evals/sec at 256^3 FP32 and batched 16x128^3; % HBM peak",
        "value": value,
        "unit": "voxel energy+gradient evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_settle_s": CLOCK_SETTLE_S,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single 256^3 periodic grid, FP32, u0~U(-1,1) seed 1005, eps=1.5h, "
                               "p=(k1+k2-2)^2+0.5k1k2, mass-projected step tau=1e-3, graph-replayed",
                   "grid": [n, n, n], "batch": 1, "launch_variant": list(fe.variants()[variant][:3]),
                   "z_chunk": zc},
        "roofline": roof,
        "roofline_other": other,
        "us_per_step_samples": single["step_spread"],
        "steps_per_s": 1e3 / ms_step,
        "energy_grad_sweep": {"value": vox / (single["grad"]["median_us"] * 1e-6), "us": single["grad"],
                              "roofline": groof},
        "energy_sweep": {"value": vox / (single["energy"]["median_us"] * 1e-6), "us": single["energy"],
                         "unit": "voxel energy evals/s", "roofline": eroof, "roofline_other": eother},
        "diagnostics_sweep": {"us": single["diag"], "voxels_per_s": vox / (single["diag"]["median_us"] * 1e-6),
                              "outputs": "H, K, kappa1, kappa2 fields, 64x64 curvature histogram, "
                                         "F_h, A_eps, discrepancy, min/max u"},
    }
    out.update(extra)
    if not args.no_cpu:
        log("CPU oracle baseline (one core, 256^3) ...")
        out["cpu_baseline"] = cpu_baseline()
        if not args.main_only and not args.batched_only:
            out["cpu_baseline"]["per_config"] = cpu_baseline_configs()
    if pool_baseline is not None:
        out["cpu_baseline_batched"] = pool_baseline
    print(json.dumps(out), flush=True)


def roofline(ops_per_voxel, bytes_per_voxel, voxels, us, kernel, traffic):
    """(the binding roof, the other) for a kernel doing `voxels` voxels in `us`: its
    algorithmic operations against the FP32 vector peak and its algorithmic bytes
    against HBM; the larger fraction is the bound."""
    tflops = ops_per_voxel * voxels / (us * 1e-6) / 1e12
    gbs = bytes_per_voxel * voxels / (us * 1e-6) / 1e9
    alu = {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic}
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": traffic}
    roof, other = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    roof = dict(roof, kernel=kernel, duration_us=us, ops_per_voxel=ops_per_voxel, bytes_per_voxel=bytes_per_voxel)
    # the published FP32 vector peak counts packed two-wide FMAs; the library
    # compiles with packed FP32 disabled, so its attainable ALU ceiling is half
    if roof["bound"] == "alu":
        roof["unpacked_fp32_peak"] = FP32_VECTOR_PEAK_TFLOPS / 2
        roof["frac_of_unpacked_peak"] = tflops / (FP32_VECTOR_PEAK_TFLOPS / 2)
    return roof, other


if __name__ == "__main__":
    main()
