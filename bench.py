"""Throughput of the ADER-DG step on one MI355X.

Workload (default): 3-D compressible Euler, order N = 5 (6^3 Gauss-Legendre
nodes per cell, 5 quantities), 64^3 periodic cells, seeded smooth Fourier
initial state, FP64.  One timed step is the whole hot path: the predictor
kernel (space-time predictor, time averages, volume integral, face
projection) and the corrector kernel (Rusanov, surface integral, update,
and the Eq. (7) maximum for the next step's dt).  The first dt comes from the
stand-alone reduction during warm-up.

Prints one JSON line.  value = DoFs per step * steps / timed seconds, with
DoFs = cells * (N+1)^3 * 5.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ADER-DG DoF-updates/s per step, FP64 vs mixed at stated L2 error; adjoint s/grad"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (= FP64 matrix) peak
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak
PEAK_HBM_GBS = 8000.0


def predictor_flops_per_cell(dim: int, N: int, nvar: int, iters: int, flux_flops: int) -> int:
    """Algorithmic FLOPs of the predictor kernel per cell and step (I Picard
    iterations of: pointwise flux, 1-D derivative contractions of every flux
    component along its direction, the K1^{-1} W time operator and the
    update; then the averages at the final iterate, the volume divergence and
    the extrapolation of qbar and Fbar_d to both faces of every line)."""
    n = N + 1
    S = n ** dim
    P = n * S                      # space-time nodes
    deriv = dim * nvar * 2 * n     # per space-time node
    timeop = nvar * 2 * n
    update = nvar * 2
    per_iter = P * (flux_flops + deriv + timeop + update)
    final = P * (flux_flops + 2 * dim * nvar + 2 * nvar)
    volume = S * dim * nvar * 2 * n
    traces = 2 * dim * (S // n) * 2 * nvar * 2 * n
    return iters * per_iter + final + volume + traces


def euler_flux_flops(dim: int) -> int:
    # 1/rho (1), |j|^2 (2 dim - 1), p (4), E + p (1); per direction: u_d (1),
    # u_d j (dim), + p (1), u_d (E + p) (1)
    return 1 + (2 * dim - 1) + 4 + 1 + dim * (3 + dim)


def kernel_source_hash() -> str:
    """Hash of the FP64 predictor's source: its file (layout struct and kernel
    body), the line derivative, tables, fma helper and channel map it inlines,
    and the Euler terms."""
    csrc = os.path.join(ROOT, "paper_1905_07987_amd", "csrc")
    k = open(os.path.join(csrc, "kernels.hpp")).read()
    a = k.index("struct CT {")
    b = k.index("};", a)
    c = k.index("// y = s D x along one line of n nodes.")  # line_deriv
    d = k.index("// Kernel A, a lane pair per node", c)
    g0 = k.index("// a * b + c with one rounding")  # fma_r and Chan
    g1 = k.index("\n};", k.index("struct Chan {"))
    pde = open(os.path.join(csrc, "pde.hpp")).read()
    e = pde.index("struct Euler {")
    f = pde.index("\n};", e)
    h = hashlib.sha256()
    h.update(open(os.path.join(csrc, "predict64.hpp")).read().encode())
    h.update(k[a:b].encode())
    h.update(k[c:d].encode())
    h.update(k[g0:g1].encode())
    h.update(pde[e:f].encode())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM bytes per predictor launch measured with rocprofv3 counters, if the
    recorded kernel-source hash matches the current sources."""
    path = os.path.join(ROOT, "profiles", f"predict_kernel_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cells: int, N: int):
    """The oracle, as it stands, timed on the host cores for one step of the
    same per-cell work on a smaller periodic mesh; also on one thread (a
    quarter of the cells)."""
    import oracle as O
    from paper_1905_07987_amd import inputs

    def one_step(m, threads):
        used = O.set_threads(threads)
        P = O.problem(3, N, O.EULER, [m] * 3, cfl=0.5)
        Q = inputs.c2_state(O.node_coords(P))
        t0 = time.perf_counter()
        dt, _ = O.stable_dt(P, Q)
        O.step(P, Q, None, dt, 0.0)
        el = time.perf_counter() - t0
        return P.ncells * 5 * (N + 1) ** 3 / el, el, used

    value, el, threads = one_step(cells, min(os.cpu_count() or 1, 16))
    m1 = max(2, cells // 4)
    v1, el1, _ = one_step(m1, 1)
    return {"value": value, "unit": "DoF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one step (dt reduction + predictor + corrector) of the same 3-D Euler N={N} "
                      f"workload on {cells}^3 periodic cells, {el:.2f} s wall",
            "single_thread": {"value": v1, "unit": "DoF-updates/s", "cores": 1,
                              "sample": f"the same step on {m1}^3 cells, {el1:.2f} s wall"}}


def euler_c1(log, steps: int = 10):
    """C1: 2-D Euler N=3, 16^2 periodic cells, CFL 0.9, 10 steps of the
    paper's density wave (Eqs. (8), (10)), Eq. (7) every step; microseconds
    per step, launched step by step and replayed from a HIP graph of the 10
    steps (the workload is launch-bound); error against the closed form."""
    import torch
    from paper_1905_07987_amd import adg, inputs
    s = adg.Solver(2, 3, "euler", [16, 16], cfl=0.9)
    xyz = s.node_coords()
    Q0 = torch.as_tensor(inputs.c1_state(xyz), device="cuda")
    stream = torch.cuda.current_stream()

    def eager():
        Q = Q0.clone()
        clock = torch.zeros(2, dtype=torch.float64, device="cuda")
        s.stable_dt(Q, None, clock)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            s.step(Q, None, clock, next_dt=True)
        b.record(stream)
        torch.cuda.synchronize()
        return Q, clock, a.elapsed_time(b) * 1e3 / steps

    for _ in range(3):
        eager()
    Q, clock, us = eager()
    t = float(clock[0])
    exact = torch.as_tensor(inputs.c1_state(xyz, t), device="cuda")
    err = float(torch.linalg.vector_norm(Q - exact) / torch.linalg.vector_norm(exact))
    res = {"workload": "c1: 2-D Euler, N=3, 16^2 periodic cells, CFL 0.9, 10 steps",
           "us_per_step": round(us, 2), "t_end": t, "rel_l2_vs_closed_form": err}
    # the same 10 steps captured once in a graph and replayed
    gs = torch.cuda.Stream()
    Qg = Q0.clone()
    cg = torch.zeros(2, dtype=torch.float64, device="cuda")
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=gs):  # gs is the current stream inside
        s.stable_dt(Qg, None, cg)
        for _ in range(steps):
            s.step(Qg, None, cg, next_dt=True)
    equal = True
    for _ in range(3):
        Qg.copy_(Q0)
        cg.zero_()
        graph.replay()
        torch.cuda.synchronize()
        equal = equal and bool(torch.equal(Qg, Q)) and bool(torch.equal(cg, clock))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    a.record(stream)
    for _ in range(reps):
        graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    res["graph_us_per_step"] = round(a.elapsed_time(b) * 1e3 / (reps * steps), 2)
    res["graph_replays_bitwise_equal_eager"] = equal
    log(f"c1: {us:.1f} us/step eager, {res['graph_us_per_step']:.1f} us/step graph replay "
        f"(bitwise {equal}), rel L2 vs closed form {err:.2e}")
    del graph
    return res


def adjoint_c4(log, steps: int | None = None, every: int = 15, grad: bool = True):
    """C4: seconds per gradient of the seismogram misfit of the 3-D elastic
    workload (N=3, 32^3 cells, 200 steps, 16 receivers) with respect to the
    per-cell (rho, cp, cs) and the initial state: forward run with
    checkpoints every `every` steps, then per segment the recomputation
    (keeping what each step's adjoint reads) and the adjoint steps (autograd
    Function over the library's adjoint)."""
    import torch
    from paper_1905_07987_amd import adg, inputs
    from paper_1905_07987_amd.autograd import seismograms
    cfg = inputs.elastic_config("c4")
    steps = steps or cfg["steps"]
    s = adg.Solver(3, cfg["order"], "elastic", cfg["cells"], cfg["lo"], cfg["hi"])
    s.set_point_sources([cfg["source"]])
    s.set_receivers(cfg["receivers"])
    params = torch.as_tensor(cfg["params"], device="cuda")
    pert = np.random.default_rng(cfg["seed"] + 1).uniform(-1.0, 1.0, cfg["params"].shape)
    params_obs = torch.as_tensor(cfg["params"] * (1.0 + 0.05 * pert), device="cuda")
    u0 = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
    clock = torch.zeros(2, dtype=torch.float64, device="cuda")
    s.stable_dt(u0, params, clock)
    dt1 = float(clock[1])
    s.stable_dt(u0, params_obs, clock)
    dt = min(dt1, float(clock[1]))
    h = [(cfg["hi"][d] - cfg["lo"][d]) / cfg["cells"][d] for d in range(3)]
    rc = np.floor((cfg["receivers"] - np.array(cfg["lo"])) / np.array(h)).astype(np.int64)
    cellsr = torch.as_tensor(rc[:, 0] + cfg["cells"][0] * (rc[:, 1] + cfg["cells"][1] * rc[:, 2]),
                             device="cuda")
    if grad:
        with torch.no_grad():
            samp = seismograms(s, u0, params_obs, dt, steps)
            data = samp[:, :, 6:9] / params_obs[cellsr, 0][None, :, None]

    def grad_once(ev):
        m = params.clone().requires_grad_(True)
        u = u0.clone().requires_grad_(True)
        sm = seismograms(s, u, m, dt, steps, every=ev)
        v = sm[:, :, 6:9] / m[cellsr, 0][None, :, None]
        J = 0.5 * dt * ((v - data) ** 2).sum()
        J.backward()
        return J, u.grad, m.grad

    el = el_all = J = gm = same = None
    if grad:
        grad_once(every)
        torch.cuda.synchronize()
        runs = []  # three timed gradients; the median is reported
        for _ in range(3):
            t0 = time.perf_counter()
            J, gu, gm = grad_once(every)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
        el = float(np.median(runs))
        # the same gradient with a checkpoint at every step (segments of one
        # step: no state is advanced twice except to keep the adjoint's inputs)
        t1 = time.perf_counter()
        J1, _, gm1 = grad_once(1)
        torch.cuda.synchronize()
        el_all = time.perf_counter() - t1
        same = bool(torch.equal(gm1, gm))
    # one forward step and one adjoint step, timed with events on the stream
    stream = torch.cuda.current_stream()
    Q = torch.randn(s.state_shape, dtype=torch.float64, device="cuda")
    lam = torch.randn(s.state_shape, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(params)
    ck = torch.tensor([0.0, dt], dtype=torch.float64, device="cuda")
    keep = torch.empty(s.keep_size(), dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    reps = 10
    for _ in range(2):
        s.step_adjoint(Q, params, ck, lam, g)
        s.step_keep(Q, params, ck.clone(), keep)
        s.step_adjoint_kept(params, ck, keep, lam, g)
    ev[0].record(stream)
    for _ in range(reps):
        s.step(Q, params, ck.clone(), next_dt=False)
    ev[1].record(stream)
    for _ in range(reps):
        s.step_adjoint(Q, params, ck, lam, g)
    ev[2].record(stream)
    for _ in range(reps):
        s.step_keep(Q, params, ck.clone(), keep)
    ev[3].record(stream)
    for _ in range(reps):
        s.step_adjoint_kept(params, ck, keep, lam, g)
    ev[4].record(stream)
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1]) / reps
    adj_ms = ev[1].elapsed_time(ev[2]) / reps
    fwdk_ms = ev[2].elapsed_time(ev[3]) / reps
    adjk_ms = ev[3].elapsed_time(ev[4]) / reps
    nseg = -(-steps // every)
    res = {"s_per_grad": round(el, 4) if grad else None,
           "s_per_grad_runs": [round(x, 4) for x in runs] if grad else None,
           "s_per_grad_checkpoint_every_step": round(el_all, 4) if grad else None,
           "every_step_gradient_bitwise_equal": same, "steps": steps, "checkpoint_every": every,
           "checkpoints": nseg, "forward_step_ms": round(fwd_ms, 4),
           "adjoint_step_ms": round(adj_ms, 4),
           "forward_step_keeping_ms": round(fwdk_ms, 4), "adjoint_step_from_kept_ms": round(adjk_ms, 4),
           "J": float(J) if grad else None,
           "grad_norm_params": float(torch.linalg.vector_norm(gm)) if grad else None,
           "workload": "c4: 3-D elastic, N=3, 32^3 cells, 16 receivers, Ricker source, "
                       "misfit vs a +-5% perturbed material, FP64, dt frozen"}
    log(f"adjoint c4: {el if grad else float('nan'):.3f} s/grad (fwd step {fwd_ms:.3f} ms, "
        f"adjoint step {adj_ms:.3f} ms; keeping / from kept: {fwdk_ms:.3f} / {adjk_ms:.3f} ms)")
    return res


def elastic_c3(log, steps: int | None = None, cfl: float = 0.5):
    """C3: 3-D elastic N=4 on 48^3 cells, layered perturbed material, Ricker
    source, 32 receivers sampled after every step, fixed dt; FP64 (fused
    corrector/predictor run, and step by step) and the FP32 predictor, with
    the FP32 run's error against the FP64 run."""
    import torch
    from paper_1905_07987_amd import adg, inputs
    cfg = inputs.elastic_config("c3")
    steps = steps or cfg["steps"]
    params = torch.as_tensor(cfg["params"], device="cuda")
    res = {}
    out = {}
    for prec in ("fp64", "fp32"):
        s = adg.Solver(3, cfg["order"], "elastic", cfg["cells"], cfg["lo"], cfg["hi"], cfl=cfl,
                       precision=prec)
        s.set_point_sources([cfg["source"]])
        s.set_receivers(cfg["receivers"])
        dofs = s.ncells * s.S * 9

        def one_run(fused: bool):
            Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
            seis = torch.empty((steps, s.nrec, 9), dtype=torch.float64, device="cuda")
            clock = torch.zeros(2, dtype=torch.float64, device="cuda")
            s.stable_dt(Q, params, clock)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if fused:
                # fixed dt: corrector and next predictor fused in one kernel
                s.run(Q, params, clock, steps, seis)
            else:
                for n in range(steps):
                    s.step(Q, params, clock, next_dt=False)
                    s.sample_receivers(Q, seis[n])
            torch.cuda.synchronize()
            return time.perf_counter() - t0, Q, seis

        el, Q, seis = one_run(True)
        res[prec] = {"value": dofs * steps / el, "ms_per_step": round(el / steps * 1e3, 4)}
        el1, Q1, _ = one_run(False)
        res[prec]["step_by_step"] = {"value": dofs * steps / el1, "ms_per_step": round(el1 / steps * 1e3, 4)}
        res[prec]["fused_state_bitwise_equal"] = bool(torch.equal(Q, Q1))
        log(f"c3 {prec} step by step: {el1 / steps * 1e3:.3f} ms/step")
        out[prec] = (Q, seis)
        log(f"c3 {prec}: {el / steps * 1e3:.3f} ms/step, {dofs * steps / el:.3e} DoF/s")
        del s
    (Q64, s64), (Q32, s32) = out["fp64"], out["fp32"]
    res["fp32"]["rel_l2_state_vs_fp64"] = float(torch.linalg.vector_norm(Q32 - Q64) /
                                                torch.linalg.vector_norm(Q64))
    res["fp32"]["rel_l2_seismograms_vs_fp64"] = float(torch.linalg.vector_norm(s32 - s64) /
                                                      torch.linalg.vector_norm(s64))
    res["workload"] = (f"c3: 3-D elastic, N=4, 48^3 cells, layered +-10% material, Ricker source, "
                       f"32 receivers, {steps} steps, CFL_N {cfl}")
    return res


def ck_compare(log, which: str, cfl: float = 0.5):
    """The linear kernels' Cauchy-Kowalevski predictor (Table 1) against the
    Picard predictor on an elastic workload: FP64 fused runs with I = N (the
    CK time average), I = N + 1 (the default) and I = 3N + 1 (the exact
    element fixed point: for a linear PDE the Picard iteration is nilpotent
    after dN + 1 steps); ms/step, and the relative L2 of the final state and
    of the seismograms against I = 3N + 1."""
    import torch
    from paper_1905_07987_amd import adg, inputs
    cfg = inputs.elastic_config(which)
    N, steps = cfg["order"], cfg["steps"]
    params = torch.as_tensor(cfg["params"], device="cuda")
    runs = {}
    for I in (N, N + 1, 3 * N + 1):
        s = adg.Solver(3, N, "elastic", cfg["cells"], cfg["lo"], cfg["hi"], cfl=cfl, picard_iters=I)
        s.set_point_sources([cfg["source"]])
        s.set_receivers(cfg["receivers"])
        Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
        seis = torch.empty((steps, s.nrec, 9), dtype=torch.float64, device="cuda")
        clock = torch.zeros(2, dtype=torch.float64, device="cuda")
        s.stable_dt(Q, params, clock)
        s.reserve_run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(Q, params, clock, steps, seis)
        torch.cuda.synchronize()
        runs[I] = ((time.perf_counter() - t0) / steps * 1e3, Q, seis)
        del s
    ref = runs[3 * N + 1]
    res = {"workload": f"{which}: 3-D elastic, N={N}, {steps} steps, fused FP64 runs, CFL_N {cfl}"}
    for I, (ms, Q, seis) in runs.items():
        key = "ck_I_eq_N" if I == N else ("picard_I_eq_N+1" if I == N + 1 else "reference_I_eq_3N+1")
        res[key] = {"picard_iters": I, "ms_per_step": round(ms, 4),
                    "rel_l2_state_vs_reference": float(torch.linalg.vector_norm(Q - ref[1]) /
                                                       torch.linalg.vector_norm(ref[1])),
                    "rel_l2_seismograms_vs_reference": float(torch.linalg.vector_norm(seis - ref[2]) /
                                                             torch.linalg.vector_norm(ref[2]))}
        log(f"{which} I={I}: {ms:.3f} ms/step, state vs reference {res[key]['rel_l2_state_vs_reference']:.2e}")
    return res


def euler_c5(log, steps: int = 50, warmup: int = 2, cells: int = 96, order: int = 3, cfl: float = 0.5):
    """C5: the paper's spherical explosion (3-D Euler, N=3, 96^3 cells on
    [0,1]^3, reflecting walls) with the a-posteriori subcell limiter: every
    step is adg_step_limited with Eq. (7) for the next step.  Reports the
    rate, the limiter's cell counts, and the change of total mass and energy
    over the run (conserved by the scheme)."""
    import torch
    from paper_1905_07987_amd import adg, inputs
    C = cells ** 3
    s = adg.Solver(3, order, "euler", [cells] * 3, bc=["wall"] * 6, cfl=cfl)
    xyz = s.node_coords()
    Q = torch.as_tensor(inputs.blast_state(xyz), device="cuda")
    del xyz
    fv, subfv = inputs.blast_fv_cells([cells] * 3, [0.0] * 3, [1.0] * 3, order)
    sin = torch.zeros(s.subcell_shape, dtype=torch.float64, device="cuda")
    fv_d = torch.as_tensor(fv, device="cuda")
    sin[fv_d] = torch.as_tensor(subfv, device="cuda")
    sout = torch.zeros_like(sin)
    status = torch.zeros(C, dtype=torch.uint8, device="cuda")
    status[fv_d] = 3
    counts = torch.zeros(3, dtype=torch.int32, device="cuda")
    clock = torch.zeros(2, dtype=torch.float64, device="cuda")
    w = torch.as_tensor(adg.basis_tables(order)["w"], device="cuda")
    wk = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)

    def totals(Q, sub, status):
        per = (Q * wk).sum(dim=2)
        fvm = status >= 2
        per[fvm] = sub[fvm].mean(dim=2)
        return per.sum(dim=0) / C

    m0 = totals(Q, sin, status)
    s.stable_dt(Q, None, clock)
    # a run of limited steps: each step takes its DG cells' t^n ranges from
    # the previous step's candidate (bitwise the same results)
    for _ in range(warmup):
        s.step_limited(Q, clock, sin, sout, status, counts, next_dt=True, reuse_ranges=True)
        sin, sout = sout, sin
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        s.step_limited(Q, clock, sin, sout, status, counts, next_dt=True, reuse_ranges=True)
        sin, sout = sout, sin
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    m1 = totals(Q, sin, status)
    c = counts.cpu().tolist()
    t, _ = s.read_clock(clock)
    dofs = C * (order + 1) ** 3 * 5
    res = {"value": dofs / (ms * 1e-3), "ms_per_step": round(ms, 4),
           "troubled_fv_dg_with_fv_face": c, "fv_fraction": round(c[1] / C, 5),
           "mass_rel_change": float((m1[0] - m0[0]) / m0[0]),
           "energy_rel_change": float((m1[4] - m0[4]) / m0[4]), "t_end": t,
           "workload": (f"c5: 3-D Euler N={order}, {cells}^3 cells, reflecting walls, spherical explosion "
                        f"(seed 7991), subcell limiter, {warmup} + {steps} steps, CFL_N {cfl}")}
    log(f"c5 limited: {ms:.3f} ms/step, {res['value']:.3e} DoF/s, counts {c}, "
        f"mass {res['mass_rel_change']:.1e}, energy {res['energy_rel_change']:.1e}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=64)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision variant")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the C4 adjoint gradient")
    ap.add_argument("--no-elastic", action="store_true", help="skip the C3 elastic variant")
    ap.add_argument("--no-limiter", action="store_true", help="skip the C5 limited explosion")
    ap.add_argument("--no-grad", action="store_true",
                    help="C4: time single forward/adjoint steps only, no misfit gradients")
    ap.add_argument("--cpu-cells", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain elementwise copy of the state (known HBM bytes) "
                         "so counter-based traffic can be scaled")
    ap.add_argument("--cfl", type=float, default=0.5,
                    help="CFL_N of Eq. (7); 0.5 = 0.9 x the linear stability limit at N = 5")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not an implemented path"}))
        sys.exit(2)

    import torch
    from paper_1905_07987_amd import adg, inputs

    N, m = args.order, args.cells
    nvar = 5
    dofs = m ** 3 * (N + 1) ** 3 * nvar

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    log(f"workload c2: 3-D Euler N={N}, {m}^3 cells, {dofs} DoFs")
    s = adg.Solver(3, N, "euler", [m, m, m], precision=args.precision, cfl=args.cfl)
    xyz = s.node_coords()
    Q0 = inputs.c2_state(xyz)
    del xyz
    Q0d = torch.as_tensor(Q0, device="cuda")
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        # two copies of known size: the runtime's buffer copy (clone) and an
        # elementwise kernel, each reading and writing the state once
        calib = Q0d.clone()
        calib2 = Q0d.mul(1.0)
        torch.cuda.synchronize()
        log(f"copy calibration: {calib.numel() * 8} bytes read and written by each copy")
        del calib, calib2

    def run(solver, steps, warmup, time_kernels=True):
        Q = Q0d.clone()
        clock = torch.zeros(2, dtype=torch.float64, device="cuda")
        solver.stable_dt(Q, None, clock)
        for _ in range(warmup):
            solver.step(Q, None, clock, next_dt=True)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        t0 = time.perf_counter()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for i in range(steps):
            ev[2 * i].record(stream)
            solver.predict(Q, None, clock, Q)         # kernel A
            ev[2 * i + 1].record(stream)
            solver.correct(Q, None, clock, next_dt=True)  # kernel B
        ev[2 * steps].record(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        total_ms = start.elapsed_time(stop)
        pred = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)]
        corr = [ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(steps)]
        return Q, clock, total_ms, wall, float(np.mean(pred)), float(np.mean(corr))

    Q64, clock64, total_ms, wall, pred_ms, corr_ms = run(s, args.steps, args.warmup)
    ms_per_step = total_ms / args.steps
    value = dofs / (ms_per_step * 1e-3)
    log(f"fp64: {ms_per_step:.3f} ms/step (predict {pred_ms:.3f}, correct {corr_ms:.3f}), "
        f"wall {wall:.2f} s, {value:.3e} DoF/s")

    flops_cell = predictor_flops_per_cell(3, N, nvar, N + 1, euler_flux_flops(3))
    flops_launch = flops_cell * m ** 3
    achieved = flops_launch / (pred_ms * 1e-3) / 1e12
    traffic = read_traffic("c2")
    # the FP32 and split-BF16 predictors compute in FP32 vector arithmetic
    # (the latter with its derivatives on the matrix cores)
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_FP32_TFLOPS
    kname = {"fp64": f"predict_kernel_n64<Euler<3>,{N}>", "fp32": f"predict_kernel_node<Euler<3>,{N},float,false>",
             "bf16x3": f"predict_kernel_node<Euler<3>,{N},float,true>"}[args.precision]
    if args.precision != "fp64":
        traffic = None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": traffic, "kernel": kname,
                "flops_per_launch": flops_launch, "ms_per_launch": round(pred_ms, 4)}

    variants = {"correct_kernel_ms": round(corr_ms, 4)}
    variants["c1"] = euler_c1(log)
    if not args.no_mixed and args.precision == "fp64":
        s32 = adg.Solver(3, N, "euler", [m, m, m], precision="fp32", cfl=args.cfl)
        Q32, clock32, t32, _, p32, c32 = run(s32, args.steps, args.warmup)
        err = float(torch.linalg.vector_norm(Q32 - Q64) / torch.linalg.vector_norm(Q64))
        v32 = dofs / (t32 / args.steps * 1e-3)
        variants["mixed_fp32"] = {"value": v32, "ms_per_step": round(t32 / args.steps, 4),
                                  "predict_ms": round(p32, 4),
                                  "rel_l2_vs_fp64_after_steps": err,
                                  "steps_compared": args.warmup + args.steps}
        log(f"mixed fp32: {t32 / args.steps:.3f} ms/step, {v32:.3e} DoF/s, rel L2 vs fp64 {err:.2e}")

    if not args.no_mixed and args.precision == "fp64":
        sb = adg.Solver(3, N, "euler", [m, m, m], precision="bf16x3", cfl=args.cfl)
        Qb, clockb, tb, _, pb, cb = run(sb, args.steps, args.warmup)
        errb = float(torch.linalg.vector_norm(Qb - Q64) / torch.linalg.vector_norm(Q64))
        variants["mixed_bf16x3"] = {"value": dofs / (tb / args.steps * 1e-3),
                                    "ms_per_step": round(tb / args.steps, 4), "predict_ms": round(pb, 4),
                                    "rel_l2_vs_fp64_after_steps": errb,
                                    "steps_compared": args.warmup + args.steps}
        log(f"mixed bf16x3: {tb / args.steps:.3f} ms/step (predict {pb:.3f}), rel L2 vs fp64 {errb:.2e}")
        del sb, Qb

    if args.precision == "fp64":
        # the CERK initial guess with N - 2 Picard passes (same order as
        # N + 1 passes from the constant guess)
        sc = adg.Solver(3, N, "euler", [m, m, m], cfl=args.cfl, initial_guess="cerk")
        Qc, clockc, tc, _, pc, cc = run(sc, args.steps, args.warmup)
        errc = float(torch.linalg.vector_norm(Qc - Q64) / torch.linalg.vector_norm(Q64))
        variants["cerk_guess"] = {"value": dofs / (tc / args.steps * 1e-3),
                                  "ms_per_step": round(tc / args.steps, 4), "predict_ms": round(pc, 4),
                                  "picard_iters": max(1, N - 2),
                                  "rel_l2_vs_constant_guess_after_steps": errc,
                                  "steps_compared": args.warmup + args.steps}
        log(f"cerk guess: {tc / args.steps:.3f} ms/step (predict {pc:.3f}), rel L2 vs constant guess {errc:.2e}")
        del sc, Qc

    if not args.no_elastic:
        variants["elastic_c3"] = elastic_c3(log)
        variants["ck_vs_picard_c3"] = ck_compare(log, "c3")
        variants["ck_vs_picard_c4"] = ck_compare(log, "c4")
    if not args.no_adjoint:
        variants["adjoint_c4"] = adjoint_c4(log, grad=not args.no_grad)
    if not args.no_limiter:
        variants["limiter_c5"] = euler_c5(log)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_cells, N)
        log(f"cpu baseline {cpu['value']:.3e} DoF/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC, "value": value, "unit": "DoF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32-predictor/f64-update",
                  "bf16x3": "bf16x3-mfma-predictor/f64-update"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"c2: 3-D Euler, N={N}, {m}^3 periodic cells, seeded 8-mode Fourier "
                               f"state, CFL_N {args.cfl}, {args.precision}",
                   "dofs_per_step": dofs, "picard_iters": N + 1},
        "roofline": roofline, "cpu_baseline": cpu, "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
