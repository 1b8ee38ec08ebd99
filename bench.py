"""Throughput of the per-cell thermochemistry hot path on one MI355X.

One step runs the whole hot path over a batch of cells already resident in
HBM: the Newton inversion T(e, Y) from a 1200 K guess, then one reverse-sweep
launch that computes the net production rates omega(rho, T, Y) at that
temperature and the reverse-mode product of L = sum wbar omega (gradients
with respect to Y, T and every Arrhenius triple), on the 53-species,
325-reaction synthetic mechanism (2^22 cells by default).  The figure of
merit is million cells per second (higher is better).

Prints one JSON line with, besides the throughput, roofline entries for the
reverse-sweep kernel ("roofline") and for the production-rate kernel alone,
timed after the steps ("roofline_other"): algorithmic FP64 flops per launch
over the average launch time, timed with HIP events on the stream they run
on; and the CPU oracle timed on a bounded sample of the same workload.

"large_mechanism" times the production rates of the 160-species,
900-reaction mechanism on 2^20 cells.  "surrogate" reports the learned
surrogate on the 53-species mechanism: its training on exact-kernel labels,
and for each target error the calibrated thresholds, the fallback fraction,
the error percentiles against the exact kernel and the speed against the
exact kernel alone.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cells N]
                       [--no-cpu-baseline] [--cpu-sample N] [--no-surrogate] [--no-large]
                       [--train-states N] [--members E] [--hidden H]
                       [--epochs K] [--batch B] [--lr LR] [--targets ...]
"""

import argparse
import json
import math
import os
import platform
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

MECH = os.path.join(REPO, "mechanisms", "cfg1.pyromech")
PEAK_FP64_TFLOPS = 78.6          # MI355X FP64 vector peak
PEAK_HBM_GBS = 8000.0
EXP_FLOPS = 20                   # convention for one exp or log


def wdot_flops_per_cell(gm):
    """Algorithmic flops of omega for one cell: S(2+20+22) + R(4+2+1+40)
    + 2 nnz(nu') + 2 nnz(nu'') + 4 nnz(nu) + 2 n_pd S + 128 n_fo + 30
    (exp and log count as 20 flops)."""
    S, R = gm.n_species, gm.n_reactions
    n_pd = gm.n_third_body + gm.n_falloff
    return (S * (2 + EXP_FLOPS + 22) + R * (4 + 2 + 1 + 2 * EXP_FLOPS)
            + 2 * gm.nnz_reactant + 2 * gm.nnz_product + 4 * gm.nnz_net
            + 2 * n_pd * gm.n_species + 128 * gm.n_falloff + 30)


def vjp_flops_per_cell(gm):
    """Algorithmic flops of the reverse sweep for one cell: the forward
    recomputation plus 2 nnz for nu^T wbar, 15 per reaction for the local
    adjoints, 4 nnz for the species sums, 6 per Arrhenius triple for the cell
    sums, 2 n_pd S for the third-body contraction, 12 S for the enthalpy
    terms and 150 per falloff reaction for the broadening-factor derivatives."""
    S, R = gm.n_species, gm.n_reactions
    nnz = gm.nnz_reactant + gm.nnz_product
    n_pd = gm.n_third_body + gm.n_falloff
    return (wdot_flops_per_cell(gm) + 2 * nnz + 15 * R + 4 * nnz + 6 * gm.n_params
            + 2 * n_pd * S + 12 * S + 150 * gm.n_falloff)


def fused_flops_per_cell(gm):
    """The reverse sweep that also returns omega: its flops plus 2 nnz(nu)
    for the sums nu q."""
    return vjp_flops_per_cell(gm) + 2 * gm.nnz_net


def fused_bytes_per_cell(gm):
    """Compulsory HBM bytes of the reverse sweep with omega per cell: read
    rho, T, Y, wbar; write Ybar, Tbar, omega."""
    return 8 * (3 + 4 * gm.n_species)


def wdot_bytes_per_cell(gm):
    """Compulsory HBM bytes of omega per cell: read rho, T, Y; write omega."""
    return 8 * (2 + 2 * gm.n_species)


def _oracle_chunk(task):
    """One worker's share of the CPU baseline: draws its cells (untimed), then
    times the oracle on them.  Returns (seconds of Newton + omega, cells,
    seconds of the complex-step VJP, cells)."""
    first_fwd, n_fwd, first_vjp, n_vjp, cfg = task
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import eos, gradients, kinetics, mechfile, newton, thermo
    from pyro_synth.states import draw_cotangent, draw_states
    with threadpool_limits(1):
        m = mechfile.load(MECH)
        T, p, Y = draw_states(cfg, n_fwd, m.S, first=first_fwd)
        rho = eos.density(m, p, T, Y)
        e = thermo.mixture_internal_energy(m, T, Y)
        t0 = time.perf_counter()
        Tn, st = newton.temperature(m, e, Y, 1200.0)
        w = kinetics.net_production_rates(m, rho, Tn, Y)
        t_fwd = time.perf_counter() - t0
        assert np.isfinite(w).all()
        T, p, Y = draw_states(cfg, n_vjp, m.S, first=first_vjp)
        rho = eos.density(m, p, T, Y)
        wbar = draw_cotangent(2, first_vjp + n_vjp, m.S)[:, first_vjp:]
        t0 = time.perf_counter()
        gradients.vjp(m, rho, T, Y, wbar)
        t_vjp = time.perf_counter() - t0
    return t_fwd, n_fwd, t_vjp, n_vjp


def host_cores():
    """Cores this process may run on, capped at the 16 a one-GPU share of
    the host provides."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(n_fwd_per_core, n_vjp_per_core, cfg=1, cores=None):
    """The oracle (NumPy, each worker one thread) on consecutive cells of the
    same workload, one forked worker process per host core: Newton from
    1200 K and omega on ``n_fwd_per_core`` cells per worker, the complex-step
    gradients on ``n_vjp_per_core`` cells per worker.  The parallel rate is
    the total cells over the slowest worker's time, per part; the parts' per-
    cell times add up to one step.  The same per-worker sample run alone
    gives the one-thread rate.  Must run before the GPU is touched (workers
    are forked)."""
    import multiprocessing as mp
    cores = cores or host_cores()
    tasks = [(i * n_fwd_per_core, n_fwd_per_core, i * n_vjp_per_core, n_vjp_per_core, cfg)
             for i in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_chunk, tasks, chunksize=1)
    t_fwd = max(r[0] for r in res)
    t_vjp = max(r[2] for r in res)
    rate = 1e-6 / (t_fwd / (cores * n_fwd_per_core) + t_vjp / (cores * n_vjp_per_core))
    one = _oracle_chunk(tasks[0])
    rate1 = 1e-6 / (one[0] / one[1] + one[2] / one[3])
    return {"value": round(rate, 6), "unit": "Mcells/s", "cores": cores,
            "kind": "oracle", "one_thread_value": round(rate1, 6),
            "host": {"nproc": os.cpu_count(), "cores_used": cores, "cpu_model": cpu_model()},
            "sample": f"consecutive cells of the 2^22-cell workload, {cores} worker processes "
                      f"of one thread each: Newton + omega on {cores} x {n_fwd_per_core} cells "
                      f"({t_fwd:.1f} s wall), complex-step VJP on {cores} x {n_vjp_per_core} "
                      f"cells ({t_vjp:.1f} s wall); one worker alone: {one[0]:.1f} s + "
                      f"{one[2]:.1f} s"}


TRAFFIC_PROFILE = os.path.join(REPO, "profiles", "traffic_cfg1_2e22.md")


def measured_traffic():
    """HBM bytes per launch of each kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by their readings for a copy of known
    size), kept only while the kernel's source still has the hash recorded
    with the measurement."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return {}
    start = text.find("<!-- traffic ")
    if start < 0:
        return {}
    data = json.loads(text[start + len("<!-- traffic "):text.index(" -->", start)])
    out = {}
    for kernel, rec in data.items():
        src = os.path.join(REPO, rec["source"])
        try:
            digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        except OSError:
            continue
        if digest == rec["sha256"]:
            out[kernel] = rec["fetch_bytes"] + rec["write_bytes"]
    return out


def _time_ms(fn, reps, stream):
    """Average time of fn() over reps launches, timed with HIP events on
    the stream the kernels run on."""
    import torch
    fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def fp32_leg(gm, rho, T, Y, stream, reps):
    """The FP32 production rates (log-space form in float) on the same cells:
    time, the fraction of cells with a non-finite result (a rate beyond the
    float range), and the per-cell normwise error of the finite ones against
    the FP64 kernel on the same float-rounded inputs (the FP64 kernel matches
    the oracle to 1e-12)."""
    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    r32, t32, y32 = rho.float(), T.float(), Y.float()
    w32 = torch.empty_like(y32)
    ms = _time_ms(lambda: pyro.production_rates(gm, r32, t32, y32, out=w32), reps, stream)
    w64 = pyro.production_rates(gm, r32.double(), t32.double(), y32.double())
    finite = torch.isfinite(w32).all(dim=0)
    diff = torch.linalg.vector_norm(w32.double() - w64, dim=0)
    ref = torch.linalg.vector_norm(w64, dim=0)
    err = (diff / torch.where(ref > 0, ref, torch.ones_like(ref)))[finite].cpu().numpy()
    over = 1.0 - float(finite.double().mean())
    n = Y.shape[1]
    del r32, t32, y32, w32, w64
    q = lambda x: float(np.quantile(err, x)) if err.size else None  # noqa: E731
    return {"ms": round(ms, 4), "Mcells_s": round(n / (ms * 1e-3) / 1e6, 3),
            "overflow_fraction": round(over, 6),
            "normwise_err_vs_fp64": {"p50": q(0.5), "p99": q(0.99), "p99.9": q(0.999),
                                     "max": float(err.max()) if err.size else None},
            "note": "log-space form in float; overflowing cells have a rate beyond the float "
                    "range (config-1 rates reach ~1e69)"}


def jacobian_leg(args, log):
    """The chemical Jacobian dS/dY at fixed density and energy on the first
    ``--jacobian-cells`` cells of the same workload (S reverse sweeps with a
    unit cotangent per row): time and throughput."""
    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from pyro_synth.states import draw_states
    gm = pyro.Mechanism(MECH)
    n = args.jacobian_cells
    T, p, Y = draw_states(1, n, gm.n_species)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T_d, p_d, Y_d = dev(T), dev(p), dev(Y)
    rho = pyro.density(gm, p_d, T_d, Y_d)
    S = gm.n_species
    J = torch.empty((S, S, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ms = _time_ms(lambda: pyro.chemical_jacobian(gm, rho, T_d, Y_d, out=J), 3, stream)
    ok = bool(torch.isfinite(J).all())
    del J
    gm.close()
    torch.cuda.empty_cache()
    log(f"jacobian: {n} cells in {ms:.2f} ms")
    out_bytes = 8 * S * S + 8 * (2 + S)
    return {"workload": f"53-species mechanism, {n} cells, fixed density and internal energy",
            "ms": round(ms, 3), "Mcells_s": round(n / (ms * 1e-3) / 1e6, 3), "finite": ok,
            "hbm_GBps_compulsory": round(out_bytes * n / (ms * 1e-3) / 1e9, 1),
            "method": "S reverse sweeps, unit cotangent W_j on species j per row, each row on "
                      "a schedule of its own reactions (nonzero net coefficient of j)"}


def other_rows_leg(args, log):
    """The remaining per-cell kernels on the 53-species workload: Newton
    inversion from the enthalpy and primitive variables from conserved ones
    (2^22 cells, HBM-bound: algorithmic bytes = inputs read + outputs
    written), mixture-averaged transport (2^20 cells, ALU-bound: about 2 S^2
    pair updates per cell) and one reactor step, RK4 (2^20 cells) and
    Crank-Nicolson with Newton on the fixed-energy Jacobian (2^18 cells).
    The steps are per cell, from the cell's fastest chemical time
    tau = min_k max(Y_k, 1e-3) / |dY_k/dt|: 0.05 tau for RK4 and tau for
    Crank-Nicolson.  (A fixed step suits no draw of these far-from-equilibrium
    states: at 1e-8 s Newton diverges in most cells, in the oracle as well.)"""
    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from pyro_synth.states import draw_states
    from pyro_synth.transport import draw_transport
    gm = pyro.Mechanism(MECH)
    S = gm.n_species
    stream = torch.cuda.current_stream()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    out = {}
    n = args.cells
    T, p, Y = (dev(x) for x in draw_states(1, n, S))
    rho = pyro.density(gm, p, T, Y)
    e = pyro.internal_energy(gm, T, Y)
    h = e + p / rho
    reps = max(args.steps, 3)
    ms = _time_ms(lambda: pyro.temperature_from_enthalpy(gm, h, Y), reps, stream)
    b = 8 * (1 + S) + 8 + 4
    out["temperature_from_enthalpy"] = {
        "cells": n, "ms": round(ms, 4), "Mcells_s": round(n / (ms * 1e-3) / 1e6, 1),
        "bytes_per_cell": b, "hbm_GBps": round(b * n / (ms * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "peak": 8000.0, "unit": "GB/s",
                     "frac": round(b * n / (ms * 1e-3) / 8e12, 3)}}
    rk = rho * Y
    mom = torch.randn((3, Y.stride(0)), dtype=torch.float64, device="cuda")[:, :n] * rho
    E = rho * e + 0.5 * (mom * mom).sum(0) / rho
    ms = _time_ms(lambda: pyro.primitive_from_conserved(gm, rk, mom, E), reps, stream)
    b = 8 * (S + 3 + 1) + 8 * (1 + S + 3 + 2) + 4
    out["primitive_from_conserved"] = {
        "cells": n, "dim": 3, "ms": round(ms, 4), "Mcells_s": round(n / (ms * 1e-3) / 1e6, 1),
        "bytes_per_cell": b, "hbm_GBps": round(b * n / (ms * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "peak": 8000.0, "unit": "GB/s",
                     "frac": round(b * n / (ms * 1e-3) / 8e12, 3)}}
    del rk, mom, E, h
    n2 = 1 << 20
    T2, Y2, rho2, e2 = T[:n2].clone(), Y[:, :n2].contiguous(), rho[:n2].clone(), e[:n2].clone()
    del T, p, Y, rho, e
    tr = pyro.Transport(gm, *draw_transport(S))
    ms = _time_ms(lambda: pyro.mixture_transport(gm, tr, T2, Y2), reps, stream)
    out["mixture_transport"] = {"cells": n2, "ms": round(ms, 4),
                                "Mcells_s": round(n2 / (ms * 1e-3) / 1e6, 1),
                                "pair_updates_per_cell": 2 * S * S}
    W = torch.tensor(gm.molecular_weights, dtype=torch.float64, device="cuda")

    def chem_time(r, Tc, Yc):
        f = (W[:, None] * pyro.production_rates(gm, r, Tc, Yc) / r).abs()
        t = torch.where(f > 0, Yc.clamp(min=1e-3) / f, torch.full_like(f, float("inf")))
        return t.min(0).values

    tau2 = chem_time(rho2, T2, Y2)
    dt_rk = (0.05 * tau2).contiguous()
    Ys, Ts = Y2.clone(), T2.clone()
    ms = _time_ms(lambda: (Ys.copy_(Y2), Ts.copy_(T2),
                           pyro.reactor_step(gm, "rk4", rho2, e2, Ys, Ts, dt_rk)), 3, stream)
    out["reactor_rk4_step"] = {"cells": n2, "dt": "0.05 tau per cell",
                               "dt_median_s": float(dt_rk.median()), "ms": round(ms, 3),
                               "Mcells_s": round(n2 / (ms * 1e-3) / 1e6, 2),
                               "note": "four stages of Newton T(e), production rates and the "
                                       "stage update; includes restoring the state per step"}
    n3 = 1 << 18
    Y3, T3, r3, e3 = (Y2[:, :n3].contiguous(), T2[:n3].clone(), rho2[:n3].clone(),
                      e2[:n3].clone())
    dt_cn = tau2[:n3].contiguous()
    Yc, Tc = Y3.clone(), T3.clone()
    st = pyro.reactor_step(gm, "cn", r3, e3, Yc, Tc, dt_cn)
    iters = st.cpu().numpy()
    ms = _time_ms(lambda: (Yc.copy_(Y3), Tc.copy_(T3),
                           pyro.reactor_step(gm, "cn", r3, e3, Yc, Tc, dt_cn)), 3, stream)
    hist = np.bincount(np.abs(iters), minlength=21)
    out["reactor_cn_step"] = {"cells": n3, "dt": "tau per cell",
                              "dt_median_s": float(dt_cn.median()), "ms": round(ms, 3),
                              "Mcells_s": round(n3 / (ms * 1e-3) / 1e6, 3),
                              "newton_updates_max": int(np.abs(iters).max()),
                              "newton_updates_histogram": hist.tolist(),
                              "converged_fraction": float((iters > 0).mean()),
                              "note": "per Newton update: T, production rates, the 53-row "
                                      "fixed-energy Jacobian and the LU solve (one cell per "
                                      "wavefront)"}
    gm.close()
    torch.cuda.empty_cache()
    log("other rows: " + ", ".join(f"{k} {v['ms']} ms" for k, v in out.items()))
    return out


def large_mechanism_leg(args, log):
    """The 160-species, 900-reaction mechanism (2^20 cells, states drawn as
    for the 53-species workload): production rates alone, with the kernel
    variant the loader selects (its species rows do not fit the LDS tile)."""
    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from paper_2503_24286_amd import _lib
    from paper_2503_24286_amd import surrogate as sur

    gm = pyro.Mechanism(os.path.join(REPO, "mechanisms", "cfg3.pyromech"))
    n = 1 << 20
    T = np.empty(n)
    p = np.empty(n)
    Y = np.empty((gm.n_species, n))
    for a, Tc, pc, Yc in sur.draw_chunks(3, n, gm.n_species, None, threads=args.threads):
        T[a:a + Tc.shape[0]], p[a:a + Tc.shape[0]], Y[:, a:a + Tc.shape[0]] = Tc, pc, Yc
    Td, pd, Yd = (torch.from_numpy(x).cuda() for x in (T, p, Y))
    rho = pyro.density(gm, pd, Td, Yd)
    w = torch.empty_like(Yd)
    stream = torch.cuda.current_stream()
    ms = _time_ms(lambda: pyro.production_rates(gm, rho, Td, Yd, out=w), args.reps, stream)
    if not bool(torch.isfinite(w).all()):
        raise RuntimeError("non-finite rates on the large mechanism")
    # the third-body concentrations (a dense contraction) on the FP64 matrix
    # cores instead of the FMA units
    base = gm.wdot_variant
    try:
        gm.wdot_variant = base | _lib.PYRO_WDOT_MFMA_THIRD_BODY
        ms_mfma = _time_ms(lambda: pyro.production_rates(gm, rho, Td, Yd, out=w), args.reps, stream)
    except _lib.PyroError:   # its [M] block does not fit beside this mechanism's tile
        ms_mfma = None
    # the net rates omega = nu q on the FP64 matrix cores (dense nu, ten
    # 16-species blocks) instead of the sparse gathering
    try:
        gm.wdot_variant = base | _lib.PYRO_WDOT_MFMA_NET_RATES
        ms_nq = _time_ms(lambda: pyro.production_rates(gm, rho, Td, Yd, out=w), args.reps, stream)
        if not bool(torch.isfinite(w).all()):
            raise RuntimeError("non-finite rates on the large mechanism (MFMA net rates)")
    except _lib.PyroError:
        ms_nq = None
    gm.wdot_variant = base
    fpc = wdot_flops_per_cell(gm)
    achieved = fpc * n / (ms * 1e-3) / 1e12
    out = {"workload": f"{gm.n_species}-species {gm.n_reactions}-reaction synthetic mechanism, "
                       f"{n} cells", "variant": "reaction-equilibrium" if gm.wdot_variant
                       else "species-equilibrium",
           "ms": round(ms, 4), "Mcells_s": round(n / ms / 1e3, 3), "flops_per_cell": fpc,
           "third_body_on_mfma_ms": None if ms_mfma is None else round(ms_mfma, 4),
           "net_rates_on_mfma_ms": None if ms_nq is None else round(ms_nq, 4),
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4)}}
    log(f"large mechanism: {out['Mcells_s']} Mcells/s")
    gm.close()
    return out


def surrogate_leg(args, log):
    """Config-4 surrogate: train an ensemble on exact-kernel labels of
    ``--train-states`` seeded states with the library's own BF16 kernels,
    calibrate the fallback thresholds on 2^20 held-out states for each
    target error, then evaluate on ``--cells`` fresh states, errors measured
    against the exact kernel."""
    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from paper_2503_24286_amd import surrogate as sur
    from pyro_synth.configs import SEEDS

    gm = pyro.Mechanism(MECH)
    stream = torch.cuda.current_stream()
    S = gm.n_species
    t0 = time.time()
    data, norm = sur.build_dataset(gm, args.train_states, SEEDS["surrogate_train"],
                                   threads=args.threads, log=log)
    t_data = time.time() - t0
    trainers, hist = [], []
    t1 = time.time()
    for e in range(args.members):
        tr, h = sur.train_member(data, args.hidden, sur.INIT_SEED + e, args.epochs, args.batch,
                                 lr=args.lr, log=log)
        trainers.append(tr)
        hist.append(h)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    del data
    model = sur.Surrogate.from_trainers(trainers, norm)
    del trainers
    torch.cuda.empty_cache()

    def draw(n, seed, cfg=4):
        T = np.empty(n)
        p = np.empty(n)
        Y = np.empty((S, n))
        for a, Tc, pc, Yc in sur.draw_chunks(cfg, n, S, seed, threads=args.threads):
            T[a:a + Tc.shape[0]] = Tc
            p[a:a + Tc.shape[0]] = pc
            Y[:, a:a + Tc.shape[0]] = Yc
        return T, p, Y

    # calibration on held-out states, errors measured against the exact kernel
    Th, ph, Yh = draw(1 << 20, SEEDS["surrogate_heldout"])
    Td, pd, Yd = (torch.from_numpy(x).cuda() for x in (Th, ph, Yh))
    rho, w_ex = sur.label(gm, Td, pd, Yd)
    w_s, _, _, ind = model.eval(gm, rho, Td, Yd, indicators=True)
    err, d2, r2 = sur.cell_errors(w_s.cpu().numpy(), w_ex.cpu().numpy())
    ind = ind.cpu().numpy()
    held_out = {"p50": float(np.median(err)), "p99": float(np.percentile(err, 99)),
                "p99.9": float(np.percentile(err, 99.9))}
    thresholds = {t: sur.calibrate(ind[0], ind[1], err, d2, r2, target=t)
                  for t in args.targets}
    del Td, pd, Yd, rho, w_ex, w_s
    log(f"surrogate: held-out errors {held_out}; thresholds {thresholds}")

    # evaluation workload: fresh config-4 states
    n = args.cells
    Td, pd, Yd = (torch.from_numpy(x).cuda() for x in draw(n, SEEDS["states"] + 4))
    rho = pyro.density(gm, pd, Td, Yd)
    w_ex = pyro.production_rates(gm, rho, Td, Yd)
    out = torch.empty_like(w_ex)
    ms_exact = _time_ms(lambda: pyro.production_rates(gm, rho, Td, Yd, out=out), args.reps,
                        stream)
    # the surrogate without fallback (thresholds infinite: network, inverse
    # transform, indicators, no exact cell) and the network's member outputs
    # alone (features and the four layers of every member)
    ms_mlp = _time_ms(lambda: model.eval(gm, rho, Td, Yd, thr_spread=math.inf,
                                         thr_resid=math.inf, out=out), args.reps, stream)
    ms_net = _time_ms(lambda: model.outputs(gm, rho, Td, Yd), args.reps, stream)
    ref_norm = torch.sqrt((w_ex * w_ex).sum(0))
    r2_sum = float((ref_norm.double() ** 2).sum())
    curve = []
    for target in args.targets:
        ts, tr, frac_cal = thresholds[target]
        w_s, flags, count, _ = model.eval(gm, rho, Td, Yd, thr_spread=ts, thr_resid=tr, out=out)
        d = torch.sqrt(((w_s - w_ex) ** 2).sum(0))
        e = (d / ref_norm.clamp_min(1e-300)).cpu().numpy()
        frob = math.sqrt(float((d.double() ** 2).sum()) / r2_sum)
        frac = int(count.item()) / n
        ms = _time_ms(lambda: model.eval(gm, rho, Td, Yd, thr_spread=ts, thr_resid=tr, out=out),
                      args.reps, stream)
        # a threshold that admits no cell makes the call the exact kernel on
        # every cell (the network is not run): no surrogate gain to report
        admits = ts > 0 and tr > 0
        row = {"target": target, "thr_spread": ts, "thr_resid": tr,
               "fallback_fraction": round(frac, 5), "fallback_fraction_heldout": round(frac_cal, 5),
               "ms": round(ms, 4), "Mcells_s": round(n / ms / 1e3, 3),
               "gain_vs_exact": round(ms_exact / ms, 4) if admits else None,
               "note": None if admits else "no admissible cell at this target: every cell "
                                           "falls back, the network is not run, gain n/a",
               "err": {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
                       "p99.9": float(np.percentile(e, 99.9)), "max": float(e.max()),
                       "frobenius": frob}}
        curve.append(row)
        log(f"surrogate: target {target}: fallback {frac:.4f}, {ms:.3f} ms, "
            f"gain {ms_exact / ms:.3f}" + ("" if admits else " (no admissible cell)"))
    main_row = curve[0]
    gm.close()
    net_flops = 2 * args.members * sum(a * b for a, b in sur.layer_dims(args.hidden))
    return {
        "workload": f"53-species mechanism; ensemble of {args.members} MLPs 64(56 used)-"
                    f"{args.hidden}-{args.hidden}-{args.hidden}-64(53 used), SiLU, BF16 "
                    f"weights/activations, FP32 accumulation; trained on {args.train_states} "
                    f"exact-kernel states, evaluated on {n} fresh states",
        "train": {"states": args.train_states, "epochs": args.epochs, "batch": args.batch,
                  "lr": args.lr, "data_s": round(t_data, 2), "train_s": round(t_train, 2),
                  "mse_by_epoch": [[round(x, 6) for x in h] for h in hist]},
        "heldout_err_without_fallback": held_out,
        "exact_ms": round(ms_exact, 4), "exact_Mcells_s": round(n / ms_exact / 1e3, 3),
        "mlp_only_ms": round(ms_mlp, 4), "mlp_only_Mcells_s": round(n / ms_mlp / 1e3, 3),
        "network_outputs_ms": round(ms_net, 4),
        "network_roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": 2500.0,
                             "achieved": round(net_flops * n / (ms_net * 1e-3) / 1e12, 1),
                             "frac": round(net_flops * n / (ms_net * 1e-3) / 2.5e15, 4),
                             "flops_per_cell": net_flops},
        "at_1e-3": main_row, "curve": curve,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=1 << 22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 16,
                    help="cells per host core for the oracle's Newton + omega (the VJP uses "
                         "1/64 of them)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-jacobian", action="store_true")
    ap.add_argument("--no-other-rows", action="store_true",
                    help="skip the enthalpy, primitive-variable, transport and reactor legs")
    ap.add_argument("--jacobian-cells", type=int, default=1 << 18)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 160-species mechanism's production-rate line")
    ap.add_argument("--train-states", type=int, default=1 << 24)
    ap.add_argument("--members", type=int, default=2)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--targets", type=float, nargs="+", default=[1e-3, 1e-2, 1e-1])
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="MIB",
                    help="end with one plain device-to-device copy of MIB MiB (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the cells are independent, so more GPUs "
              "would each run this same per-GPU workload on their own share; "
              "this benchmark runs one GPU only.", file=sys.stderr)
        sys.exit(2)

    # the oracle's workers are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample, max(args.cpu_sample // 64, 16))
        print(f"# cpu baseline: {cpu['value']} Mcells/s on {cpu['cores']} cores",
              file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from pyro_synth.states import draw_cotangent, draw_states

    torch.cuda.set_device(0)
    gm = pyro.Mechanism(MECH)
    n = args.cells
    t0 = time.time()
    T, p, Y = draw_states(1, n, gm.n_species)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T_d, p_d, Y_d = dev(T), dev(p), dev(Y)
    del T, p, Y
    rho = pyro.density(gm, p_d, T_d, Y_d)
    e = pyro.internal_energy(gm, T_d, Y_d)
    T_out = torch.empty_like(T_d)
    status = torch.empty(n, dtype=torch.int32, device="cuda")
    w = torch.empty_like(Y_d)
    wbar = dev(draw_cotangent(2, n, gm.n_species))
    Ybar = torch.empty_like(Y_d)
    Tbar = torch.empty_like(T_d)
    pbar = torch.empty((gm.n_params, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    print(f"# inputs ready: {n} cells in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    def events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev0, ev1 = events(), events()

    def step(i=None):
        pyro.temperature(gm, e, Y_d, T_guess=1200.0, out=T_out, status=status)
        if i is not None:
            ev0[i].record(stream)
        # one reverse-sweep launch: omega and the VJP of sum(wbar * omega)
        pyro.production_rates_vjp(gm, rho, T_out, Y_d, wbar, Ybar=Ybar, Tbar=Tbar,
                                  params_bar=pbar, wdot=w)
        if i is not None:
            ev1[i].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(args.steps):
        step(i)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    fused_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))
    if not bool(torch.isfinite(w).all()) or not bool((status > 0).all()):
        raise RuntimeError("non-finite rates or unconverged Newton in the benchmark")
    if not bool(torch.isfinite(Ybar).all()) or not bool(torch.isfinite(pbar).all()):
        raise RuntimeError("non-finite gradients in the benchmark")
    # the production-rate kernel alone (for callers that need omega only),
    # timed after the steps
    w2 = torch.empty_like(w)
    wdot_ms = _time_ms(lambda: pyro.production_rates(gm, rho, T_out, Y_d, out=w2),
                       max(args.steps, 3), stream)
    # the same with each alternative kernel variant (equilibrium constants per
    # reaction; third-body concentrations, net rates nu q on the FP64 matrix cores)
    from paper_2503_24286_amd import _lib
    variant_ms = {}
    default_variant = gm.wdot_variant
    for name, v in (("reaction_equilibrium", _lib.PYRO_WDOT_REACTION_EQUILIBRIUM),
                    ("third_body_on_mfma", default_variant | _lib.PYRO_WDOT_MFMA_THIRD_BODY),
                    ("net_rates_on_mfma", default_variant | _lib.PYRO_WDOT_MFMA_NET_RATES),
                    ("third_body_and_net_rates_on_mfma", default_variant
                     | _lib.PYRO_WDOT_MFMA_THIRD_BODY | _lib.PYRO_WDOT_MFMA_NET_RATES),
                    ("reaction_equilibrium_third_body_on_mfma",
                     _lib.PYRO_WDOT_REACTION_EQUILIBRIUM | _lib.PYRO_WDOT_MFMA_THIRD_BODY),
                    ("log_space", _lib.PYRO_WDOT_LOG_SPACE),
                    ("log_space_log_products_on_mfma",
                     _lib.PYRO_WDOT_LOG_SPACE | _lib.PYRO_WDOT_MFMA_LOG_PRODUCTS)):
        gm.wdot_variant = v
        variant_ms[name] = round(_time_ms(
            lambda: pyro.production_rates(gm, rho, T_out, Y_d, out=w2), 3, stream), 4)
    gm.wdot_variant = default_variant
    del w2
    fp32 = fp32_leg(gm, rho, T_out, Y_d, stream, max(args.steps, 3))
    print(f"# fp32: {fp32['ms']} ms, {fp32['overflow_fraction']:.4f} of the cells overflow",
          file=sys.stderr, flush=True)

    ms_per_step = total_ms / args.steps
    value = n / (ms_per_step * 1e-3) / 1e6

    traffic = measured_traffic()

    def roof(name, ms, fpc, bpc):
        achieved = fpc * n / (ms * 1e-3) / 1e12
        t = traffic.get(name)
        return {"kernel": name, "bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": t if (t is not None and n == 1 << 22) else None,
                "flops_per_cell": fpc,
                "hbm_GBps_compulsory": round(bpc * n / (ms * 1e-3) / 1e9, 1)}

    result = {
        "metric": "Mcells/s for wdot (53sp/325rxn FP64) + VJP; surrogate vs exact at <=1e-3 rel err",
        "value": round(value, 3),
        "unit": "Mcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"53-species 325-reaction synthetic mechanism, {n} cells, "
                        "T U[300,3000] K, log10 p U[4,6.5], Y Dirichlet(0.3)",
            "step": "newton T(e,Y) from 1200 K, then one reverse-sweep launch returning "
                    "wdot(rho,T,Y) and the VJP of sum(wbar*wdot) w.r.t. Y, T, ln A, b, Ea",
            "n_cells": n, "species": gm.n_species, "reactions": gm.n_reactions,
        },
        "kernels_ms": {"vjp_with_wdot": round(fused_ms, 4),
                       "newton_and_rest": round(ms_per_step - fused_ms, 4),
                       "wdot_alone_outside_step": round(wdot_ms, 4),
                       "wdot_variants_outside_step": variant_ms},
        "roofline": roof("vjp_kernel", fused_ms, fused_flops_per_cell(gm),
                         fused_bytes_per_cell(gm)),
        "roofline_other": roof("wdot_kernel", wdot_ms, wdot_flops_per_cell(gm),
                               wdot_bytes_per_cell(gm)),
        "fp32": fp32,
    }
    gm.close()
    del T_d, p_d, Y_d, rho, e, T_out, status, w, wbar, Ybar, Tbar, pbar
    torch.cuda.empty_cache()
    def log(msg):
        print(f"# {msg}", file=sys.stderr, flush=True)
    if not args.no_jacobian:
        result["jacobian"] = jacobian_leg(args, log)
    if not args.no_other_rows:
        result["other_rows"] = other_rows_leg(args, log)
    if not args.no_large:
        result["large_mechanism"] = large_mechanism_leg(args, log)
    if not args.no_surrogate:
        result["surrogate"] = surrogate_leg(args, log)
    if args.calibration_copy > 0:
        src = torch.empty(args.calibration_copy << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
