"""Throughput of the per-cell thermochemistry hot path on one MI355X.

One step runs the whole hot path over a batch of cells already resident in
HBM: the Newton inversion T(e, Y) from a 1200 K guess, then the net
production rates omega(rho, T, Y) at that temperature, on the 53-species,
325-reaction synthetic mechanism (2^22 cells by default).  The figure of merit
is million cells per second (higher is better).

Prints one JSON line with, besides the throughput, a roofline entry for the
production-rate kernel (algorithmic FP64 flops per launch over its average
launch time, timed with HIP events on the stream it runs on) and the CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cells N]
                       [--no-cpu-baseline] [--cpu-sample N]
"""

import argparse
import json
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


def wdot_bytes_per_cell(gm):
    """Compulsory HBM bytes of omega per cell: read rho, T, Y; write omega."""
    return 8 * (2 + 2 * gm.n_species)


def cpu_baseline(n_sample, cfg=1):
    """The oracle (NumPy, single thread for its elementwise work) on the first
    ``n_sample`` cells of the same workload: Newton from 1200 K, then omega."""
    import numpy as np
    from oracle import eos, kinetics, mechfile, newton, thermo
    from pyro_synth.states import draw_states
    m = mechfile.load(MECH)
    chunk = 8192
    elapsed = 0.0
    done = 0
    while done < n_sample:
        k = min(chunk, n_sample - done)
        T, p, Y = draw_states(cfg, k, m.S, first=done)
        rho = eos.density(m, p, T, Y)
        e = thermo.mixture_internal_energy(m, T, Y)
        t0 = time.perf_counter()
        Tn, st = newton.temperature(m, e, Y, 1200.0)
        w = kinetics.net_production_rates(m, rho, Tn, Y)
        elapsed += time.perf_counter() - t0
        assert np.isfinite(w).all()
        done += k
    return {"value": n_sample / elapsed / 1e6, "unit": "Mcells/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {n_sample} cells of the 2^22-cell workload, Newton + omega, "
                      f"NumPy oracle in chunks of {chunk} ({elapsed:.1f} s), "
                      f"host {platform.processor() or platform.machine()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=1 << 22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the cells are independent, so more GPUs "
              "would each run this same per-GPU workload on their own share; "
              "multi-GPU runs are not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2503_24286_amd as pyro
    from pyro_synth.states import draw_states

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
    torch.cuda.synchronize()
    print(f"# inputs ready: {n} cells in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(i=None):
        pyro.temperature(gm, e, Y_d, T_guess=1200.0, out=T_out, status=status)
        if i is not None:
            ev[i][0].record(stream)
        pyro.production_rates(gm, rho, T_out, Y_d, out=w)
        if i is not None:
            ev[i][1].record(stream)

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
    wdot_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    if not bool(torch.isfinite(w).all()) or not bool((status > 0).all()):
        raise RuntimeError("non-finite rates or unconverged Newton in the benchmark")

    ms_per_step = total_ms / args.steps
    value = n / (ms_per_step * 1e-3) / 1e6
    flops = wdot_flops_per_cell(gm) * n
    achieved = flops / (wdot_ms * 1e-3) / 1e12
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
            "step": "newton T(e,Y) from 1200 K + wdot(rho,T,Y)",
            "n_cells": n, "species": gm.n_species, "reactions": gm.n_reactions,
        },
        "kernels_ms": {"wdot": round(wdot_ms, 4), "newton_and_rest": round(ms_per_step - wdot_ms, 4)},
        "roofline": {
            "kernel": "wdot_f64_kernel",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
            "traffic": None,
            "flops_per_cell": wdot_flops_per_cell(gm),
            "hbm_GBps_compulsory": round(wdot_bytes_per_cell(gm) * n / (wdot_ms * 1e-3) / 1e9, 1),
        },
    }
    gm.close()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
