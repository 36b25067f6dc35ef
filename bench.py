"""Benchmark: DMC walker-moves per second (local energy every step) on one MI355X.

Default workload (the largest configuration that fits one GPU): fixed-node
DMC on the 64-electron synthetic molecule -- 16 nuclei (Z in {1, 6, 8}),
32 up + 32 down electrons, 240 contracted Gaussians (4s2p1d per atom),
46 orbitals (30 inactive + 16 active), 32 VB structures / 128 determinant
pairs (83 distinct spin determinants per spin), Pade Jastrow -- with 32768
target walkers, tau = 0.005, per-electron drift-diffusion moves with
Metropolis acceptance, E_L every step, branching with population control and
on-device compaction, FP64.  One walker-move is one walker advanced by one
step (64 single-electron moves and its local energy).  Inputs are seeded and
synthetic and resident in device memory when timing starts.

Other forms: --form vmc (the F2-shaped VMC row kernel; --system precision the 40-electron molecule,
--system h2 the all-electron H2 workload), precision, adjoint, ecp.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--form ...]
Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, FP64 vector (published)
# HBM bytes per launch of the dominant kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) scaled by the copy-kernel calibration (the
# factors), each with the SHA-256 prefix of the kernel's source file and the
# shared headers it was taken on (traffic_bytes reports it only while they
# are unchanged, else null).  The sweep: k_sweep_g<32, 0, 0> on the F2-shaped
# workload (4096 walkers, one step per launch); the row kernel: one launch of
# 100 steps on the same workload.
SWEEP_TRAFFIC = {"src": "vbqmc_sweep.hip", "src_sha": "7bce33b7a54dd23e", "fetch_kib": 4567.5, "write_kib": 8256.0,
                 "fetch_factor": 2.000, "write_factor": 1.000, "walkers": 4096, "lanes": 32}
ROWS_TRAFFIC = {"src": "vbqmc_rows.hip", "src_sha": "f1cf94c2b2c6a6d1", "fetch_kib": 5603.6, "write_kib": 9861.4,
                "fetch_factor": 2.000, "write_factor": 1.000, "walkers": 4096, "steps_per_launch": 100}
# the walker-resident kernel in VMC mode on the 40-electron molecule (two
# replaced columns at most per determinant, 160 padded basis functions)
WRES_VMC_KERNEL = "k_dmcw<32, 2, 16, true, false>"
EXP_FLOPS = 20                  # one double-precision exp counted as 20 flops


def _dims(ctx, system):
    info = ctx.info
    P = sum(len(s["exps"]) for s in system["shells"])
    spins = [(info["n_up"], info["n_table_up"], info["n_unique_up"]),
             (info["n_dn"], info["n_table_dn"], info["n_unique_dn"])]
    return info["n_electrons"], info["n_basis"], info["n_orbitals"], info["n_nuclei"], P, spins


def sweep_flops_per_walker_move(ctx, system, accept_rate):
    """Algorithmic FLOPs of one sweep of one walker (N single-electron moves,
    no local energy), from the system's dimensions.

    Counted per move: basis values at the trial point (per primitive 4 flops
    + one exp; per function 2), the basis->orbital contraction (2 M N_orb),
    the determinant-table ratio (2n + 2 n nP + 6U) and the Jastrow change
    (2 pair functions of 12 flops per partner); per accepted move the
    Sherman-Morrison update (4n^2 + 3 n nP + 8U)."""
    N, M, norb, nnuc, P, spins = _dims(ctx, system)
    total = 0.0
    for n, nP, u in spins:
        per_move = (P * (4 + EXP_FLOPS) + 2 * M) + 2 * M * norb + (2 * n + 2 * n * nP + 6 * u) \
            + (N - 1 + nnuc) * 2 * 12
        per_accept = 4 * n * n + 3 * n * nP + 8 * u
        total += n * (per_move + accept_rate * per_accept)
    return total


def measure_flops_per_walker(ctx, system):
    """Algorithmic FLOPs of one local energy of one walker from its stored
    inverse and table: basis gradients and Laplacians (per primitive 6 flops
    + one exp, per function 16), their contraction (4 channels, 2 M N_orb
    each), 4 row-operator ratios per electron (2n + 2 n nP + 8U each), the
    Jastrow gradients and Laplacians (30 flops per pair, 10 per electron)."""
    N, M, norb, nnuc, P, spins = _dims(ctx, system)
    total = sum(n * 4 * (2 * n + 2 * n * nP + 8 * u) for n, nP, u in spins)
    total += N * (P * (6 + EXP_FLOPS) + 16 * M) + 2 * 4 * N * M * norb
    total += (N * (N - 1) / 2 + N * nnuc) * 30 + 10 * N
    return total


def vmc_flops_per_walker_move(ctx, system, accept_rate):
    """One VMC step of one walker: a sweep and one local energy."""
    return sweep_flops_per_walker_move(ctx, system, accept_rate) + measure_flops_per_walker(ctx, system)


def adjoint_flops_per_gradient(ctx, system):
    """Algorithmic FLOPs of one walker's full gradient with the adjoint through
    each spin's reference determinant: 5-channel basis values (per primitive
    6 flops + one exp, per function 16) and their contraction for all
    electrons; per spin, in each of the two passes, the reference inversion
    (2 n^3), S = K_0 B and B S (2 n^3 each), T, Xi and B Xi (2 n^2 n_P each)
    and the kinetic rows (8 n (n + n_P)); per distinct determinant the e x e
    minor, its inverse and V Xi_Q (about 60) and its share of the sums per
    table orbital (20 n); the scatter onto orbital rows (8 n (n + n_P) n_P)
    and the drift and Laplacian ratios from it (8 N_orb per electron); the
    Jastrow pair derivatives (12 parameters x 12 flops per pair); and the two
    orbital-coefficient contractions (3 x 2 N N_orb M)."""
    info = ctx.info
    N, M, norb, nnuc = info["n_electrons"], info["n_basis"], info["n_orbitals"], info["n_nuclei"]
    P = sum(len(s["exps"]) for s in system["shells"])
    total = N * (P * (6 + EXP_FLOPS) + 16 * M) + 2 * 5 * N * M * norb
    for n, nP, u in ((info["n_up"], info["n_table_up"], info["n_unique_up"]),
                     (info["n_dn"], info["n_table_dn"], info["n_unique_dn"])):
        total += 2 * (6 * n ** 3 + 6 * n * n * nP + 8 * n * (n + nP))
        total += u * (60 + 20 * n) + 8 * n * (n + nP) * nP + 8 * norb * n
    total += (N * (N - 1) / 2 + N * nnuc) * 12 * 12
    total += 3 * 2 * N * norb * M
    return total


def cpu_baseline(system, step_size, steps=300, walkers=1024, seed=11):
    """The oracle (plain FP64 CPU code, OpenMP over walkers) on a bounded
    sample of the same workload: `walkers` walkers x `steps` steps."""
    import oracle
    import systems as S
    o = oracle.Oracle(system)
    R0 = S.initial_walkers(system, walkers, seed=seed)
    t0 = time.perf_counter()
    o.vmc(R0, steps, 1234, 0, step_size, False)
    dt = time.perf_counter() - t0
    return {"value": walkers * steps / dt, "unit": "walker-moves/s", "cores": oracle.max_threads(),
            "kind": "oracle", "sample": f"{walkers} walkers x {steps} steps of the same VMC workload, "
            f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for the DMC headline, the form's own for the others)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default: 3, or the form's own)")
    ap.add_argument("--walkers", type=int, default=None,
                    help="walkers (target population for DMC; default: the workload's)")
    ap.add_argument("--steps-per-launch", type=int, default=100,
                    help="VMC steps per call (warm-up calls, and timed calls of the row kernel)")
    ap.add_argument("--no-precision-compare", action="store_true",
                    help="dmc form: skip the short mixed-precision run reported beside the FP64 line")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16", "mixed"],
                    help="mixed: FP32 trial/proposal rows, FP64 inverse rebuilt before every E_L and FP64 E_L")
    ap.add_argument("--walker-lanes", type=int, default=0, choices=[0, 16, 32, 64],
                    help="lanes per walker in the single-electron sweep (0: library choice)")
    ap.add_argument("--step-kernel", type=int, default=0, choices=[0, 1, 2, 3],
                    help="single-electron step kernel: 0 library choice, 1 sweep + local-energy kernels, "
                         "2 row kernel, 3 walker-resident kernel")
    ap.add_argument("--een", action="store_true",
                    help="dmc and vmc forms: add the three-body Jastrow f_een to the workload's wave function")
    ap.add_argument("--een-scale", type=float, default=0.01,
                    help="standard deviation of the f_een coefficients (default 0.01)")
    ap.add_argument("--system", default="f2", choices=["f2", "precision", "h2"],
                    help="vmc form: the F2-shaped diatomic or the 40-electron molecule of the precision form")
    ap.add_argument("--dmc-kernel", type=int, default=0, choices=[0, 1, 2, 3],
                    help="DMC: 0 library choice, 1 one workgroup per walker, 2 electron-major launches, "
                         "3 walker-resident")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-exponent", type=float, default=1e4,
                    help="precision form: cap on the Gaussian exponents of the molecule (default: the workload's 1e4)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--form", default="dmc", choices=["dmc", "vmc", "plain", "precision", "adjoint", "ecp"],
                    help="dmc: the headline DMC line on the 64-electron molecule; vmc (or plain): VMC on the "
                         "F2-shaped diatomic; precision: FP32/BF16 basis+contraction forms on the 10-nucleus "
                         "molecule; adjoint: parameter gradients on the 6-nucleus molecule")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: walkers are independent between branching steps, so the "
                          "path would shard them across GPUs, but no multi-GPU run is provided"}))
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = 256 * 1024 * 1024 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))
        return
    if args.form == "precision":
        return precision_form(args)
    if args.form == "adjoint":
        return adjoint_form(args)
    if args.form == "ecp":
        return ecp_form(args)
    if args.form == "dmc":
        return dmc_form(args)
    if args.system == "h2":
        return h2_form(args)
    return vmc_form(args)


def h2_form(args):
    """All-electron VMC on the H2 Heitler-London function (2 protons at
    +-0.7 bohr, covalent and ionic structures, Pade Jastrow): 1024 walkers,
    Metropolis moves of all electrons at once in a 0.5-bohr cube, E_L every
    step, 1000 steps in one launch of the all-electron kernel (bracketed by
    events on the launch stream) after a warm-up call."""
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    system = S.h2_heitler_london()
    W = args.walkers or 1024
    steps = args.steps if args.steps is not None else 1000
    warm = args.warmup if args.warmup is not None else 100
    step_size, seed = 0.5, 20220728
    ctx = vb.Context(system)
    state = ctx.walkers_init(torch.from_numpy(S.initial_walkers(system, W, seed=5)).cuda())
    acc = ctx.new_vmc_acc(W)
    if warm > 0:
        ctx.vmc_advance(state, warm, seed, 0, step_size, True, acc)
    acc = ctx.new_vmc_acc(W)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.vmc_advance(state, steps, seed, warm, step_size, True, acc)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = e0.elapsed_time(e1) / 1e3
    moves = W * steps
    accept = float(acc["n_accept"].sum().item()) / moves
    # per walker-step: one full evaluation at the proposal (basis values,
    # gradients and Laplacians, the determinants and E_L)
    _, _, _, _, _, spins = _dims(ctx, system)
    fl = measure_flops_per_walker(ctx, system) + sum(2.0 * n ** 3 / 3 + 2.0 * n * n * nP for n, nP, _ in spins)
    achieved = fl * moves / kernel_s / 1e12
    line = {
        "metric": "walker-moves/sec incl. E_L", "value": moves / wall, "unit": "walker-moves/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": wall / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "H2 Heitler-London VMC: 2 protons at +-0.7 bohr, 1 up + 1 down electron, 3 "
                               "contracted s Gaussians per atom, covalent + ionic structures (0.9, 0.3), Pade "
                               f"Jastrow, {W} walkers, all-electron Metropolis moves of 0.5 bohr, E_L every step",
                   "walkers": W, "electrons": ctx.N, "precision": "fp64", "step_kernel": "all-electron"},
        "acceptance": accept,
        "mean_eloc": float(acc["e_sum"].sum().item()) / moves,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_vmc (all-electron)", "kernel_avg_ms_per_launch": kernel_s * 1e3,
                     "flops_per_walker_step": fl, "walkers_per_launch": W, "steps_per_launch": steps},
    }
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Oracle(system)
        R0 = S.initial_walkers(system, W, seed=11)
        t0 = time.perf_counter()
        o.vmc(R0, steps, 1234, 0, step_size, True)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": W * steps / dt, "unit": "walker-moves/s", "cores": oracle.max_threads(),
                                "kind": "oracle",
                                "sample": f"the whole workload: {W} walkers x {steps} all-electron steps, {dt:.1f} s"}
    print(json.dumps(line))


def vmc_form(args):
    """Single-electron VMC, walker-moves/s with E_L every step: on the
    F2-shaped diatomic (18 electrons, 4096 walkers, row kernel), or with
    --system precision on the 10-nucleus, 40-electron molecule (16384
    walkers, walker-resident kernel)."""
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    big = args.system == "precision"
    args.steps = (200 if big else 2000) if args.steps is None else args.steps
    args.warmup = (20 if big else 100) if args.warmup is None else args.warmup
    args.walkers = (16384 if big else 4096) if args.walkers is None else args.walkers
    system = S.precision_molecule() if big else S.f2_shaped()
    if args.een:
        system = S.with_een(system, scale=args.een_scale)
    W, step_size = args.walkers, 0.3
    ctx = vb.Context(system, precision=args.precision, walker_lanes=args.walker_lanes,
                     step_kernel=args.step_kernel)
    R0 = torch.from_numpy(S.initial_walkers(system, W, seed=5)).cuda()
    state = ctx.walkers_init(R0)
    acc = ctx.new_vmc_acc(W)
    seed = 20220728
    spl = max(1, args.steps_per_launch)
    step = 0
    while step < args.warmup:
        k = min(spl, args.warmup - step)
        ctx.vmc_advance(state, k, seed, step, step_size, False, acc)
        step += k
    torch.cuda.synchronize()
    acc = ctx.new_vmc_acc(W)
    stream = torch.cuda.current_stream()
    rows = ctx.info["step_kernel"] == 2
    wres = ctx.info["step_kernel"] == 3
    lanes = ctx.info["sweep_lanes"]
    if rows or wres:
        # timed region: calls of `spl` steps, each one launch of the row
        # kernel (moves and E_L of every step), or for the walker-resident
        # kernel 1 + spl launches (the record rebuild that opens the call,
        # then one per step), bracketed by events on the launch stream; a
        # shorter last call is timed but not averaged
        chunks = [spl] * (args.steps // spl) + ([args.steps % spl] if args.steps % spl else [])
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(chunks))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, c in enumerate(chunks):
            ev[2 * k].record(stream)
            ctx.vmc_advance(state, c, seed, step, step_size, False, acc)
            ev[2 * k + 1].record(stream)
            step += c
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        full = [k for k, c in enumerate(chunks) if c == spl] or [0]
        kernel_s = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in full) / 1e3
        launches = len(full) * (chunks[full[0]] + 1 if wres else 1)
        steps_launch = chunks[full[0]] / (chunks[full[0]] + 1) if wres else chunks[full[0]]
        measure_s = None
    else:
        # timed region: per step one sweep (the dominant kernel, bracketed by
        # events on the launch stream) and one measurement of E_L
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[2 * k].record(stream)
            ctx.vmc_sweep(state, seed, step, step_size, acc["n_accept"])
            ev[2 * k + 1].record(stream)
            ctx.vmc_measure(state, acc)
            step += 1
        ev[2 * args.steps].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_s = sum(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)) / 1e3
        measure_s = sum(ev[2 * k + 1].elapsed_time(ev[2 * k + 2]) for k in range(args.steps)) / 1e3
        launches = args.steps
        steps_launch = 1
    moves = W * args.steps
    accept_rate = float(acc["n_accept"].sum().item()) / (moves * ctx.N)
    e_mean = float(acc["e_sum"].sum().item()) / moves
    sweep_flops = sweep_flops_per_walker_move(ctx, system, accept_rate) * W
    measure_flops = measure_flops_per_walker(ctx, system) * W
    prec_tag = {"fp64": 0, "fp32": 1, "bf16": 2, "mixed": 0}[args.precision]
    if wres:
        # every launch but the rebuild makes the moves and E_L of one step;
        # the rebuild's work is not counted (steps_launch = spl / (spl + 1))
        kernel = wres_kernel_name(ctx, True) if args.een else WRES_VMC_KERNEL
        if args.een:
            sweep_flops += een_flops_per_walker_step(ctx, False) * W
        flops_launch = (sweep_flops + measure_flops) * steps_launch
        t = WRES_VMC_TRAFFIC
        traffic = (traffic_bytes(t) if (big and W == t["walkers"] and args.precision == "fp64" and not args.een)
                   else None)
    elif rows:
        # the dominant (and only) kernel makes moves and E_L of every step
        ne = 10 if max(ctx.info["n_up"], ctx.info["n_dn"]) <= 10 else 16  # register columns per lane
        kernel = f"k_vmc_rows<1, 0, {ne}>" if args.precision == "mixed" else f"k_vmc_rows<{prec_tag}, {prec_tag}, {ne}>"
        flops_launch = (sweep_flops + measure_flops) * steps_launch
        t = ROWS_TRAFFIC
        traffic = (traffic_bytes(t) if (W == t["walkers"] and args.precision == "fp64" and
                                        steps_launch == t["steps_per_launch"]) else None)
    else:
        pt = 1 if args.precision == "mixed" else prec_tag
        kernel = f"k_sweep_g<{lanes}, {pt}, {prec_tag}>" if lanes < 64 else f"k_sweep<64, {prec_tag}>"
        flops_launch = sweep_flops
        t = SWEEP_TRAFFIC
        traffic = (traffic_bytes(t) if lanes == t["lanes"] and W == t["walkers"] and args.precision == "fp64"
                   else None)
    kernel_avg = kernel_s / launches
    achieved = flops_launch / kernel_avg / 1e12
    line = {
        "metric": "walker-moves/sec incl. E_L",
        "value": moves / wall,
        "unit": "walker-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": _dtype(args.precision),
        "data": "synthetic",
        "config": {"workload": ("40-electron molecule VMC: 10 nuclei (Z in {1,6,7,8}), 20 up + 20 down "
                                "electrons, 150 Gaussian basis functions, 20 VB structures / 64 determinants" +
                                (f", three-body f_een (23 coefficients per element ~ N(0, {args.een_scale}^2))"
                                 if args.een else "") +
                                f", {W} walkers, single-electron moves of 0.3 bohr with Sherman-Morrison "
                                "updates, E_L every step" if big else
                                "F2-shaped diatomic VMC: 18 electrons (9 up, 9 down), 28 Gaussian basis "
                                "functions, 3 VB structures / 4 determinants, 4096 walkers, single-electron "
                                "moves of 0.3 bohr with Sherman-Morrison updates, E_L every step"),
                   "walkers": W, "electrons": ctx.N, "precision": args.precision,
                   "step_kernel": "rows" if rows else "walker-resident" if wres else
                   f"sweep {lanes} lanes + local energy"},
        "electron_moves_per_s": moves * ctx.N / wall,
        "acceptance": accept_rate,
        "mean_eloc": e_mean,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": kernel, "kernel_avg_ms_per_launch": kernel_avg * 1e3,
                     "flops_per_launch": flops_launch, "walkers_per_launch": W,
                     "steps_per_launch": steps_launch},
    }
    if measure_s is not None:
        line["measure"] = {"kernels": f"k_eloc_tiles<{prec_tag}> + k_eloc_finish",
                           "avg_ms_per_step": measure_s / args.steps * 1e3, "flops_per_step": measure_flops,
                           "achieved_tflops": measure_flops / (measure_s / args.steps) / 1e12}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = (cpu_baseline(system, step_size, steps=8, walkers=512) if big else
                                cpu_baseline(system, step_size))
    print(json.dumps(line))


def _dtype(prec):
    if prec == "fp64":
        return "f64"
    if prec == "mixed":
        return "fp32 trial rows; f64 E_L, inverse refresh and determinants"
    return f"{prec} basis/contraction, f64 determinants"


def _timed(fn):
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    out = fn()
    ev1.record()
    torch.cuda.synchronize()
    return out, ev0.elapsed_time(ev1) / 1e3


def precision_form(args):
    """Mixed-precision forms on the 10-nucleus, 40-electron, 150-function,
    20-structure / 64-determinant molecule: walker-moves/s of FP64, FP32 and
    BF16 basis values + contraction (determinants in FP64 throughout) and of
    the mixed form (FP32 trial rows, FP64 inverse rebuilt before every E_L,
    FP64 E_L); per-walker |E_L(form) - E_L(FP64)| at identical configurations
    (evaluate, and the chain's own last E_L against an FP64 evaluation of its
    configurations), and the mean-energy shift by correlated sampling."""
    import numpy as np
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    system = S.precision_molecule(max_exponent=args.max_exponent)
    W = args.walkers or 16384
    steps, step_size, seed = args.steps if args.steps is not None else 20, 0.3, 777
    R0 = torch.from_numpy(S.initial_walkers(system, W, seed=9)).cuda()
    c64 = vb.Context(system, precision="fp64", walker_lanes=args.walker_lanes)
    st = c64.walkers_init(R0)
    c64.vmc_advance(st, args.warmup if args.warmup is not None else 20, seed, 0, step_size)  # burn-in in FP64
    Rb = c64.positions(st)
    ref = c64.evaluate(Rb, want=("eloc",))["eloc"]
    res = {"metric": "walker-moves/sec incl. E_L (precision forms)", "unit": "walker-moves/s", "n_gpus": 1,
           "walkers": W, "steps": steps, "data": "synthetic", "sweep_lanes": c64.info["sweep_lanes"],
           "config": {"workload": "10 nuclei (Z in {1,6,7,8}), 40 electrons, 150 Gaussian basis functions, "
                                  "20 VB structures / 64 determinants, VMC single-electron moves 0.3 bohr, "
                                  "E_L every step, inverse refresh every 32 updates",
                      "max_exponent": args.max_exponent}, "forms": {}}
    for prec in ("fp64", "fp32", "bf16", "mixed"):
        ctx = c64 if prec == "fp64" else vb.Context(system, precision=prec, refresh_every=32,
                                                     walker_lanes=args.walker_lanes)
        ev = ctx.evaluate(Rb, want=("eloc",))["eloc"]
        d = (ev - ref).abs().cpu().numpy()
        stp = ctx.walkers_init(Rb.clone())
        acc = ctx.new_vmc_acc(W)
        _, t = _timed(lambda: ctx.vmc_advance(stp, steps, seed, 1000, step_size, False, acc))
        # correlated sampling: FP64 E_L on the final configurations of this chain
        Rm = ctx.positions(stp)
        e_mixed = acc["e_last"]
        e_64 = c64.evaluate(Rm, want=("eloc",))["eloc"]
        shift = (e_mixed - e_64).cpu().numpy()
        rate = float(acc["n_accept"].sum().item()) / (W * steps * ctx.N)
        fl = vmc_flops_per_walker_move(ctx, system, rate) * W * steps / t / 1e12
        # the reduced forms run the basis values and the contraction on the
        # FP32 unit (FP32 VALU / FP32 MFMA, 157.3 TFLOP/s) or the BF16 MFMA
        # (2500 TFLOP/s dense) and everything else in FP64: their fraction is
        # given against both peaks, each named
        red_peak = {"fp32": ("fp32", 157.3), "bf16": ("bf16 mfma", 2500.0), "mixed": ("fp32", 157.3)}.get(prec)
        roof = {"bound": "alu", "achieved": fl, "peak": FP64_VECTOR_PEAK_TFLOPS, "peak_unit": "fp64",
                "unit": "TFLOP/s", "frac": fl / FP64_VECTOR_PEAK_TFLOPS}
        if red_peak:
            roof["reduced_peak"] = {"unit": red_peak[0], "peak": red_peak[1], "frac": fl / red_peak[1]}
        res["forms"][prec] = {"value": W * steps / t, "ms_per_step": t / steps * 1e3,
                              "roofline": roof,
                              "abs_dEL_max": float(np.nanmax(d)), "abs_dEL_p99": float(np.nanpercentile(d, 99)),
                              "abs_dEL_median": float(np.nanmedian(d)),
                              "mean_shift": float(np.nanmean(shift)),
                              "abs_dEL_chain_max": float(np.nanmax(np.abs(shift))),
                              "mean_shift_stderr": float(np.nanstd(shift) / np.sqrt(W)),
                              "meets_1e-5": bool(max(np.nanmax(d), np.nanmax(np.abs(shift))) <= 1e-5 and
                                                 abs(np.nanmean(shift)) <= 1e-5)}
    print(json.dumps(res))


def adjoint_form(args):
    """Parameter gradients (d lnPsi/dp and d E_L/dp, all ~3054 parameters) for
    8192 walkers of the 6-nucleus, 30-electron, 120-function, 12-structure /
    40-determinant molecule, against the plain-FP64 alternative of central
    finite differences (2 N_p + 1 evaluations per gradient), timed as
    single evaluate calls of the same batch."""
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    system = S.adjoint_molecule()
    W = args.walkers or 8192
    ctx = vb.Context(system)
    R0 = torch.from_numpy(S.initial_walkers(system, W, seed=3)).cuda()
    st = ctx.walkers_init(R0)
    ctx.vmc_advance(st, max(args.warmup if args.warmup is not None else 20, 1), 5, 0, 0.3)
    R = ctx.positions(st)
    ctx.param_grad(R)  # warm-up
    reps = 3
    _, t = _timed(lambda: [ctx.param_grad(R) for _ in range(reps)])
    t /= reps
    _, te = _timed(lambda: [ctx.evaluate(R, want=("eloc",)) for _ in range(reps)])
    te /= reps
    npar = ctx.n_params
    fd = W / (te * (2 * npar + 1))
    gfl = adjoint_flops_per_gradient(ctx, system) * W / t / 1e12
    # linear-method sample sums of the same gradients (FP64 MFMA over the
    # walkers: three (P+1) x W x (P+1) products, 6 (P+1)^2 W FLOP)
    dl, de = ctx.param_grad(R)
    el = ctx.evaluate(R, want=("eloc",))["eloc"]
    acc = ctx.new_lm_acc()
    ctx.lm_accumulate(dl, de, el, acc)
    _, tl = _timed(lambda: [ctx.lm_accumulate(dl, de, el, acc) for _ in range(reps)])
    tl /= reps
    lm_tf = 6.0 * (npar + 1) ** 2 * W / tl / 1e12
    print(json.dumps({"metric": "walker-gradients/s (d lnPsi/dp and d E_L/dp)", "value": W / t,
                      "unit": "gradients/s", "n_gpus": 1, "walkers": W, "n_params": npar,
                      "ms_per_call": t * 1e3, "fp64_central_difference_gradients_per_s": fd,
                      "speedup_vs_fd": (W / t) / fd, "evaluate_ms": te * 1e3,
                      "lm_accumulate": {"ms_per_call": tl * 1e3, "achieved": lm_tf, "unit": "TFLOP/s",
                                        "peak": FP64_VECTOR_PEAK_TFLOPS, "frac": lm_tf / FP64_VECTOR_PEAK_TFLOPS,
                                        "bound": "mfma"},
                      "roofline": {"bound": "alu", "achieved": gfl, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": gfl / FP64_VECTOR_PEAK_TFLOPS,
                                   "flops_per_gradient": adjoint_flops_per_gradient(ctx, system)},
                      "config": {"workload": "6 nuclei, 30 electrons, 120 Gaussian basis functions, 12 VB "
                                             "structures / 40 determinants, kappa = 0.8 Jastrow with polynomials"}}))


def ecp_points(system, R):
    """(electron, pseudo-nucleus) pairs within r_cut per configuration, times
    the 12 points of the angular rule: the ratio evaluations of one E_L."""
    import numpy as np
    pos = np.asarray(system["nuclei"]["pos"], np.float64)
    n = 0
    for cen in system["ecp"]:
        if cen["channels"]:
            d = np.linalg.norm(R - pos[cen["center"]], axis=-1)
            n += int((d < cen["r_cut"]).sum())
    return 12 * n / R.shape[0]


def ecp_flops_per_point(ctx, system):
    """One ratio of the nonlocal projection: the work of a single-electron
    move's ratio (basis values and contraction at the point, determinant-table
    ratio, Jastrow change; averaged over the two spins) plus the Legendre
    weights (15)."""
    N, M, norb, nnuc, P, spins = _dims(ctx, system)
    per = [(P * (4 + EXP_FLOPS) + 2 * M) + 2 * M * norb + (2 * n + 2 * n * nP + 6 * u) + (N - 1 + nnuc) * 2 * 12
           for n, nP, u in spins]
    return sum(per) / len(per) + 15


def ecp_form(args):
    """E_L with semilocal pseudopotentials on the F2 valence system (14
    electrons, Z_eff = 7 per atom, s and p nonlocal channels, r_cut 2.5 bohr,
    12-point rule): evaluate calls of the one-workgroup-per-walker kernel on
    8192 VMC-equilibrated configurations, with and without the
    pseudopotential term, and VMC and DMC steps with it."""
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    system = S.f2_valence_ecp()
    plain = {k: v for k, v in system.items() if k != "ecp"}
    W = args.walkers or 8192
    ctx = vb.Context(system)
    ctx0 = vb.Context(plain)
    # the pseudopotential does not change Psi: sample with the plain context
    st = ctx0.walkers_init(torch.from_numpy(S.initial_walkers(system, W, seed=3)).cuda())
    ctx0.vmc_advance(st, max(args.warmup if args.warmup is not None else 30, 1), 5, 0, 0.4)
    R = ctx0.positions(st)
    reps = 3
    ctx.evaluate(R, want=("eloc",))
    _, t = _timed(lambda: [ctx.evaluate(R, want=("eloc",)) for _ in range(reps)])
    t /= reps
    _, t0 = _timed(lambda: [ctx0.evaluate(R, want=("eloc",)) for _ in range(reps)])
    t0 /= reps
    pts = ecp_points(system, R.cpu().numpy())
    fl = measure_flops_per_walker(ctx, system) + pts * ecp_flops_per_point(ctx, system)
    tf = fl * W / t / 1e12
    # VMC steps (single-electron moves + E_L with the term) on the same walkers
    st1 = ctx.walkers_init(R)
    nst = 2
    _, tv = _timed(lambda: ctx.vmc_advance(st1, nst, 7, 100, 0.4))
    # DMC steps with the term in the branching E_L (locality approximation)
    d0, d1 = ctx.new_state(2 * W), ctx.new_state(2 * W)
    ctx.walkers_init(R, d0)
    et = float(ctx.evaluate(R, want=("eloc",))["eloc"].mean())
    ctx.dmc_advance([d0, d1], W, 1, 9, 0, 0.01, et, W)
    out, td = _timed(lambda: ctx.dmc_advance([d0, d1], W, nst, 9, 1, 0.01, et, W))
    print(json.dumps({"metric": "configurations/s (E_L with pseudopotentials)", "value": W / t,
                      "unit": "configurations/s", "n_gpus": 1, "walkers": W, "dtype": "f64",
                      "evaluate_ms": t * 1e3, "evaluate_without_ecp_ms": t0 * 1e3,
                      "ratio_points_per_config": pts, "vmc_walker_steps_per_s": W * nst / tv,
                      "dmc_walker_steps_per_s": W * nst / td,
                      "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
                                   "flops_per_config": fl, "traffic": None},
                      "config": {"workload": "F2 valence: 2 pseudo-nuclei (Z_eff 7), 14 electrons, 28 Gaussian "
                                             "basis functions, 3 VB structures, s + p nonlocal channels"}}))


HEADLINE_METRIC = "walker-moves/sec incl. E_L; mixed-prec & adjoint vs FP64 plain at \u0394E\u22641e-5 Ha"
DMC_KERNEL_NAMES = {1: "k_dmc_step<256, 0>", 2: "electron-major launches (k_dmcb_*)", 3: "k_dmcw<32, 2, 16, false, false>"}
# HBM bytes of one launch of the walker-resident DMC step kernel on the
# the headline workload (32768 walkers, one step launch of the walker-resident
# kernel), and one step launch of that kernel in VMC mode on the 40-electron
# molecule (16384 walkers; the mean of 12 step dispatches); see SWEEP_TRAFFIC
DMCW_TRAFFIC = {"src": "vbqmc_dmcw.hip", "src_sha": "aa2f209f56d80e78", "fetch_kib": 3408928.9, "write_kib": 4309978.0,
                "fetch_factor": 2.000, "write_factor": 1.000, "walkers": 32768}
WRES_VMC_TRAFFIC = {"src": "vbqmc_dmcw.hip", "src_sha": "aa2f209f56d80e78", "fetch_kib": 353397.0, "write_kib": 593276.6,
                    "fetch_factor": 2.000, "write_factor": 1.000, "walkers": 16384}
# headers every kernel source includes (their layouts and device helpers)
SHARED_HEADERS = ("vbqmc_internal.h", "vbqmc_device.h", "vbqmc_group.h")


def traffic_bytes(t):
    """Calibrated HBM bytes per launch of a traffic record, or None when its
    kernel source or a shared header changed since the counters were taken."""
    if not t.get("src_sha") or _src_sha(t["src"]) != t["src_sha"]:
        return None
    return (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"]) * 1024


def dmc_flops_per_walker_step(ctx, system, accept, refresh_per_step):
    """Algorithmic FLOPs of one DMC step of one walker on the walker-resident
    kernel (N drift-diffusion moves, the refreshes, one local energy), from
    the system's dimensions (P primitives, M basis functions, No orbitals, and
    per spin n electrons, nP table orbitals, nU distinct determinants).

    Per move of an electron of spin (n, nP, nU): value and gradient basis
    functions at the proposal (per primitive one exp + 6, per function 15),
    their contraction (4 channels x 2 M No); the drift at the current point
    (3 row products 2 n (n + nP) with the cached gradient rows, 3 nU x 10 for
    the determinant lanes); the ratio and the drift at the proposal (4 row
    products, nU x 10 + 3 nU x 15); Jastrow: per partner (N - 1 + nuclei) two
    pair functions with derivatives (25 each) and one value (12); per accepted
    move the Sherman-Morrison update (2 n (n + nP) + 8 nU).
    Per electron in the local energy: the Laplacian basis functions (per
    primitive one exp + 8, per function 3) and their contraction (2 M No),
    4 row products and 4 nU x 10, and per partner one pair function with
    derivatives (25) and 10 for the gradient, Laplacian and potential sums.
    Per refresh of a spin: Gauss-Jordan 2 n^3 and the table 2 n^2 nP."""
    N, M, norb, nnuc, P, spins = _dims(ctx, system)
    partners = N - 1 + nnuc
    tot = 0.0
    for s, (n, nP, nU) in enumerate(spins):
        if n == 0:
            continue
        row = 2 * n * (n + nP)
        move = (P * (EXP_FLOPS + 6) + 15 * M) + 4 * 2 * M * norb + (3 * row + 30 * nU) + \
            (4 * row + 10 * nU + 45 * nU) + partners * (2 * 25 + 12) + accept * (row + 8 * nU)
        eloc = (P * (EXP_FLOPS + 8) + 3 * M) + 2 * M * norb + 4 * row + 40 * nU + partners * 35
        tot += n * (move + eloc) + refresh_per_step[s] * (2 * n ** 3 + 2 * n * n * nP)
    return tot


# f_een (Sec. 2.1) cost per (electron i, partner j, nucleus) triple, counted
# low: the powers of the three scaled distances (12) and, per term of the
# 23, the value (5 FLOP), with the first partial derivatives in a and b (11)
# plus the chain rule into grad_i (15), or with the second ones as well (18)
# plus the chain rule into grad_i and lap_i (30)
EEN_TRIPLE_FLOPS = {"value": 12 + 23 * 5, "grad": 12 + 23 * 11 + 15, "lap": 12 + 23 * 18 + 30}


def wres_kernel_name(ctx, vmc):
    """The walker-resident kernel a system with f_een launches: three
    replaced columns, the k-steps per wave of its basis padded to 16
    functions (one k-step of four per 16), VMC or DMC form."""
    kper = -(-ctx.info["n_basis"] // 16)
    lk = 4 if kper <= 4 else 8 if kper <= 8 else 16
    return f"k_dmcw<32, 3, {lk}, {'true' if vmc else 'false'}, true>"


def een_flops_per_walker_step(ctx, dmc):
    """f_een FLOPs of one step of one walker on the walker-resident kernel:
    per move the pair sums of the moving electron at its current point and at
    the proposal ((N - 1) partners x nuclei triples each, with the gradient
    for the DMC drift, values only for VMC), and in E_L every electron's
    gradient and Laplacian (N (N - 1) x nuclei triples)."""
    N, nn = ctx.N, ctx.info["n_nuclei"]
    move = EEN_TRIPLE_FLOPS["grad" if dmc else "value"]
    return 2 * N * (N - 1) * nn * move + N * (N - 1) * nn * EEN_TRIPLE_FLOPS["lap"]


def cpu_baseline_dmc(system, walkers=64, steps=5, seed=13):
    """The oracle's DMC (plain FP64 CPU code, OpenMP over walkers, every
    determinant by a fresh LU for every proposal) on a bounded sample of the
    same workload: `walkers` walkers x `steps` steps from the same start."""
    import numpy as np
    import oracle
    import systems as S
    o = oracle.Oracle(system)
    R0 = S.initial_walkers(system, walkers, seed=seed)
    e0 = o.evaluate(R0)["eloc"]
    t0 = time.perf_counter()
    r = o.dmc(R0, e0, steps, 2022, 0, 0.005, float(np.median(e0)), walkers, capacity=4 * walkers)
    dt = time.perf_counter() - t0
    moves = float(r["pop"].sum())
    return {"value": moves / dt, "unit": "walker-moves/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{walkers} walkers x {steps} DMC steps of the same molecule (tau 0.005), {dt:.1f} s"}


def reblock(x, w):
    """Weighted mean of a serially correlated series and its error bar by
    blocking (Flyvbjerg and Petersen 1989): pairs of consecutive blocks are
    merged level by level (weighted means), the naive standard error of the
    block means is taken at each level with at least 4 blocks, and the largest
    is reported (the plateau value for a long enough series; conservative for
    a short one).  Returns (mean, error, levels)."""
    import numpy as np
    x, w = np.asarray(x, float), np.asarray(w, float)
    mean = float((w * x).sum() / w.sum())
    best, levels = 0.0, 0
    while len(x) >= 4:
        ww = w / w.sum()
        var = float((ww * (x - mean) ** 2).sum() / (1.0 - (ww * ww).sum()))
        neff = 1.0 / (ww * ww).sum()
        best = max(best, (var / neff) ** 0.5)
        levels += 1
        m = len(x) // 2
        xs, ws = x[:2 * m].reshape(m, 2), w[:2 * m].reshape(m, 2)
        w = ws.sum(axis=1)
        x = (xs * ws).sum(axis=1) / w
    return mean, best, levels


def _src_sha(name):
    """SHA-256 prefix of a kernel source file followed by the shared headers."""
    import hashlib
    h = hashlib.sha256()
    for n in (name,) + SHARED_HEADERS:
        with open(os.path.join(ROOT, "paper_2207_14715_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _dmc_mixed_compare(vb, system, c64, R_burn, W, tau, fp64_value, steps=10):
    """The mixed-precision DMC form (FP32 proposal rows, FP64 determinants and
    E_L) from the same burn-in walkers: walker-moves/s over `steps` timed
    steps (after one warm-up step) and, at the configurations those steps
    leave, each walker's recorded E_L against an FP64 evaluation."""
    import numpy as np
    import torch
    cm = vb.Context(system, precision="mixed")
    st = [cm.new_state(3 * W), cm.new_state(3 * W)]
    cm.walkers_init(R_burn, st[0])
    et = float(cm.record_eloc(st[0], W).median().item())
    out = cm.dmc_advance(st, W, 1, 4044, 0, tau, et, W)
    Wc, et = out["W"], out["e_trial"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = cm.dmc_advance(st, Wc, steps, 4044, 1, tau, et, W)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    moves = float(out["pop"].sum().item())
    Wn = out["W"]
    e_rec = cm.record_eloc(st[0], Wn)
    e_64 = c64.evaluate(cm.positions(st[0], Wn).contiguous(), want=("eloc",))["eloc"]
    d = (e_rec - e_64).abs().cpu().numpy()
    del st
    torch.cuda.empty_cache()
    return {"value": moves / wall, "unit": "walker-moves/s", "steps": steps,
            "dmc_kernel": {1: "workgroup per walker", 2: "electron-major", 3: "walker-resident"}[cm.info["dmc_kernel"]],
            "speed_vs_fp64": moves / wall / fp64_value,
            "abs_dEL_max": float(np.nanmax(d)), "abs_dEL_p99": float(np.nanpercentile(d, 99)),
            "abs_dEL_median": float(np.nanmedian(d)), "meets_1e-5": bool(np.nanmax(d) <= 1e-5)}


def dmc_form(args):
    """The headline: fixed-node DMC on the 16-nucleus, 64-electron,
    240-function, 32-structure / 128-determinant molecule with 32768 target
    walkers, tau = 0.005.  Walkers start from a short FP64 VMC burn-in; the
    warm-up call and the timed call of `steps` steps (default 100, against
    the workload's 5000-step runs) each begin by rebuilding the records from
    their positions (one launch, amortised over the call).  walker-moves/s counts the walkers
    present at each timed step over the wall time of the timed call; the
    dominant kernel (the per-step move-and-energy kernel) is timed with HIP
    events on the launch stream inside the library (log step_ms)."""
    import numpy as np
    import torch

    import paper_2207_14715_amd as vb
    import systems as S
    system = S.dmc_molecule()
    if args.een:
        system = S.with_een(system, scale=args.een_scale)
    W = args.walkers or 32768
    steps = args.steps if args.steps is not None else (20 if args.een else 100)
    warm = args.warmup if args.warmup is not None else 3
    tau = 0.005
    c64 = vb.Context(system, dmc_kernel=args.dmc_kernel)
    ctx = c64 if args.precision == "fp64" else vb.Context(system, dmc_kernel=args.dmc_kernel,
                                                          precision=args.precision)
    cap = 3 * W
    st = [ctx.new_state(cap), ctx.new_state(cap)]
    R0 = torch.from_numpy(S.initial_walkers(system, W, seed=13)).cuda()
    # FP64 burn-in for every form, so that the forms start from the same walkers
    c64.walkers_init(R0, st[0])
    c64.vmc_advance(st[0], 3, 17, 0, 0.3, False, None, W)
    R_burn = c64.positions(st[0], W).clone()
    # the synthetic trial function has a wide E_L distribution: start E_T at
    # the median
    et = float(c64.record_eloc(st[0], W).median().item())
    Wc = W
    if warm > 0:
        out = ctx.dmc_advance(st, W, warm, 2022, 0, tau, et, W)
        Wc, et = out["W"], out["e_trial"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.dmc_advance(st, Wc, steps, 2022, warm, tau, et, W, time_steps=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pop = out["pop"].cpu().numpy()
    moves = float(pop.sum())
    accept = float(out["n_accept"].sum().item() / max(out["n_prop"].sum().item(), 1))
    e_mixed = float(out["wesum"].sum().item() / out["wsum"].sum().item())
    e_mixed_clipped = float(out["wcsum"].sum().item() / out["wsum"].sum().item())
    # effective time step of the moves with rejections: tau <|dr|^2 accepted> / <|dr|^2 proposed>
    tau_eff = tau * float(out["dr2_acc"].sum().item() / out["dr2_prop"].sum().item())
    ws_np = out["wsum"].cpu().numpy()
    _, e_clip_err, e_clip_levels = reblock(out["wcsum"].cpu().numpy() / ws_np, ws_np)
    kern = ctx.info["dmc_kernel"]
    step_ms = out["step_ms"]
    nupd_rate = [accept * n / 32.0 for n in (ctx.info["n_up"], ctx.info["n_dn"])]  # refreshes per step per spin
    fl_walker = dmc_flops_per_walker_step(ctx, system, accept, nupd_rate)
    if args.een:
        fl_walker += een_flops_per_walker_step(ctx, True)
    flops_launch = fl_walker * float(pop.mean())
    kavg = float(np.mean(step_ms)) / 1e3
    achieved = flops_launch / kavg / 1e12
    traffic = None
    if kern == 3 and args.precision == "fp64" and W == DMCW_TRAFFIC["walkers"] and not args.een:
        traffic = traffic_bytes(DMCW_TRAFFIC)
    line = {
        "metric": HEADLINE_METRIC,
        "value": moves / wall,
        "unit": "walker-moves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": _dtype(args.precision),
        "data": "synthetic",
        "config": {"workload": "fixed-node DMC of the 64-electron synthetic molecule: 16 nuclei (Z in {1,6,8}), "
                               "32 up + 32 down electrons, 240 Gaussian basis functions, 32 VB structures / 128 "
                               "determinants, Pade Jastrow" +
                               (f" with the three-body f_een (23 coefficients per element ~ N(0, {args.een_scale}^2))"
                                if args.een else "") +
                               ", 32768 target walkers, tau = 0.005, per-electron "
                               "drift-diffusion moves, E_L every step, branching with +-10 % population control",
                   "target_walkers": W, "electrons": ctx.N, "precision": args.precision,
                   "dmc_kernel": {1: "workgroup per walker", 2: "electron-major", 3: "walker-resident"}[kern]},
        "electron_moves_per_s": moves * ctx.N / wall,
        "acceptance": accept,
        "tau_eff": tau_eff,
        "population": [int(p) for p in pop],
        "population_band": [float(pop.min() / W - 1), float(pop.max() / W - 1)],
        "e_trial": out["e_trial"],
        "e_mixed": e_mixed,
        "e_mixed_clipped": e_mixed_clipped,
        "e_mixed_clipped_err": e_clip_err,
        "e_mixed_clipped_blocking_levels": e_clip_levels,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": wres_kernel_name(ctx, False) if args.een else DMC_KERNEL_NAMES[kern],
                     "kernel_avg_ms_per_launch": kavg * 1e3,
                     "kernel_share_of_step": float(np.sum(step_ms) / 1e3 / wall),
                     "flops_per_launch": flops_launch, "flops_per_walker_step": fl_walker,
                     "walkers_per_launch": float(pop.mean())},
    }
    if args.precision == "fp64" and not args.een and not args.no_precision_compare:
        del st
        torch.cuda.empty_cache()
        line["mixed_precision"] = _dmc_mixed_compare(vb, system, c64, R_burn, W, tau, line["value"])
    if not args.no_cpu_baseline:
        # (the oracle's f_een gradients by jets cost about 50x: a smaller sample)
        line["cpu_baseline"] = cpu_baseline_dmc(system, walkers=32, steps=2) if args.een else cpu_baseline_dmc(system)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
