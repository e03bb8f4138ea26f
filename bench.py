"""Benchmark: Split Bregman reconstructions per second at 256 x 256, 12 coils
(line mask R = 4, 24 centre lines, TV + 3-level Daubechies-4, mu = 1e-3,
lambda = gamma = 4e-3, 20 outer iterations, PCG tolerance 1e-3) with the
circulant preconditioner, and PCG iterations to 1e-3 for none / circulant.

One step = build the preconditioner + one full reconstruction of every slice
of the batch (all rows of the hot path: spectrum build, system operator,
preconditioner, PCG updates, Split Bregman steps).  The batch is split into
independent contexts (default 3 x 128 slices), each with its own stream and
host thread, so that their kernel chains overlap on the GPU.  Inputs are
synthetic (seeded phantoms, coil maps, masks, noise) and resident in HBM
before timing.

Prints ONE JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1710_01758_amd import inputs as gen  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def apply_bytes(specs) -> int:
    """Algorithmic HBM bytes of one apply_A over the batch: read x and the coil
    maps, write y, 8 bytes per complex64 element: 8 N (N_c + 2) per slice."""
    return int(sum(8 * s.m * s.n * (s.ncoils + 2) for s in specs))


def reconstruction_bytes(spec, pcg_iters: int, n_outer: int = 20) -> int:
    """Algorithmic HBM bytes of one slice's Split Bregman reconstruction with
    the circulant preconditioner (build included, n_inner = 1), from each
    kernel's reads and writes of image- and coil-shaped arrays (8 bytes per
    complex64 element, 4 per float), given the slice's total PCG iterations:
      build            (8 N_c + 20) N   coil maps, coil energy, k and 1/k
      initialisation   (24 N_c f + 8 N_c + 32) N   sampled k-space rows (f of
                       them) through the row pass, coil maps, g_1 g rhs x
      first set-up     (8 N_c + 92) N   operator on x_0, row / column / row pass
      later set-ups    76 N each        r = b - q, M^-1 r
      shrinks          (140 + sum_l 44 / 4^l) N per outer iteration: level-0
                       analysis with TV shrink and outer update 116, level-0
                       synthesis 24, coarser levels l = 1.. 28 + 16 per 4^l
      PCG iteration    (8 N_c + 132) N  operator 8 N_c + 32, row pass 56,
                       column pass 20, row pass 24"""
    N = spec.m * spec.n
    C = spec.ncoils
    f = round(spec.m / spec.accel) / spec.m
    coarse = sum(44.0 / 4 ** l for l in range(1, spec.levels)) if spec.levels > 0 else 0.0
    per_px = ((8 * C + 20) + (24 * C * f + 8 * C + 32) + (8 * C + 92) + 76 * (n_outer - 1)
              + n_outer * (140 + coarse) + pcg_iters * (8 * C + 132))
    return int(per_px * N)


def hold_stream(torch, stream, cycles=100_000_000):
    """Enqueue a spin kernel (tens of milliseconds at the counter rate seen
    on MI355X, about 3.6e6 counts per ms) on `stream`, so that the work
    enqueued behind it runs back to back however slowly the host submits it."""
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(cycles))


def time_apply_kernel(torch, ctx, xd, yd, reps=50, terms=None):
    """Average duration of one apply_A call (for a slice context one launch
    of the fused operator kernel): a pair of HIP events recorded on the library's stream around
    each of `reps` calls, enqueued behind a spin kernel so that they run back
    to back on the GPU; the per-launch elapsed times are averaged (the gaps
    between launches are not counted)."""
    stream = torch.cuda.ExternalStream(ctx.stream) if ctx.stream else torch.cuda.current_stream()
    kw = {} if terms is None else {"terms": terms}
    for _ in range(5):
        ctx.apply_A(xd, yd, **kw)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    hold_stream(torch, stream)
    for e0, e1 in ev:
        e0.record(stream)
        ctx.apply_A(xd, yd, **kw)
        e1.record(stream)
    ev[-1][1].synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps * 1e-3  # seconds


COPY_CAL_BYTES = 256 * 2**20


def copy_calibration(torch):
    """A plain device copy of COPY_CAL_BYTES (read + write of known size);
    its FETCH_SIZE / WRITE_SIZE counters calibrate the apply kernel's."""
    src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src, dst


def run_apply_mode(torch, ctx, insts):
    xa = torch.randn(ctx.image_elems, dtype=torch.complex64, device="cuda")
    ya = torch.empty_like(xa)
    t_apply = time_apply_kernel(torch, ctx, xa, ya, reps=20)
    copy_calibration(torch)
    b = apply_bytes([i.spec for i in insts])
    print(json.dumps({"apply_avg_us": round(t_apply * 1e6, 2), "bytes_per_launch": b,
                      "achieved_GBs": round(b / t_apply / 1e9, 1), "copy_cal_bytes": COPY_CAL_BYTES}), flush=True)


def run_apply_ragged(torch, B):
    """The ragged 64-slice batch's operator: the whole batch (size groups on
    side streams), then each size group alone in its own context (one JSON
    line each)."""
    specs = gen.ragged_specs()
    insts = [gen.make_instance(sp, gen.eval_seed(4, i)) for i, sp in enumerate(specs)]
    groups = [("all", insts)]
    for shape in gen.RAGGED_SHAPES:
        groups.append((f"{shape[0]}x{shape[1]}", [it for it in insts if (it.spec.m, it.spec.n) == shape]))
    for label, gi in groups:
        ctx, _ = B.context_for(gi)
        split = ctx.autotune()
        xa = torch.randn(ctx.image_elems, dtype=torch.complex64, device="cuda")
        ya = torch.empty_like(xa)
        t = time_apply_kernel(torch, ctx, xa, ya, reps=20)
        b = apply_bytes([i.spec for i in gi])
        print(json.dumps({"group": label, "slices": len(gi), "coils": sum(i.spec.ncoils for i in gi),
                          "coil_split": split, "apply_avg_us": round(t * 1e6, 2), "bytes_per_launch": b,
                          "achieved_GBs": round(b / t / 1e9, 1)}), flush=True)
        ctx.close()
    copy_calibration(torch)  # for counter runs: a copy of known size


def run_step_mode(torch, B, spec, steps):
    """One context of ROOFLINE_BATCH headline slices, no autotuning (the
    batch keeps the default launch shape): preconditioner build + Split
    Bregman reconstruction, 1 + `steps` times; prints the PCG iterations per
    reconstruction.  Every kernel of the run belongs to these steps, so
    whole-run counter totals divided by 1 + steps are per batch
    reconstruction."""
    insts = [gen.make_instance(spec, gen.eval_seed(2, i)) for i in range(ROOFLINE_BATCH)]
    ctx, ksp = B.context_for(insts)
    x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")
    for k in range(1 + steps):
        ctx.build_preconditioner("circulant")
        it, _ = ctx.split_bregman_recon(ksp, x, n_outer=20, n_inner=1, tol=1e-3, maxit=1000)
        print(json.dumps({"reconstruction": k, "slices": ROOFLINE_BATCH, "pcg_iters_total": int(it.sum()),
                          "pcg_iters_per_solve_mean": round(float(it.mean()), 3)}), flush=True)
    torch.cuda.synchronize()
    ctx.close()


def run_pcg_mode(torch, ctx, iters=10, reps=5):
    """Iteration-locked PCG solves (every slice runs exactly `iters`
    iterations from x = 0, circulant preconditioner), so that every launch
    of the PCG kernels works on the whole batch (for kernel traces)."""
    ctx.build_preconditioner("circulant")
    b = torch.randn(ctx.image_elems, dtype=torch.complex64, device="cuda")
    x = torch.zeros_like(b)
    lock = [iters] * ctx.n
    ctx.pcg_solve(b, x, 0.0, 0, maxit_per_slice=lock)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x.zero_()
        ctx.pcg_solve(b, x, 0.0, 0, maxit_per_slice=lock)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"pcg_iters": iters, "slices": ctx.n, "ms_per_solve": round(dt * 1e3, 3),
                      "us_per_iteration": round(dt / iters * 1e6, 2)}), flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "apply_A_256x256x12_batch128_hbm_traffic.md")
VALU_PROFILE = os.path.join(ROOT, "profiles", "apply_A_256x256x12_batch128_valu.md")
SIMDS, PEAK_CLOCK_HZ = 1024, 2.4e9  # 256 CUs x 4 SIMDs; a wave64 FP32 VALU op issues in 4 cycles
ROOFLINE_BATCH = 128  # slices per apply_A launch in the roofline measurement and the counter summaries


def profile_fields(path):
    """The `key: value` lines of a committed counter summary, or None if the
    kernel sources changed since the counters were taken."""
    import hashlib
    try:
        txt = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and not line.startswith(("|", "#")))
    try:
        h = hashlib.sha256()
        for f in fields["kernel_source_files"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"].strip():
            return None
    except (KeyError, OSError):
        return None
    return fields


def measured_traffic():
    """HBM bytes per apply_A launch from the committed counter summary, or None
    if the kernel sources changed since the counters were taken."""
    f = profile_fields(TRAFFIC_PROFILE)
    try:
        return int(f["traffic_bytes_per_launch"]) if f else None
    except (KeyError, ValueError):
        return None


def valu_roofline(avg_s):
    """The apply kernel against its vector-ALU issue bound: counted wave64 VALU
    instructions per launch (committed counter summary) x 4 cycles over the
    1024 SIMDs at the 2.4 GHz peak clock, against this run's launch time."""
    f = profile_fields(VALU_PROFILE)
    try:
        instr = float(f["valu_wave_instr_per_launch"]) if f else None
    except (KeyError, ValueError):
        instr = None
    if instr is None:
        return None
    floor = instr * 4 / (SIMDS * PEAK_CLOCK_HZ)
    return {"bound": "alu", "valu_wave_instr_per_launch": int(instr), "floor_us_at_peak_clock": round(floor * 1e6, 2),
            "frac": round(floor / avg_s, 4)}


def cpu_baseline(inst, min_seconds=10.0):
    """The FP64 oracle (Algorithm 1 as written, circulant preconditioner) on
    full 20-iteration reconstructions of one 256^2 x 12 slice, repeated until
    at least `min_seconds` of CPU work."""
    from threadpoolctl import threadpool_limits

    from oracle import sb as osb
    s = inst.spec
    t0 = time.perf_counter()
    count = 0
    with threadpool_limits(limits=1):  # one core: BLAS and OpenMP pools held to one thread
        while True:
            ref = osb.split_bregman(inst.kspace, inst.sens, inst.mask, s.mu, s.lam, s.gam, s.wavelet, s.levels,
                                    n_outer=20, tol=1e-3, precond="circulant")
            count += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                break
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(count / dt, 4), "unit": "recons/s", "cores": 1, "kind": "oracle",
            "host": f"{model}, os.cpu_count() = {os.cpu_count()}",
            "sample": f"{count} full reconstructions (20 outer iterations, circulant, build included) of one "
                      f"256x256x12 slice in FP64 NumPy with single-threaded pocketfft, {dt:.1f} s",
            "result": ref}


def parity_against_oracle(torch, B, inst, ref):
    """The GPU reconstruction of the slice the oracle baseline reconstructed,
    with each PCG solve locked to the oracle's count: relative image error
    against the FP64 result, and the GPU's free-running counts beside the
    oracle's."""
    ctx, ksp = B.context_for([inst])
    ctx.build_preconditioner("circulant")
    x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")
    lock = np.array(ref.pcg_iters, np.int32).reshape(-1, 1)
    ctx.split_bregman_recon(ksp, x, n_outer=len(ref.pcg_iters), lock=lock)
    got = x.cpu().numpy().reshape(ref.x.shape).astype(np.complex128)
    err = float(np.linalg.norm(got - ref.x) / np.linalg.norm(ref.x))
    x.zero_()
    free, _ = ctx.split_bregman_recon(ksp, x, n_outer=len(ref.pcg_iters), tol=1e-3, maxit=1000)
    ctx.close()
    return {"rel_err_locked_split_bregman": err, "oracle_pcg_iters": [int(v) for v in ref.pcg_iters],
            "gpu_pcg_iters_free_running": free[:, 0].tolist(),
            "note": "the slice the one-core oracle reconstructed, GPU locked to the oracle's per-solve PCG counts"}


def cpu_worker(seconds: float) -> None:
    """One single-threaded oracle process of the all-cores baseline: full
    reconstructions of the headline slice until `seconds` have passed; prints
    {"count", "seconds"} as JSON."""
    from threadpoolctl import threadpool_limits

    from oracle import sb as osb
    spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)
    inst = gen.make_instance(spec, gen.eval_seed(2, 0))
    t0 = time.perf_counter()
    count = 0
    with threadpool_limits(limits=1):
        while True:
            osb.split_bregman(inst.kspace, inst.sens, inst.mask, spec.mu, spec.lam, spec.gam, spec.wavelet,
                              spec.levels, n_outer=20, tol=1e-3, precond="circulant")
            count += 1
            dt = time.perf_counter() - t0
            if dt >= seconds:
                break
    print(json.dumps({"count": count, "seconds": dt}), flush=True)


def cpu_baseline_all_cores(procs: int, seconds: float = 10.0):
    """The oracle on `procs` host cores at once: independent single-threaded
    processes, one reconstruction after another each (slices are independent,
    so this is how a CPU would serve the batch).  Run before the GPU is
    touched: the workers are plain child processes of a GPU-free parent."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    ps = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(seconds)],
                           stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env) for _ in range(procs)]
    rate, count, longest = 0.0, 0, 0.0
    for p in ps:
        out, err = p.communicate(timeout=600)
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed: {err[-2000:]}")
        r = json.loads(out.strip().splitlines()[-1])
        rate += r["count"] / r["seconds"]
        count += r["count"]
        longest = max(longest, r["seconds"])
    return {"value": round(rate, 4), "unit": "recons/s", "cores": procs, "count": count, "seconds": round(longest, 1)}


def workload_section(torch, B, insts, label, steps=2):
    """Reconstructions per second and the apply_A roofline for another batch."""
    ctx, ksp = B.context_for(insts)
    split = ctx.autotune()
    x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")

    def run():
        ctx.build_preconditioner("circulant")
        return ctx.split_bregman_recon(ksp, x, n_outer=20, tol=1e-3, maxit=1000)[0]

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        it = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    xa = torch.randn(ctx.image_elems, dtype=torch.complex64, device="cuda")
    ya = torch.empty_like(xa)
    t_apply = time_apply_kernel(torch, ctx, xa, ya, reps=20)
    byts = apply_bytes([i.spec for i in insts])
    ctx.close()
    return {"workload": label, "slices": len(insts), "recons_per_s": round(len(insts) / dt, 2),
            "ms_per_batch": round(dt * 1e3, 3), "pcg_iters_total": int(it.sum()), "coil_split": split,
            "pcg_iters_first_solve_max": int(it[0].max()),
            "apply_roofline": {"bound": "hbm", "achieved": round(byts / t_apply / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(byts / t_apply / 1e9 / HBM_PEAK_GBS, 4),
                               "avg_us": round(t_apply * 1e6, 2), "bytes_per_launch": byts}}


def mask2d_section(torch, B, batch=32, steps=2):
    """The fully random variable-density 2D mask at 256 x 256 x 12 (R = 4,
    24 x 24 centre): reconstructions per second of a batch, PCG iterations of
    the first solve and over 20 Bregman iterations (none / circulant), and the
    apply_A rate against the algorithmic floor 8 N (N_c + 2) and against the
    three-pass traffic 8 N (5 N_c + 3) of the 2D-transform path."""
    spec = gen.SliceSpec(256, 256, 12, 4.0, 24, mask_kind="2d", wavelet="db4", levels=3)
    insts = [gen.make_instance(spec, gen.eval_seed(6, i)) for i in range(batch)]
    ctx, ksp = B.context_for(insts)
    x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")

    def run(kind="circulant"):
        ctx.build_preconditioner(kind)
        return ctx.split_bregman_recon(ksp, x, n_outer=20, tol=1e-3, maxit=1000)[0]

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        it = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    it_none = run("none")
    run()
    xa = torch.randn(ctx.image_elems, dtype=torch.complex64, device="cuda")
    ya = torch.empty_like(xa)
    t_apply = time_apply_kernel(torch, ctx, xa, ya, reps=20)
    n_pix = spec.m * spec.n * batch
    floor = 8 * n_pix * (spec.ncoils + 2)
    passes = 8 * n_pix * (5 * spec.ncoils + 3)
    ctx.close()
    return {"workload": "256x256, 12 coils, random variable-density 2D mask R=4 (24x24 centre), TV + db4 x3, "
                        f"batch of {batch}",
            "recons_per_s": round(batch / dt, 2), "ms_per_batch": round(dt * 1e3, 3),
            "pcg_iters": {"none": {"first_solve": int(it_none[0, 0]), "total_20_solves": int(it_none[:, 0].sum())},
                          "circulant": {"first_solve": int(it[0, 0]), "total_20_solves": int(it[:, 0].sum())}},
            "apply_A": {"avg_us": round(t_apply * 1e6, 2), "bytes_floor": floor, "bytes_three_pass": passes,
                        "GBs_vs_floor": round(floor / t_apply / 1e9, 1),
                        "GBs_three_pass": round(passes / t_apply / 1e9, 1),
                        "frac_three_pass": round(passes / t_apply / 1e9 / HBM_PEAK_GBS, 4)}}


def coil_compression_section(torch, B, batch=32, nvirt=6, steps=2):
    """Coil compression (the paper's Fig. 7 comparison) at 256 x 256 x 12:
    Split Bregman with all 12 coils and with the 6 most dominant virtual coils
    (circulant preconditioner rebuilt on them): reconstructions per second of
    a batch of 32 (compression included in the compressed timing), slice 0's
    PCG iterations per Bregman iteration and the retained coil energy; at the
    literal data scale and at 1e3."""
    out = {}
    for scale in (1.0, 1e3):
        spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3, data_scale=scale)
        insts = [gen.make_instance(spec, gen.eval_seed(2, i)) for i in range(batch)]
        ctx, ksp = B.context_for(insts)
        tot = nvirt * spec.m * spec.n * batch
        kout = torch.empty(tot, dtype=torch.complex64, device="cuda")
        sout = torch.empty(tot, dtype=torch.complex64, device="cuda")
        descs = [dict(B.spec_desc(spec), ncoils=nvirt) for _ in insts]
        masks = B.to_device(B.pack_masks([it.mask for it in insts]))
        eig = ctx.coil_compress(ksp, nvirt, kout, sout)
        cv = B.Context(descs, sout, masks)
        x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")

        def full():
            ctx.build_preconditioner("circulant")
            return ctx.split_bregman_recon(ksp, x, n_outer=20, tol=1e-3, maxit=1000)[0]

        def compressed():
            ctx.coil_compress(ksp, nvirt, kout, sout)
            cv.build_preconditioner("circulant")
            return cv.split_bregman_recon(kout, x, n_outer=20, tol=1e-3, maxit=1000)[0]

        row = {}
        for name, fn in (("all_12_coils", full), (f"virtual_{nvirt}_coils", compressed)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                it = fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            row[name] = {"recons_per_s": round(batch / dt, 1), "slice0_per_bregman_iteration": it[:, 0].tolist(),
                         "mean_total": float(it.sum(axis=0).mean())}
        w = eig[:spec.ncoils]
        row["retained_energy_slice0"] = round(float(w[:nvirt].sum() / w.sum()), 6)
        out[f"data_scale_{scale:g}"] = row
        ctx.close()
        cv.close()
    return out


def volume_section(torch, B):
    """The 3D extension on a 128 x 256 x 256 volume with 8 coils (2D random
    variable-density pattern over (z, y), fully sampled along x, R = 4): PCG
    from 0 to 1e-3 with none and with the 3D circulant preconditioner
    (iterations, seconds), the preconditioner build and one operator
    application."""
    spec = gen.VolumeSpec(128, 256, 256, 8, 4.0, 24)
    inst = gen.make_volume_instance(spec, gen.eval_seed(9))
    vol, ksp = B.volume_for(inst)
    b = torch.empty(vol.voxels, dtype=torch.complex64, device="cuda")
    vol.rhs(ksp, b)
    out = {"workload": "volume 128x256x256, 8 coils, random VD (z, y) pattern R=4, 24x24 centre, fully sampled x"}
    for kind in ("none", "circulant"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vol.build_preconditioner(kind)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        x = torch.zeros_like(b)
        t0 = time.perf_counter()
        it, rel, _ = vol.pcg_solve(b, x, 1e-3, 500)
        torch.cuda.synchronize()
        out[kind] = {"pcg_iters": it, "relres": rel, "solve_s": round(time.perf_counter() - t0, 4),
                     "build_s": round(tb, 4)}
    y = torch.empty_like(b)
    # one operator application (all its x chunks and passes) per timed call,
    # at every admissible chunk width and at the automatic one
    sweep = {}
    for X in [c for c in range(16, spec.n + 1, 16) if spec.n % c == 0] + [0]:
        vol.set_option(B.OPT3_XCHUNK, X)
        sweep[X or "auto"] = time_apply_kernel(torch, vol, b, y, reps=10)
    X = vol.get_option(B.OPT3_XCHUNK)
    t_apply = sweep["auto"]
    floor = 8 * spec.p * spec.m * spec.n * (spec.ncoils + 2)
    out["apply_A_ms"] = round(t_apply * 1e3, 3)
    out["x_chunk"] = X
    out["apply_A_ms_per_x_chunk"] = {str(k): round(v * 1e3, 3) for k, v in sweep.items()}
    out["apply_roofline"] = {"bound": "hbm", "achieved": round(floor / t_apply / 1e9, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(floor / t_apply / 1e9 / HBM_PEAK_GBS, 4),
                             "bytes_per_launch": floor,
                             "note": "algorithmic floor 8 V (N_c + 2): read x and the coil maps, write y; "
                                     "one application = three passes per x chunk"}
    vol.close()
    return out


def param_sets_section(torch, B, nslices=8):
    """PCG iterations per Bregman iteration for the paper's three parameter
    sets with none / Jacobi / circulant at 256 x 256 x 12 (the structure of the
    paper's Fig. 5): slice 0's per-solve counts, the batch-mean total over 20
    Bregman iterations and the none / circulant gain, at the literal data scale
    and at 1e3 (shrinks active)."""
    out = {}
    for scale in (1.0, 1e3):
        rows = {}
        for sid, (mu, lam, gam) in gen.PARAM_SETS.items():
            spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3, mu=mu, lam=lam, gam=gam,
                                 data_scale=scale)
            insts = [gen.make_instance(spec, gen.eval_seed(2, i)) for i in range(nslices)]
            ctx, ksp = B.context_for(insts)
            row = {"mu": mu, "lambda": lam, "gamma": gam}
            for kind in ("none", "jacobi", "circulant"):
                ctx.build_preconditioner(kind)
                x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")
                it, _ = ctx.split_bregman_recon(ksp, x, n_outer=20, tol=1e-3, maxit=1000)
                row[kind] = {"slice0_per_bregman_iteration": it[:, 0].tolist(),
                             "mean_total": float(it.sum(axis=0).mean())}
            row["gain_total"] = round(row["none"]["mean_total"] / row["circulant"]["mean_total"], 2)
            row["gain_first"] = round(float(np.mean([row["none"]["slice0_per_bregman_iteration"][0]]))
                                      / max(1, row["circulant"]["slice0_per_bregman_iteration"][0]), 2)
            rows[f"set{sid}"] = row
            ctx.close()
        out[f"data_scale_{scale:g}"] = rows
    return out


def superoptimal_loss(data) -> float:
    """Reporting: the loss floor of a per-instance diagonal d = H / G (each
    instance's own per-frequency optimum), from the probe statistics."""
    G = data.G.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    H = data.H.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    Z = data.Z.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    per = (Z - H * H / G).sum(axis=1) / Z.sum(axis=1)
    return float(per.mean())


def superoptimal_correction(torch, B, instance, nprobes: int = 32, probe_seed: int = 97_000):
    """Reporting: probe estimate of the per-frequency optimum c* = G / (k H)
    of the loss at the slice's own resolution (the ceiling of any spectrum
    correction), from the library's spectrum and probe statistics."""
    ctx, _ = B.context_for([instance])
    s = instance.spec
    khat = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    ctx.build_preconditioner("circulant", khat=khat)
    probes = np.stack([gen.probe_vectors(probe_seed + p, 1, s.m, s.n)[0].ravel() for p in range(nprobes)])
    pd = B.to_device(probes.astype(np.complex64).ravel())
    G = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    H = torch.empty_like(G)
    Z = torch.empty_like(G)
    ctx.probe_stats(pd, nprobes, G, H, Z)
    c = (G.double() / (khat.double() * H.double())).float()
    ctx.close()
    return c


def learned_section(torch, B, steps):
    """Train the spectrum correction on 2000 instances of the 64 x 64 x 4
    training distribution (random R in [2, 8], mu / lambda / gamma within a
    decade), report held-out losses (200 instances) and compare circulant with
    learned on the 256 x 256 x 12 slice: Split Bregman per-solve PCG counts and
    a PCG solve of A x = A x_true from 0 (iterations to 1e-3, relative residual
    after 0..3 iterations); the same solve for two harder operators (mu = 1e-2
    and 1e-1) beside the superoptimal diagonal's count."""
    from paper_1710_01758_amd import learned as LD
    t0 = time.perf_counter()
    log("bench: learned - building datasets")
    train = LD.build_dataset(gen.training_instances(2000, base=gen.TRAIN_SEED_BASE), nprobes=8)
    held = LD.build_dataset(gen.training_instances(200, base=gen.HELDOUT_SEED_BASE), nprobes=8, probe_seed=95_000)
    net = B.Net(16)
    net.set_params(gen.net_init(20_260).astype(np.float32))
    circ = LD.dataset_loss(net, held)
    tr0 = LD.dataset_loss(net, train)
    t1 = time.perf_counter()
    LD.train(net, train, steps=steps, batch=16, lr=1e-3, log_every=500, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    learned = LD.dataset_loss(net, held)
    tr1 = LD.dataset_loss(net, train)
    floor = superoptimal_loss(held)
    tfloor = superoptimal_loss(train)
    inst = gen.make_instance(gen.LEARNED_SLICE, gen.eval_seed(5))
    sb = LD.evaluate_on(inst, net, n_outer=20)
    pcg = LD.pcg_first_solve(inst, net, curve=3)
    inst_s = gen.make_instance(gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3, data_scale=1e3),
                               gen.eval_seed(5))
    sb_scaled = LD.evaluate_on(inst_s, net, n_outer=20)
    ceiling = LD.evaluate_correction(inst, superoptimal_correction(torch, B, inst, nprobes=32))
    # harder operators at 256 x 256 x 12: parameter set 2 (mu = 1e-2, inside
    # the training range) and mu = 1e-1 (data term dominant, outside it); the
    # probe-estimated superoptimal diagonal bounds what any spectrum
    # correction can reach
    harder = {}
    for label, mu in (("mu_1e-2", 1e-2), ("mu_1e-1", 1e-1)):
        inst_h = gen.make_instance(gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3, mu=mu, lam=4e-3,
                                                 gam=1e-3), gen.eval_seed(5))
        ceil_h = LD.evaluate_correction(inst_h, superoptimal_correction(torch, B, inst_h, nprobes=32), n_outer=2)
        harder[label] = {"pcg_from_zero": LD.pcg_first_solve(inst_h, net, curve=3),
                         "superoptimal_probe_ceiling_iters_to_1e-3": ceil_h["pcg_iters_to_1e-3"]}
    for d in (train, held):
        d.ctx.close()
    net.close()
    return {
        "train": {"instances": 2000, "steps": steps, "batch": 16, "lr": 1e-3, "seconds": round(t_train, 2),
                  "loss_initial": tr0, "loss_final": tr1, "superoptimal_floor": tfloor,
                  "gap_closed": (tr0 - tr1) / (tr0 - tfloor) if tr0 > tfloor else None,
                  "note": "mean loss over all 2000 training instances before and after training; the network starts "
                          "at correction 1 (the circulant spectrum)"},
        "heldout_loss": {"circulant": circ, "learned": learned, "superoptimal_floor": floor,
                         "gap_closed": (circ - learned) / (circ - floor) if circ > floor else None},
        "slice_256x256x12": {"split_bregman": sb, "pcg_from_zero": pcg, "split_bregman_data_scale_1e3": sb_scaled,
                             "superoptimal_probe_ceiling": ceiling},
        "slice_256x256x12_harder": harder,
        "seconds_total": round(time.perf_counter() - t0, 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=384, help="slices reconstructed per step")
    ap.add_argument("--contexts", type=int, default=3,
                    help="independent contexts the batch is split into, each with its own stream and host thread")
    ap.add_argument("--scale", type=float, default=1.0, help="data scale (1e3 makes the shrinks active)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip training / evaluating the learned correction")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 512^2 x 32 slice, the ragged batch, the 2D-mask batch and the "
                         "parameter-set comparison")
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--mode", choices=["full", "apply", "apply2d", "apply_ragged", "pcg", "volume", "step"],
                    default="full",
                    help="apply: only the apply_A timing loop and a copy-kernel calibration (for counter runs); "
                         "apply2d: the same for the 2D-mask operator (256^2 x 12, batch of 32); "
                         "apply_ragged: the ragged 64-slice batch's operator, whole and per size group; "
                         "volume: the 3D section alone; "
                         "step: 1 + --steps reconstructions of one 128-slice context at the default launch shape "
                         "(whole-step counter runs); "
                         "pcg: iteration-locked PCG solves over 128 slices (for kernel traces)")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="oracle processes of the all-cores CPU baseline (capped by the host's CPU count)")
    a = ap.parse_args()
    if a.cpu_worker is not None:
        cpu_worker(a.cpu_worker)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    cpu_all = None
    if a.mode == "full" and not a.no_cpu_baseline:
        # the all-cores oracle baseline first, while this process has not
        # touched the GPU (its workers are child processes)
        procs = max(1, min(a.cpu_procs, os.cpu_count() or 1))
        log(f"bench: cpu baseline (oracle) on {procs} cores")
        cpu_all = cpu_baseline_all_cores(procs)

    import torch
    from paper_1710_01758_amd import binding as B

    B.lib()
    torch.cuda.set_device(0)
    if a.mode == "apply2d":
        spec2 = gen.SliceSpec(256, 256, 12, 4.0, 24, mask_kind="2d", wavelet="db4", levels=3)
        insts2 = [gen.make_instance(spec2, gen.eval_seed(6, i)) for i in range(32)]
        ctx2, _ = B.context_for(insts2)
        run_apply_mode(torch, ctx2, insts2)
        return
    if a.mode == "apply_ragged":
        run_apply_ragged(torch, B)
        return
    if a.mode == "volume":
        print(json.dumps(volume_section(torch, B)), flush=True)
        return
    spec = gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3, data_scale=a.scale)
    if a.mode == "step":
        run_step_mode(torch, B, spec, a.steps)
        return
    if a.mode in ("apply", "pcg"):
        insts = [gen.make_instance(spec, gen.eval_seed(2, i)) for i in range(ROOFLINE_BATCH)]
        ctx, _ = B.context_for(insts)
        if a.mode == "apply":
            run_apply_mode(torch, ctx, insts)
        else:
            run_pcg_mode(torch, ctx)
        return
    if a.contexts < 1 or a.batch % a.contexts:
        print(json.dumps({"error": "--batch must be a multiple of --contexts"}))
        sys.exit(2)
    insts = [gen.make_instance(spec, gen.eval_seed(2, i)) for i in range(a.batch)]
    # the batch as `contexts` independent contexts, each with its own stream
    # and host thread: their kernel chains interleave on the GPU (one's
    # VALU-bound operator beside another's memory-bound passes)
    per = a.batch // a.contexts
    runs = []
    for k in range(a.contexts):
        st = torch.cuda.Stream()
        c, kk = B.context_for(insts[k * per:(k + 1) * per], stream=st.cuda_stream)
        runs.append({"ctx": c, "ksp": kk, "x": torch.zeros(c.image_elems, dtype=torch.complex64, device="cuda"),
                     "stream": st})
    split = [r["ctx"].autotune() for r in runs][0]
    ctx, ksp, x = runs[0]["ctx"], runs[0]["ksp"], runs[0]["x"]
    torch.cuda.synchronize()
    pool = cf.ThreadPoolExecutor(max_workers=a.contexts)

    def recon(r, kind="circulant"):
        r["ctx"].build_preconditioner(kind)
        iters, _ = r["ctx"].split_bregman_recon(r["ksp"], r["x"], n_outer=20, n_inner=1, tol=1e-3, maxit=1000)
        return iters

    def steps_of(r, count):
        # one context's share of `count` steps, back to back on its thread;
        # returns the wall time of each reconstruction
        times = []
        for k in range(count):
            ts = time.perf_counter()
            r["iters"] = recon(r)
            times.append((time.perf_counter() - ts) * 1e3)
            if r is runs[0] and (k + 1) % 10 == 0:
                log(f"bench: step {k + 1}/{count} done")
        return times

    log(f"bench: warmup {a.warmup} steps, batch {a.batch} as {a.contexts} contexts")
    for f in [pool.submit(steps_of, r, a.warmup) for r in runs]:
        f.result()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    futs = [pool.submit(steps_of, r, a.steps) for r in runs]
    per_ctx_ms = [f.result() for f in futs]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = runs[0]["iters"]
    # the step's algorithmic bytes: every slice's reconstruction with its own
    # PCG iteration count (last timed step of each context)
    step_bytes = sum(reconstruction_bytes(spec, int(it)) for r in runs for it in r["iters"].sum(axis=0))
    step_ms = np.array(per_ctx_ms).ravel()
    value = a.batch * a.steps / dt
    ms_per_step = dt / a.steps * 1e3
    pool.shutdown()

    # host-to-device bandwidth from pinned memory: what a slice's inputs
    # (zero-filled k-space and coil maps, c64) would cost if they arrived from
    # the host instead of being resident (the timed steps above exclude it)
    h2d_bytes = 256 * 2**20
    hbuf = torch.empty(h2d_bytes, dtype=torch.uint8, pin_memory=True)
    dbuf = torch.empty(h2d_bytes, dtype=torch.uint8, device="cuda")
    dbuf.copy_(hbuf, non_blocking=True)
    torch.cuda.synchronize()
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record()
    for _ in range(5):
        dbuf.copy_(hbuf, non_blocking=True)
    h1.record()
    h1.synchronize()
    h2d_gbs = 5 * h2d_bytes / (h0.elapsed_time(h1) * 1e-3) / 1e9
    slice_in_bytes = 2 * 8 * spec.m * spec.n * spec.ncoils
    del hbuf, dbuf

    # the preconditioner build alone (Table 2 reports it separately), one context
    for _ in range(2):
        ctx.build_preconditioner("circulant")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(5):
        ctx.build_preconditioner("circulant")
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) / 5 * 1e3

    # single-slice latency (one reconstruction alone)
    ctx1, ksp1 = B.context_for(insts[:1])
    split1 = ctx1.autotune()
    x1 = torch.zeros(ctx1.image_elems, dtype=torch.complex64, device="cuda")
    for _ in range(2):
        ctx1.build_preconditioner("circulant")
        ctx1.split_bregman_recon(ksp1, x1, n_outer=20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n1 = 5
    for _ in range(n1):
        ctx1.build_preconditioner("circulant")
        ctx1.split_bregman_recon(ksp1, x1, n_outer=20)
    torch.cuda.synchronize()
    single = n1 / (time.perf_counter() - t1)

    # PCG iterations to 1e-3: none vs circulant (first slice, every solve)
    it_none = recon(runs[0], "none")
    it_circ = recon(runs[0], "circulant")

    # one context alone (the same 128 slices, no other context beside it)
    steps_of(runs[0], 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n1c = 5
    steps_of(runs[0], n1c)
    torch.cuda.synchronize()
    one_ctx = per * n1c / (time.perf_counter() - t1)

    # the same batch at data scale 1e3 (k-space x 1e3 on the device: the
    # instances of data_scale 1e3 up to rounding), where the shrinks act:
    # same contexts, threads and launch shape as the headline
    for r in runs:
        r["ksp"].mul_(1e3)
    pool2 = cf.ThreadPoolExecutor(max_workers=a.contexts)
    for f in [pool2.submit(steps_of, r, 1) for r in runs]:
        f.result()
    torch.cuda.synchronize()
    steps_1e3 = max(3, a.steps // 5)
    t1 = time.perf_counter()
    for f in [pool2.submit(steps_of, r, steps_1e3) for r in runs]:
        f.result()
    torch.cuda.synchronize()
    value_1e3 = a.batch * steps_1e3 / (time.perf_counter() - t1)
    it_1e3 = runs[0]["iters"]
    pool2.shutdown()
    for r in runs:
        r["ctx"].close()
    del runs

    # roofline of the dominant kernel (fused apply_A) over a batch of
    # ROOFLINE_BATCH slices (the committed counter summaries' launch)
    rinsts = insts[:ROOFLINE_BATCH]
    rctx, _ = B.context_for(rinsts)
    rsplit = rctx.autotune()
    rtile = rctx.tuning_tiles()
    xa = torch.randn(rctx.image_elems, dtype=torch.complex64, device="cuda")
    ya = torch.empty_like(xa)
    t_apply = time_apply_kernel(torch, rctx, xa, ya)
    bytes_apply = apply_bytes([i.spec for i in rinsts])
    achieved = bytes_apply / t_apply / 1e9
    # the same operator with gamma W^H W evaluated through the wavelet
    # analysis and synthesis (W is unitary, so the fused kernel's gamma x is
    # the same term)
    t_explicit = time_apply_kernel(torch, rctx, xa, ya, reps=20, terms=B.TERM_ALL | B.TERM_WAVELET_EXPLICIT)
    rctx.close()

    out = {
        "metric": "recons/s + PCG iters to 1e-3, 256^2 x 12 coils: circulant vs learned precond",
        "value": round(value, 3),
        "unit": "recons/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "dtype_note": "complex64 (FP32) vectors and transforms, FP64 inner products and PCG scalars",
        "data": "synthetic",
        "config": {"workload": f"split_bregman_recon 256x256, 12 coils, R=4 lines (24 centre), TV + db4 x3, "
                               f"mu=1e-3 lambda=gamma=4e-3, 20 outer iters, PCG tol 1e-3, circulant; "
                               f"batch of {a.batch} slices per step as {a.contexts} concurrent contexts of {per} "
                               f"(one stream and host thread each), data_scale {a.scale:g}",
                   "global_batch": a.batch, "contexts": a.contexts, "m": 256, "n": 256, "ncoils": 12,
                   "parallelism": "none (1 GPU)"},
        "step_ms_stats": {"median": round(float(np.median(step_ms)), 3), "p10": round(float(np.percentile(step_ms, 10)), 3),
                          "p90": round(float(np.percentile(step_ms, 90)), 3),
                          "source": "host wall clock of each context's reconstruction (the contexts run concurrently)"},
        "h2d": {"GB_per_s": round(h2d_gbs, 1), "input_bytes_per_slice": slice_in_bytes,
                "recons_per_s_if_inputs_come_from_host": round(h2d_gbs * 1e9 / slice_in_bytes, 1),
                "note": "pinned host to device, 256 MiB copies; inputs per slice = k-space + coil maps (c64)"},
        "build_preconditioner_ms_context": round(build_ms, 3),
        "build_preconditioner_slices": per,
        "single_slice_recons_per_s": round(single, 3),
        "one_context_recons_per_s": {"value": round(one_ctx, 2), "slices": per,
                                     "note": "one context of the batch alone (one stream, one host thread)"},
        "data_scale_1e3": {"recons_per_s": round(value_1e3, 2), "steps": steps_1e3,
                           "pcg_iters_total_20_solves_slice0": int(it_1e3[:, 0].sum()),
                           "pcg_iters_mean_per_solve": round(float(it_1e3.mean()), 3),
                           "note": "the headline batch and launch configuration with the k-space scaled by 1e3 "
                                   "(data_scale 1e3: the TV and wavelet shrinks act); the headline itself is the "
                                   "literal scale, where they do not"},
        "coil_split": {"batch": split[0], "single_slice": split1[0]},
        "pcg_iters": {
            "none": {"first_solve": int(it_none[0, 0]), "total_20_solves": int(it_none[:, 0].sum()),
                     "per_solve": it_none[:, 0].tolist()},
            "circulant": {"first_solve": int(it_circ[0, 0]), "total_20_solves": int(it_circ[:, 0].sum()),
                          "per_solve": it_circ[:, 0].tolist()},
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if (rsplit[0], rtile[0]) == (1, 16) else None,
                     "kernel": (f"k_col_apply<256, 0, 0, {rtile[0]}> (fused apply_A, {ROOFLINE_BATCH} slices "
                                f"per launch, {rtile[0]}-column tiles)" if rsplit[0] == 1
                                else f"k_col_apply<256, 0, 1> + <256, 0, 2> (apply_A, coil split {rsplit[0]})"),
                     "avg_us": round(t_apply * 1e6, 2), "bytes_per_launch": bytes_apply,
                     "valu": valu_roofline(t_apply) if (rsplit[0], rtile[0]) == (1, 16) else None},
        "step_roofline": {"bound": "hbm", "achieved": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "bytes_per_step": step_bytes,
                          "note": "whole step: algorithmic bytes of every slice's reconstruction (build, "
                                  "initialisation, set-ups, PCG iterations at their measured counts, shrinks) "
                                  "over the step's wall time"},
        "apply_A_explicit_wavelet": {"avg_us": round(t_explicit * 1e6, 2),
                                     "vs_fused": round(t_explicit / t_apply, 3),
                                     "note": f"{ROOFLINE_BATCH} slices; gamma W^H W through the 3-level db4 analysis "
                                             "and synthesis instead of gamma x"},
    }
    if not a.no_extra:
        log("bench: 512x512x32 slice")
        out["slice_512x512x32"] = workload_section(
            torch, B, [gen.make_instance(gen.SLICE_512, gen.eval_seed(3))],
            "512x512, 32 coils, variable-density lines R=6 (32 centre), TV + db4 x4")
        log("bench: 1024x1024x12 slice")
        out["slice_1024x1024x12"] = workload_section(
            torch, B, [gen.make_instance(gen.SliceSpec(1024, 1024, 12, 4.0, 64, wavelet="db4", levels=4),
                                         gen.eval_seed(7))],
            "1024x1024, 12 coils, random lines R=4 (64 centre), TV + db4 x4 (the paper's largest size)")
        log("bench: ragged batch of 64 slices")
        specs = gen.ragged_specs()
        out["ragged_batch_64"] = workload_section(
            torch, B, [gen.make_instance(sp, gen.eval_seed(4, i)) for i, sp in enumerate(specs)],
            "64 slices {128^2, 192^2, 256x224, 320^2}, 8-32 coils, R in {3,4,6}, TV + db4 x3")
    if not a.no_extra:
        log("bench: 2D random variable-density mask, batch of 32")
        out["mask2d_256x256x12"] = mask2d_section(torch, B)
        log("bench: 3D volume 128x256x256x8")
        out["volume_128x256x256x8"] = volume_section(torch, B)
        log("bench: coil compression 12 -> 6 virtual coils")
        out["coil_compression_256x256x12"] = coil_compression_section(torch, B)
        log("bench: parameter sets 1-3, none / Jacobi / circulant")
        out["param_sets_256x256x12"] = param_sets_section(torch, B)
    if not a.no_learned:
        out["learned"] = learned_section(torch, B, a.train_steps)
        # the metric's second half in one place: PCG iterations from 0 to 1e-3
        # on the 256^2 x 12 slice, per preconditioner
        pz = out["learned"]["slice_256x256x12"]["pcg_from_zero"]
        out["pcg_iters_to_1e-3_256x256x12"] = {k: v["iters_to_1e-3"] for k, v in pz.items()}
    if not a.no_cpu_baseline:
        log("bench: cpu baseline (oracle), one core")
        one = cpu_baseline(insts[0])
        out["cpu_baseline"] = {
            "value": cpu_all["value"], "unit": "recons/s", "cores": cpu_all["cores"], "kind": "oracle",
            "host": one["host"],
            "sample": (f"{cpu_all['count']} full reconstructions (20 outer iterations, circulant, build included) of "
                       f"one 256x256x12 slice by {cpu_all['cores']} concurrent single-threaded FP64 NumPy oracle "
                       f"processes over {cpu_all['seconds']} s (slices are independent)"),
            "single_core": {k: one[k] for k in ("value", "unit", "cores", "sample")},
            "parity": parity_against_oracle(torch, B, insts[0], one["result"]),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
