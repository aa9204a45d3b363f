"""Throughput of the beam-plasma PIC step on one MI355X.

Workload (the headline configuration): 2D3V periodic 1024 x 1024 grid,
dx = 0.2 c/w_p, dt = 0.1/w_p, 64 particles per cell per species (beam n_b =
0.1 n0 at gamma = 3 with u_th = 0.3 m c; return-current plasma 0.9 n0, u_th =
0.01 m c, scattering off the ions at nu = 0.05 w_p), 134,217,728 particles,
mixed precision.  The same workload in FP64 (the plain-method baseline) is
timed beside it.  A step is the whole hot path: gather, Boris push, move,
Esirkepov deposit, scattering, tile binning, FP64 current reduction, Yee
update, diagnostics every 10 steps.  Inputs are generated on the device
before the timed region.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: the library
runs one GPU per run and has no domain decomposition across GPUs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit), mixed-FP32 vs FP64, 2D 1024^2 64 ppc"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_0808_4078_amd/csrc/pic_kernels.hip", "paper_0808_4078_amd/csrc/pic_internal.hpp")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_particle_c3_hbm_traffic.txt")


def kernel_source_hash() -> str:
    """SHA-256 over the particle kernel's source files: a hardware-counter
    reading of the kernel is valid only for the source it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per particle-kernel launch from the committed counter
    summary, or None when the summary is absent or was taken on other
    kernel sources."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes: int = 1 << 30, reps: int = 5):
    """A plain device-to-device copy of known size, the calibration kernel
    for the FETCH_SIZE / WRITE_SIZE counters (each dispatch reads and writes
    nbytes)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "dispatches": reps,
                      "ms": ms, "GBs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


COPY_CHUNKS = (256, 1024, 4096, 32768)     # words per workgroup; 32768: a C3 tile's bin per species


def copy_ceiling(words: int = 1 << 27, reps: int = 5):
    """Copy ceilings of the device for the particle kernel's access pattern:
    pic_copy_probe over 1..8 arrays of `words` 4-byte words (one launch, one
    SoA stream per array, as the particle state), with each workgroup
    streaming chunks of 256 (one word per lane) to 32768 words (a C3 tile's
    bin per species), and torch's own copy of one array of the same total
    size for reference.  Bytes counted: read + written."""
    import torch
    from paper_0808_4078_amd import pic
    out = {"words_per_array": words, "reps": reps, "pic_copy_probe_GBs": {}}
    for na in (1, 2, 4, 6, 7, 8):
        src = [torch.full((words,), float(k + 1), dtype=torch.float32, device="cuda") for k in range(na)]
        dst = [torch.empty_like(t) for t in src]
        for chunk in COPY_CHUNKS if na == 7 else COPY_CHUNKS[:1]:
            pic.copy_probe(src, dst, chunk=chunk)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                pic.copy_probe(src, dst, chunk=chunk)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if not all(bool(torch.equal(a, b)) for a, b in zip(src, dst)):
                raise RuntimeError("copy probe: destination differs from source")
            gbs = 2 * 4 * words * na / (ms * 1e-3) / 1e9
            out["pic_copy_probe_GBs"][f"{na} arrays, chunk {chunk}"] = gbs
            progress(f"copy probe: {na} arrays of {words} words, chunks of {chunk}: {ms:.3f} ms, "
                     f"{gbs:.0f} GB/s read + write")
        del src, dst
        torch.cuda.empty_cache()
    a = torch.ones(7 * words, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["torch_copy_one_array_GBs"] = 2 * 4 * 7 * words / (ms * 1e-3) / 1e9
    progress(f"torch copy of one array of {7 * words} words: {out['torch_copy_one_array_GBs']:.0f} GB/s")
    print(json.dumps(out), flush=True)


def particle_kernel_bytes(wl, precision: str, tile: int) -> float:
    """Algorithmic HBM bytes of one particle-kernel launch.

    Every particle's state is read once and written once:
      mixed: 16-bit cell within the tile + one FP32 offset per resolved axis
             + 3 FP32 momenta (2D: 22 B, 3D: 26 B);
      FP64:  one FP64 position per resolved axis + 3 FP64 momenta (2D: 40 B);
    a collisional particle's state also holds its 4-byte id, which keys its
    scattering draw and therefore travels with it (read and written).
    Each tile stages E and B on (T+2)^D nodes and writes its partial current on
    (T+3)^D nodes."""
    r = 4 if precision == "mixed" else 8
    d = wl.ndim
    state = (2 + d * 4 + 3 * 4) if precision == "mixed" else (d * 8 + 3 * 8)
    total = 0.0
    for sc in wl.species:
        n = wl.cells * sc.ppc
        total += n * 2 * (state + (4 if sc.nu > 0 else 0))
    tiles = wl.cells // tile ** d
    total += tiles * (6 * (tile + 2) ** d * r + 3 * (tile + 3) ** d * r)
    return total


# Algorithmic bytes per particle-step of the headline workload's particle
# kernel as the byte model of the hot path counts them: 24 B of mixed state
# (int32 cell, two FP32 offsets, three FP32 momenta) read and written, 2 B of
# the collisional half's id, 1.1 B of per-tile field staging and current
# partials.  The kernel's own count of what its layout moves,
# particle_kernel_bytes() (a 16-bit in-tile cell; the id written back as
# well), is reported beside it.
MODEL_BYTES_PER_PARTICLE_STEP = 51.1

GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "oracle_c3_1024.txt")


def c3_error(log_every: int = 10):
    """C3 itself (1024^2, 64 ppc per species, 134 217 728 particles) over 800
    steps, in the launch configuration of the timed line (tile 16, the
    store reserve, graph replay), stepped on the GPU in mixed precision and
    in FP64 from the same host-loaded particles as the stored FP64-oracle
    series (tests/golden/oracle_c3_1024.txt, written by the oracle alone):
    the worst per-record relative error of the six field energies W_i and
    of the kinetic energies, and the growth rate of the transverse magnetic
    energy over the oracle's linear window (a least-squares fit of ln W),
    against the oracle's."""
    import numpy as np
    import synth
    from paper_0808_4078_amd import pic
    header = [ln for ln in open(GOLDEN_C3) if ln.startswith("# fit:")][0].split()
    a, b, rate_o = int(header[4]), int(header[5]), float(header[-1])
    o = np.loadtxt(GOLDEN_C3)
    t, Wo, Ko = o[:, 1], o[:, 2:8], o[:, 8:10]
    wl = synth.beam_plasma((1024, 1024), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=800,
                           name="c3-1024")
    parts = synth.load(wl)
    out = {"workload": "C3 (1024x1024, 64 ppc per species, 134217728 particles), 800 steps, records every "
                       "10 steps, same initial particles as the FP64 oracle series",
           "oracle_growth_rate": rate_o, "fit_window_t": [float(t[a]), float(t[b - 1])]}
    for name, prec in (("mixed", pic.PIC_PREC_MIXED), ("fp64", pic.PIC_PREC_FP64)):
        g, sp = pic.workload_descs(wl, precision=prec, tile=16, diag_every=log_every, reserve=RESERVE_2D,
                                   flags=pic.PIC_FLAG_HOST_LOAD | pic.PIC_FLAG_TRACK_IDS)
        run = pic.Run(g, sp)
        for s_, p_ in enumerate(parts):
            run.load_particles(s_, p_.x, p_.u, p_.id)
        run.step(wl.steps)
        h = run.history()
        run.close()
        W = np.array([x["W"] for x in h])
        K = np.array([x["kinetic"][:2] for x in h])
        Wb = W[a:b, 3] + W[a:b, 4]
        rate = 0.5 * float(np.polyfit(t[a:b], np.log(Wb), 1)[0])
        out[name] = {"W_rel_err_max": float(np.max(np.abs(W - Wo)[1:] / np.abs(Wo)[1:])),
                     "kinetic_rel_err_max": float(np.max(np.abs(K - Ko) / Ko)),
                     "growth_rate": rate, "growth_rate_rel_err": rate / rate_o - 1.0}
        progress(f"C3 1024^2 vs the oracle series, {name}: worst W_i error {out[name]['W_rel_err_max']:.2e}, "
                 f"growth rate {rate:.6f} vs oracle {rate_o:.6f}")
    return out


def host_cpu():
    """Host cores and CPU model (lscpu) of the machine the baseline runs on."""
    import subprocess
    model = None
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in txt.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "sched_affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Spare particle-store capacity per tile (fraction of the nominal load).
# Spare slots are never read, so they cost HBM capacity only; with the
# capacity of this GPU the single-run workloads take more than the library
# default, which makes store re-layouts (triggered when a filament outgrows
# its tile's spare room) rarer.  The ensemble keeps the default.
RESERVE_2D = 3.0      # C2/C3: 32 GB of particle store
RESERVE_3D = 2.9      # C4: ~145 GB; the largest below the library's 4 GiB cap per particle array
# Coulomb-model line: the momentum-transfer rate is nu at this speed (about
# the return current's drift speed in C3)
COULOMB_VREF = 0.1
# Binary-collision line: electron-electron rate at this relative speed
BINARY_NU, BINARY_VREF = 0.05, 0.1


def tune_shape(wl, tile: int, reserve: float, nsteps: int = 10):
    """pic_tune_shape on the workload itself (mixed precision, one run):
    the particle kernel's launch shape that steps it fastest."""
    from paper_0808_4078_amd import pic

    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=tile, reserve=reserve)
    t0 = time.time()
    fastest, ms = pic.tune_shape(g, sp, nsteps=nsteps)
    best = pic.pick_shape(ms)
    progress(f"{wl.name}: launch shape {best} {pic.SHAPES[best]} (threads, in flight) in {time.time() - t0:.1f} s; "
             + ", ".join(f"{k} {pic.SHAPES[k]}: {v:.3f}" for k, v in ms.items()) + " ms/step")
    return best, {"chosen": best, "fastest": fastest, "threads_per_workgroup": pic.SHAPES[best][0],
                  "particles_in_flight": pic.SHAPES[best][1], "nsteps": nsteps,
                  "rule": f"the fastest shape if it beats shape 0 by more than {pic.SHAPE_MARGIN:.0%}, else shape 0",
                  "ms_per_step": {f"{k}: {pic.SHAPES[k][0]}x{pic.SHAPES[k][1]}": v for k, v in ms.items()},
                  "gain_of_fastest_over_default": ms[0] / ms[fastest] - 1.0}


def run_gpu(wl, precision: str, steps: int, warmup: int, tile: int, diag_every: int, profile: bool = True,
            reserve: float = 0.0, shape: int = 0):
    """Two fresh runs of the same workload.  Timed run: `warmup` untimed
    steps, then exactly `steps` steps as enqueued by pic_step (one captured
    graph replay per step), bracketed by device synchronisations and HIP
    events on the run's stream.  Profiled run (if requested): the same steps
    launched kernel by kernel with start/stop events on every dispatch,
    which give the per-kernel-group times and the particle kernel's average
    duration."""
    import torch
    from paper_0808_4078_amd import pic

    prec = pic.PIC_PREC_MIXED if precision == "mixed" else pic.PIC_PREC_FP64
    g, sp = pic.workload_descs(wl, precision=prec, tile=tile, diag_every=diag_every, reserve=reserve, shape=shape)
    t0 = time.time()
    run = pic.Run(g, sp)
    run.sync()
    init_s = time.time() - t0
    progress(f"{wl.name} {precision}: initialised {wl.particles} particles in {init_s:.2f} s")
    run.step(warmup)
    run.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(run.stream)
    run.step(steps)
    e1.record(run.stream)
    torch.cuda.synchronize()
    run.sync()
    ms = e0.elapsed_time(e1)
    info = run.info()
    # every timed (and warm-up) step was one replay of the captured graph
    if not (info["graph"] == 1 and info["graph_launches"] == warmup + steps and info["direct_steps"] == 0):
        raise RuntimeError(f"{wl.name}: steps were not graph replays: {info}")
    if info["shape"] != shape:
        raise RuntimeError(f"{wl.name}: ran in launch shape {info['shape']}, asked for {shape}")
    diag = run.diagnostics() if diag_every else None
    device_bytes = run.device_bytes
    run.close()
    del run
    torch.cuda.empty_cache()
    groups, prof_ms = None, None
    if profile:
        run = pic.Run(g, sp)
        run.step(warmup)
        run.sync()
        torch.cuda.synchronize()
        p0 = torch.cuda.Event(enable_timing=True)
        p1 = torch.cuda.Event(enable_timing=True)
        p0.record(run.stream)
        groups = run.step_profiled(steps)
        p1.record(run.stream)
        torch.cuda.synchronize()
        prof_ms = p0.elapsed_time(p1)
        run.close()
        del run
        torch.cuda.empty_cache()
    n = int(wl.particles)
    msg = f"{wl.name} {precision}: {steps} steps {ms / steps:.3f} ms/step"
    if profile:
        msg += (f" ({prof_ms / steps:.3f} ms/step launched kernel by kernel with events; particle kernel "
                f"{groups['particle'] / steps:.3f} ms)")
    if diag:
        msg += f"; re-layouts {diag['rebins']}"
    progress(msg)
    return dict(particles=n, init_s=init_s, ms=ms, profiled_ms=prof_ms, groups_ms=groups, diag=diag,
                device_bytes=device_bytes, graph_replays=info["graph_launches"])


def run_c5(steps: int, warmup: int, diag_every: int, prof_steps: int = 5):
    """The ensemble: 256 independent 2D3V runs of uneven size and load, tile
    edges from the autotuner, stepped as one batch (one graph per step)."""
    import torch
    import synth
    from paper_0808_4078_amd import autotune, pic

    members = synth.c5_members()
    t0 = time.time()
    tiles, shapes, report = autotune.choose_launch(members, precision=pic.PIC_PREC_MIXED, nsteps=5, log=progress)
    tune_s = time.time() - t0
    t0 = time.time()
    runs = []
    for i, (wl, t, sh) in enumerate(zip(members, tiles, shapes)):
        g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=t, diag_every=diag_every, shape=sh)
        runs.append(pic.Run(g, sp))
    batch = pic.Batch(runs)
    init_s = time.time() - t0
    n = int(sum(wl.particles for wl in members))
    progress(f"C5: {len(runs)} runs, {n} particles, tiles {dict((e, tiles.count(e)) for e in (8, 16, 32))}, "
             f"tuned in {tune_s:.1f} s, initialised in {init_s:.1f} s")
    batch.step(warmup)
    batch.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    li = batch.launch_info()
    if not (li["graph"] == 1 and li["graph_launches"] == warmup + steps and li["direct_steps"] == 0):
        raise RuntimeError(f"C5: batch steps were not graph replays: {li}")
    groups = batch.step_profiled(prof_steps)
    batch.sync()
    info = batch.info()
    rebins = sum(r.diagnostics()["rebins"] for r in runs) if diag_every else None
    batch.close()
    for r in runs:
        r.close()
    del runs, batch
    torch.cuda.empty_cache()
    progress(f"C5: {steps} batch steps {ms / steps:.3f} ms/step, {n * steps / (ms * 1e-3):.3e} particle-steps/s")
    return {"workload": "C5: 256 independent 2D3V runs, side in {64,128,256,512}, beam u_th ~ U[0.05,0.5], "
                        "nu ~ U[0,0.1], ppc ~ U{16..64} per species, mixed precision, one batch (persistent "
                        "particle kernel over a (run, tile) queue, one graph replay per step)",
            "runs": len(members), "particles": n, "steps": steps,
            "value": n * steps / (ms * 1e-3), "unit": "particle-steps/s", "ms_per_step": ms / steps,
            "tiles": {str(e): tiles.count(e) for e in (8, 16, 32)},
            "shapes_per_edge": {e: {"shape": sh, "threads_per_workgroup": pic.SHAPES[sh][0],
                                    "particles_in_flight": pic.SHAPES[sh][1]}
                                for e, sh in report["_edges"].items()},
            "autotune": {k: {"tile": v["tile"], "ms": v.get("ms"), "shape": v["shape"], "shape_ms": v["shape_ms"],
                             "members": v["members"]}
                         for k, v in report.items() if not k.startswith("_")},
            "persistent_blocks": info["persistent_blocks"], "work_items": info["items"],
            "batch_shapes": info["shapes"],
            "graph_replays": li["graph_launches"],
            "step_breakdown_ms": {k: v / prof_steps for k, v in groups.items()},
            "relayouts_total": rebins, "tune_s": tune_s, "init_s": init_s}


HYB_SORT_EVERY = 10      # reduced model: particle sort interval (steps)


def hybrid_particle_bytes(wl) -> float:
    """Algorithmic HBM bytes of one launch of the reduced model's particle
    kernel: x, y, u_x, u_y, p_z read (5 x 8 B) and x, y, u_x, u_y written
    (4 x 8 B) per particle; per tile, a^n, a^(n-1) and psi read on its
    field window and the four deposit planes added on its deposit window
    (counted once per node: 3 + 4 planes of FP64)."""
    return wl.particles * 72.0 + wl.cells * 7 * 8.0


def run_hybrid(steps: int, warmup: int, diag_every: int, prof_steps: int = 20):
    """The reduced quasi-neutral model (Eqs. 1-7) at the paper's 2D hot-beam
    collisional parameters on a 1024^2 grid (H2): graph-replayed steps, then
    kernel-by-kernel steps with events on every launch for the breakdown and
    the particle kernel's average duration."""
    import torch
    import synth
    from paper_0808_4078_amd import pic

    wl = synth.H2
    t0 = time.time()
    x, u, uz = synth.hybrid_load(wl)
    n = x.shape[1]
    run = pic.HybridRun(pic.hyb_desc(wl, n, diag_every=diag_every, sort_every=HYB_SORT_EVERY),
                        x[0], x[1], u[0], u[1], uz)
    del x, u, uz
    run.sync()
    init_s = time.time() - t0
    progress(f"H2 reduced model: {n} beam particles, initialised in {init_s:.1f} s")
    run.step(warmup)
    run.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(run.stream)
    run.step(steps)
    e1.record(run.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    groups = run.step_profiled(prof_steps)
    hist = run.history(8)
    run.close()
    del run
    torch.cuda.empty_cache()
    pk = groups["particle"] / prof_steps
    nbytes = hybrid_particle_bytes(wl)
    progress(f"H2 reduced model: {steps} steps {ms / steps:.3f} ms/step, particle kernel {pk:.3f} ms")
    return {"workload": "H2: the reduced quasi-neutral model (kinetic beam, fluid return current with drag, "
                        "A_z from Eq. 2 by 10 FFT sweeps), 1024x1024 nodes, dx=0.125, dt=0.0625, 64 beam "
                        "particles per cell, v_b=0.9c, u_th=0.37, nu=0.15, FP64",
            "particles": n, "steps": steps, "value": n * steps / (ms * 1e-3), "unit": "particle-steps/s",
            "ms_per_step": ms / steps, "sort_every": HYB_SORT_EVERY, "iters": wl.iters,
            "step_breakdown_ms": {k: v / prof_steps for k, v in groups.items()},
            "particle_kernel": {"ms": pk, "algorithmic_bytes": nbytes,
                                "GBs": nbytes / (pk * 1e-3) / 1e9,
                                "frac_of_hbm_peak": nbytes / (pk * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "eq7_last": hist[-1]["eq7"] if hist else None, "init_s": init_s}


def cpu_baseline(wl, target_s: float = 10.0, max_steps: int = 40):
    """The FP64 oracle on a bounded sample of the workload: a 256 x 256 box
    with the same per-cell load and physics, timed for whole steps until
    about target_s seconds have passed.  The oracle is compiled here for this
    host (-O3 -march=native, OpenMP, no fast-math, no FMA contraction: the
    arithmetic is the same as the tests' build)."""
    import oracle
    import synth
    from dataclasses import replace

    flags = oracle.build_native()

    sample = replace(wl, n=(256, 256), name=wl.name + "-256^2-sample")
    parts = synth.load(sample)
    sp = [oracle.SpeciesState(sc.q, sc.m, sc.weight, sc.nu, p.x, p.u, p.id) for sc, p in zip(sample.species, parts)]
    run = oracle.OracleRun(sample.ndim, sample.n, sample.d, sample.dt, sp, sample.seed)
    progress(f"cpu baseline: {sample.particles} particles loaded, {oracle.num_threads()} threads")
    run.step(1)
    n = sample.particles
    steps = 0
    t0 = time.time()
    while steps < max_steps and (time.time() - t0) < target_s:
        run.step(1)
        steps += 1
    dt = time.time() - t0
    return dict(value=n * steps / dt, unit="particle-steps/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"2D3V 256x256 box of the same workload ({n} particles, 64 ppc/species, same "
                       f"physics), {steps} FP64 oracle steps in {dt:.1f} s",
                host=host_cpu(), build=" ".join(flags))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the 1 GiB copy that calibrates the HBM byte counters, then exit")
    ap.add_argument("--copy-ceiling", action="store_true",
                    help="measure the copy ceilings of the particle state's access pattern (pic_copy_probe) and exit")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--shape", type=int, default=-1,
                    help="particle-kernel launch shape 0..4 for the mixed runs (-1: chosen by pic_tune_shape)")
    ap.add_argument("--diag-every", type=int, default=10)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="256^2 grid instead of 1024^2 (for profiling)")
    ap.add_argument("--c4", type=int, default=500, metavar="K",
                    help="also time K steps of the 3D 256x256x512 8-ppc workload (mixed; 0 = skip)")
    ap.add_argument("--coulomb", type=int, default=300, metavar="K",
                    help="also time K steps of C3 with the plasma on the Coulomb scattering model (0 = skip)")
    ap.add_argument("--binary", type=int, default=50, metavar="K",
                    help="also time K steps of C3 with binary electron-electron collisions (mixed; 0 = skip)")
    ap.add_argument("--paper", type=int, default=500, metavar="K",
                    help="also time K steps of the paper's 2D case (d) at its own parameters (0: skip)")
    ap.add_argument("--hybrid", type=int, default=200, metavar="K",
                    help="also time K steps of the reduced quasi-neutral model on 1024^2 nodes (FP64; 0 = skip)")
    ap.add_argument("--no-c3-error", dest="c3_error", action="store_false",
                    help="skip the mixed/FP64 error report against the stored FP64-oracle series")
    ap.add_argument("--c5", type=int, default=300, metavar="K",
                    help="also time K batch steps of the 256-run 2D ensemble (mixed, autotuned tiles; 0 = skip)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} refused: the PIC library runs on a single GPU "
              "(domain decomposition across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
        return
    if a.copy_ceiling:
        copy_ceiling()
        return
    import synth
    from dataclasses import replace
    from paper_0808_4078_amd.pic import SHAPES

    wl = synth.C3
    if a.quick:
        wl = replace(wl, n=(256, 256), name="C3-quick-256^2")
    if a.shape >= 0:
        shape, shape_tuning = a.shape, None
    else:
        shape, shape_tuning = tune_shape(wl, a.tile, RESERVE_2D, nsteps=20)
    mixed = run_gpu(wl, "mixed", a.steps, a.warmup, a.tile, a.diag_every, reserve=RESERVE_2D, shape=shape)
    fp64 = None if a.skip_fp64 else run_gpu(replace(wl, name="C2"), "fp64", a.steps, a.warmup, a.tile,
                                            a.diag_every, reserve=RESERVE_2D)
    n = mixed["particles"]
    ms_step = mixed["ms"] / a.steps
    value = n / (ms_step * 1e-3)
    pk_ms = mixed["groups_ms"]["particle"] / a.steps
    pk_bytes = particle_kernel_bytes(wl, "mixed", a.tile)
    model_bytes = MODEL_BYTES_PER_PARTICLE_STEP * n
    achieved = model_bytes / (pk_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (device-generated seeded load)",
        "config": {
            "workload": f"{wl.name}: 2D3V periodic {wl.n[0]}x{wl.n[1]}, dx=0.2, dt=0.1, 64 ppc per species; "
                        "beam n_b=0.1 gamma=3 u_th=0.3 + return-current plasma 0.9 u_th=0.01 nu=0.05",
            "particles": n,
            "precision": "mixed: int32 cell + FP32 offset/momentum/push/tile current; FP64 grid current "
                         "reduction and diagnostics",
            "tile": a.tile,
            "particle_kernel_shape": {"shape": shape, "threads_per_workgroup": SHAPES[shape][0],
                                      "particles_in_flight": SHAPES[shape][1],
                                      "chosen_by": "pic_tune_shape" if shape_tuning else "--shape"},
            "store_reserve": RESERVE_2D,
            "diag_every": a.diag_every,
            "parallelism": "single GPU",
        },
        "particle_kernel": {"ms": pk_ms, "particle_steps_per_s": n / (pk_ms * 1e-3),
                            "algorithmic_bytes": model_bytes,
                            "bytes_per_particle_step": MODEL_BYTES_PER_PARTICLE_STEP,
                            "kernel_count_bytes": pk_bytes,
                            "kernel_count_GBs": pk_bytes / (pk_ms * 1e-3) / 1e9,
                            "kernel_count_frac": pk_bytes / (pk_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "launch_tuning": shape_tuning,
        "graph_replays": mixed["graph_replays"],
        "step_breakdown_ms": {k: v / a.steps for k, v in mixed["groups_ms"].items()},
        "relayouts": mixed["diag"]["rebins"],
        "kernel_by_kernel_ms_per_step": mixed["profiled_ms"] / a.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic() if not a.quick else None},
    }
    if fp64 is not None:
        f_ms = fp64["ms"] / a.steps
        f_pk = fp64["groups_ms"]["particle"] / a.steps
        f_bytes = particle_kernel_bytes(wl, "fp64", a.tile)
        rec["fp64"] = {"workload": "C2 (same workload, FP64 throughout)", "value": n / (f_ms * 1e-3),
                       "ms_per_step": f_ms, "particle_kernel_ms": f_pk,
                       "particle_kernel_GBs": f_bytes / (f_pk * 1e-3) / 1e9,
                       "step_breakdown_ms": {k: v / a.steps for k, v in fp64["groups_ms"].items()}}
        rec["mixed_over_fp64"] = rec["value"] / rec["fp64"]["value"]
    if a.c4 > 0:
        if a.shape >= 0:
            c4_shape, c4_tuning = a.shape, None
        else:
            c4_shape, c4_tuning = tune_shape(synth.C4, 8, RESERVE_3D, nsteps=6)
        c4 = run_gpu(synth.C4, "mixed", a.c4, min(a.warmup, 5), 8, a.diag_every, reserve=RESERVE_3D, shape=c4_shape)
        c4_pk = c4["groups_ms"]["particle"] / a.c4
        c4_bytes = particle_kernel_bytes(synth.C4, "mixed", 8)
        rec["c4"] = {"workload": "C4: 3D3V periodic 256x256x512, dx=0.2, dt=0.1, 8 ppc per species, beam "
                                 "gamma=3 u_th=0.1 + collisionless return-current plasma, mixed precision",
                     "particles": c4["particles"], "steps": a.c4,
                     "value": c4["particles"] / (c4["ms"] / a.c4 * 1e-3),
                     "ms_per_step": c4["ms"] / a.c4, "particle_kernel_ms": c4_pk,
                     "particle_kernel_GBs": c4_bytes / (c4_pk * 1e-3) / 1e9,
                     "particle_kernel_shape": {"shape": c4_shape, "threads_per_workgroup": SHAPES[c4_shape][0],
                                               "particles_in_flight": SHAPES[c4_shape][1]},
                     "launch_tuning": c4_tuning,
                     "step_breakdown_ms": {k: v / a.c4 for k, v in c4["groups_ms"].items()}}
    if a.coulomb > 0:
        sp0, sp1 = wl.species
        wc = replace(wl, name=f"{wl.name}-coulomb",
                     species=(sp0, replace(sp1, coll_model=1, coll_vref=COULOMB_VREF)))
        cm = run_gpu(wc, "mixed", a.coulomb, min(a.warmup, 5), a.tile, a.diag_every, reserve=RESERVE_2D,
                     shape=shape)
        cm_pk = cm["groups_ms"]["particle"] / a.coulomb
        rec["coulomb"] = {"workload": f"{wl.name} with the return-current plasma on the Coulomb small-angle "
                                      f"model (nu=0.05 at v={COULOMB_VREF}c, every plasma particle turned every "
                                      "step), mixed precision",
                          "particles": cm["particles"], "steps": a.coulomb,
                          "value": cm["particles"] / (cm["ms"] / a.coulomb * 1e-3),
                          "ms_per_step": cm["ms"] / a.coulomb, "particle_kernel_ms": cm_pk,
                          "particle_kernel_GBs": pk_bytes / (cm_pk * 1e-3) / 1e9,
                          "step_breakdown_ms": {k: v / a.coulomb for k, v in cm["groups_ms"].items()}}
    if a.binary > 0:
        wb = replace(wl, name=f"{wl.name}-binary", nu_ee=BINARY_NU, ee_vref=BINARY_VREF,
                     species=tuple(replace(sc, binary=True) for sc in wl.species))
        bm = run_gpu(wb, "mixed", a.binary, min(a.warmup, 5), a.tile, a.diag_every, reserve=RESERVE_2D,
                     shape=shape)
        rec["binary"] = {"workload": f"{wl.name} with binary electron-electron collisions among all particles "
                                     f"(beam-plasma and plasma-plasma pairs in every cell, nu_ee={BINARY_NU} at "
                                     f"relative speed {BINARY_VREF}c), mixed precision",
                         "particles": bm["particles"], "steps": a.binary,
                         "value": bm["particles"] / (bm["ms"] / a.binary * 1e-3),
                         "ms_per_step": bm["ms"] / a.binary,
                         "pairs_last_record": bm["diag"]["ee_pairs"] if bm["diag"] else None,
                         "step_breakdown_ms": {k: v / a.binary for k, v in bm["groups_ms"].items()}}
    if a.paper > 0:
        # the paper's collisional hot-beam case (d): 160^2 cells of 0.125 c/w_p, 64 ppc per species,
        # v_b = 0.9 c, u_th = 0.37, nu = 0.15, dt = 0.0625 (2011 steps to T = 20 plasma periods)
        import math
        u_b = 0.9 / math.sqrt(1.0 - 0.81)
        wp = synth.beam_plasma((160, 160), d=(0.125, 0.125), dt=0.0625, steps=a.paper, ppc=64, u_th_beam=0.37,
                               nu=0.15, u_beam=u_b, name="paper-d")
        from paper_0808_4078_amd import pic
        gt, st = pic.workload_descs(wp, precision=pic.PIC_PREC_MIXED)
        ptile, ptile_ms = pic.tune(gt, st, nsteps=10)
        pm = run_gpu(wp, "mixed", a.paper, min(a.warmup, 5), ptile, a.diag_every, shape=0)
        rec["paper_d"] = {"workload": "the paper's 2D case (d): 160x160 cells, dx=0.125, dt=0.0625, 64 ppc per "
                                      "species, v_b=0.9c, u_th=0.37, nu=0.15, mixed precision",
                          "tile": ptile, "tile_ms_per_step": {str(k): v for k, v in ptile_ms.items()},
                          "particles": pm["particles"], "steps": a.paper,
                          "value": pm["particles"] / (pm["ms"] / a.paper * 1e-3),
                          "ms_per_step": pm["ms"] / a.paper,
                          "steps_to_T20_s": pm["ms"] / a.paper * 2011 * 1e-3,
                          "step_breakdown_ms": {k: v / a.paper for k, v in pm["groups_ms"].items()}}
    if a.hybrid > 0:
        rec["hybrid"] = run_hybrid(a.hybrid, a.warmup, a.diag_every)
    if a.c5 > 0:
        rec["c5"] = run_c5(a.c5, min(a.warmup, 5), a.diag_every)
    if a.c3_error:
        rec["c3_error"] = c3_error()
    if not a.skip_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
