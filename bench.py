#!/usr/bin/env python3
"""Throughput of the compact 8th-order GKS step on one MI355X.

Workload (default): 2D Euler, periodic 1024x1024 grid on [-1,1]^2, background
(rho,U,V,p) = (1,0,0,1/gamma) plus a Gaussian density and pressure pulse of
amplitude 1e-3 and half-width 0.05 at a centre drawn by default_rng(0); CFL 0.3;
FP64.  One step = one two-stage fourth-order (MSMD) step of the whole hot path.

Prints one JSON line: cell-updates/s (cells x steps / wall time, inputs
resident in HBM), the roofline entry of the dominant kernel (HIP events on the
solver's stream over the timed region) and the oracle's CPU rate on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_flops():
    path = os.path.join(ROOT, 'paper_2001_01570_amd', 'flops.json')
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def cpu_baseline(prob, target_s=10.0):
    """The oracle, as it stands, timed on this host: one MSMD step of a
    horizontal band of the same workload (full width, periodic in x) with a
    4-row margin, rows counted only in the band's exact core.  The band height
    is chosen from a 16-row probe so that the timed step takes about target_s
    seconds (at most the whole grid).  Threads: the host cores this process may
    use, at most 16 (one GPU's share of a host)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2001_01570_amd import inputs as I
    threads = len(os.sched_getaffinity(0)) if hasattr(os, 'sched_getaffinity') else os.cpu_count()
    threads = max(1, min(threads, 16))

    def band_step(rows):
        j0 = prob.ny // 2 - rows // 2
        iy = np.arange(j0 - 4, j0 + rows + 4) % prob.ny
        band = np.ascontiguousarray(prob.fields[:, iy, :])
        p = I.Problem('band', 2, prob.nx, len(iy), prob.x0, prob.x1, 0.0, prob.dy * len(iy), band,
                      bc=(I.PERIODIC, I.PERIODIC, I.FREE, I.FREE), cfl=prob.cfl)
        o = O.Oracle(p, threads=threads)
        dt = o.cfl_dt()
        t0 = time.perf_counter()
        o.step(dt)
        return time.perf_counter() - t0

    probe = band_step(16)
    rows = int(min(prob.ny, max(16, 24 * target_s / max(probe, 1e-6) - 8)))   # the probe computes 24 rows
    el = band_step(rows)
    cells = prob.nx * rows
    return dict(value=cells / el, unit='cell-updates/s', cores=threads, kind='oracle',
                sample='1 MSMD step of a %dx%d band (+4-row margins) of the %dx%d workload, %.1f s on %d threads'
                       % (prob.nx, rows, prob.nx, prob.ny, el, threads))


def launch_units(kernel, nx, ny):
    """Algorithmic units one launch processes: face segments or cells."""
    return {'xfaces1': ny * (nx + 1), 'xfaces2': ny * (nx + 1), 'yfaces1': (ny + 1) * nx,
            'yfaces2': (ny + 1) * nx, 'update1': nx * ny, 'update2': nx * ny}[kernel]


def source_digest():
    """Digest of the HIP sources: counter-based figures are valid only for the
    kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for rel in ('paper_2001_01570_amd/csrc/cgks.hip', 'paper_2001_01570_amd/csrc/cgks_device.h'):
        with open(os.path.join(ROOT, rel), 'rb') as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, nx, ny):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy's counters), or None if the
    summary is missing, covers another workload or predates the sources."""
    path = os.path.join(ROOT, 'profiles', 'hbm_traffic_faces_1024sq.json')
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get('source_digest') != source_digest() or t.get('nx') != nx or t.get('ny') != ny:
        return None
    k = t.get('kernels', {}).get(kernel)
    return None if k is None else k['bytes_per_launch']


def main():
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=500)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--n', type=int, default=1024, help='grid side (the workload is defined at 1024)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--copy-calibration', type=int, default=0, metavar='MIB',
                    help='also run one plain device copy of this many MiB (reference for HBM byte counters)')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py measures one GPU: the solver runs on a single MI355X (use --gpus 1).', file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2001_01570_amd import inputs as I
    from paper_2001_01570_amd.cgks import Solver

    log('[bench] building workload %dx%d' % (args.n, args.n))
    prob = I.acoustic_pulse_2d(args.n, seed=0)
    fields = torch.from_numpy(prob.fields).to('cuda')
    torch.cuda.synchronize()
    s = Solver(prob, load_state=False)
    s.set_state(fields, 0.0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device='cuda')
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log('[bench] copy calibration: %d MiB read + %d MiB written' % (args.copy_calibration, args.copy_calibration))
        del src, dst
    log('[bench] warmup %d steps' % args.warmup)
    s.run_steps(args.warmup)
    torch.cuda.synchronize()

    log('[bench] timing %d steps' % args.steps)
    s.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_steps(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ktimes = s.kernel_times()
    s.set_profiling(False)
    cells = prob.nx * prob.ny
    value = cells * args.steps / el
    log('[bench] %.3f s, %.4e cell-updates/s; kernel ms: %s' % (el, value, {k: round(v[0], 2) for k, v in ktimes.items()}))

    # roofline of the dominant kernel
    dom = max(ktimes.items(), key=lambda kv: kv[1][0])
    name, (ms, calls) = dom
    avg_s = ms / max(calls, 1) / 1e3
    flops = load_flops()
    roof = None
    if flops is not None and name in flops.get('per_launch_units', {}):
        unit = flops['per_launch_units'][name]
        nunits = launch_units(name, prob.nx, prob.ny)
        alg = unit['flops_per_unit'] * nunits
        achieved = alg / avg_s / 1e12
        roof = {'bound': 'alu', 'kernel': name, 'achieved': achieved, 'peak': FP64_VECTOR_PEAK_TFLOPS,
                'unit': 'TFLOP/s', 'frac': achieved / FP64_VECTOR_PEAK_TFLOPS,
                'traffic': measured_traffic(name, prob.nx, prob.ny),
                'avg_ms': avg_s * 1e3, 'flops_per_launch': alg}

    cpu = None
    if not args.no_cpu_baseline:
        log('[bench] oracle CPU baseline')
        cpu = cpu_baseline(prob)
        log('[bench] cpu', cpu)

    out = {
        'metric': 'cell-updates/s per MSMD step (2D FP64)',
        'value': value,
        'unit': 'cell-updates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': el / args.steps * 1e3,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64',
        'data': 'synthetic',
        'config': {'workload': 'acoustic_pulse_2d periodic %dx%d on [-1,1]^2, amp 1e-3, half-width 0.05, CFL 0.3'
                               % (prob.nx, prob.ny), 'cells': cells, 'seed': 0},
        'roofline': roof,
        'kernel_ms_per_step': {k: v[0] / max(v[1], 1) for k, v in ktimes.items()},
        'cpu_baseline': cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
