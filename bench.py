#!/usr/bin/env python3
"""Throughput of the compact 8th-order GKS step on one MI355X.

Workload (default): 2D Euler, periodic 1024x1024 grid on [-1,1]^2, background
(rho,U,V,p) = (1,0,0,1/gamma) plus a Gaussian density and pressure pulse of
amplitude 1e-3 and half-width 0.05 at a centre drawn by default_rng(0); CFL
0.3; FP64.  One step = one two-stage fourth-order (MSMD) step of the whole
hot path.

Prints one JSON line: cell-updates/s (cells x steps / wall time, inputs
resident in HBM), the roofline entry of the dominant kernel (HIP events on the
solver's stream over the timed region) and the oracle's CPU rate on a bounded
sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

C3_CFL = 0.3
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


def cpu_baseline(prob, target_s=10.0, threads=None):
    """The oracle, as it stands, timed on this host: one MSMD step of a
    horizontal band of the same workload (full width, every parameter of the
    problem kept, free-flow rows beyond the band) with a margin of 4 rows
    (6 with four Gauss points: a step reads 2, resp. 3, cells per stage);
    rows are counted only in the band's exact core.  The band height is
    chosen from a 16-row probe so that the timed step takes about target_s
    seconds; if the whole grid takes less, consecutive steps of it are timed
    until about target_s.  threads: the host cores this process may use, at
    most 16 (one GPU's share of a host), or the given number."""
    import numpy as np
    from oracle import oracle as O
    from paper_2001_01570_amd import inputs as I
    if threads is None:
        threads = len(os.sched_getaffinity(0)) if hasattr(os, 'sched_getaffinity') else os.cpu_count()
        threads = max(1, min(threads, 16))
    margin = 6 if prob.gauss_points == 4 else 4

    def band_step(rows, steps=1):
        if rows == prob.ny:              # the whole grid
            p = prob
        else:
            j0 = prob.ny // 2 - rows // 2
            idx = np.arange(j0 - margin, j0 + rows + margin)
            if prob.bc[2] == I.PERIODIC:
                idx %= prob.ny
            else:
                idx = np.clip(idx, 0, prob.ny - 1)
            band = np.ascontiguousarray(prob.fields[:, idx, :])
            p = dataclasses.replace(prob, ny=len(idx), fields=band, y0=0.0, y1=prob.dy * len(idx),
                                    bc=(prob.bc[0], prob.bc[1], I.FREE, I.FREE))
        o = O.Oracle(p, threads=threads)
        dt = o.cfl_dt()
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step(dt)
        return time.perf_counter() - t0

    probe = band_step(16)
    rows_probe = 16 + 2 * margin
    rows = int(min(prob.ny, max(16, rows_probe * target_s / max(probe, 1e-6) - 2 * margin)))
    steps = 1
    if rows == prob.ny:
        steps = max(1, int(round(target_s / (probe * (prob.ny + 2 * margin) / rows_probe))))
    el = band_step(rows, steps)
    cells = prob.nx * rows * steps
    what = ('%d MSMD step%s of the whole %dx%d workload' % (steps, 's' if steps > 1 else '', prob.nx, prob.ny)
            if rows == prob.ny else
            '1 MSMD step of a %dx%d band (+%d-row margins) of the %dx%d workload'
            % (prob.nx, rows, margin, prob.nx, prob.ny))
    return dict(value=cells / el, unit='cell-updates/s', cores=threads, kind='oracle',
                sample='%s, %.1f s on %d thread%s' % (what, el, threads, 's' if threads > 1 else ''))


def launch_units(kernel, nx, ny):
    """Algorithmic units one launch processes: face segments or cells."""
    return {'xfaces1': ny * (nx + 1), 'xfaces2': ny * (nx + 1), 'yfaces1': (ny + 1) * nx,
            'yfaces2': (ny + 1) * nx, 'update1': nx * ny, 'update2': nx * ny}[kernel]


def source_digest():
    from paper_2001_01570_amd.build import source_digest as d
    return d()


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


def _make_request(k):
    from paper_2001_01570_amd import inputs as I
    p = I.serving_request(k)
    return k, p


def serving_requests(nreq):
    """The serving workload's requests (inputs.serving_request: side 64..512,
    pulse + vortex, 200 steps each), generated in worker processes.  Call it
    before anything touches the GPU (the workers are started by spawn)."""
    from multiprocessing import get_context
    log('[serving] generating %d requests' % nreq)
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, 'sched_getaffinity') else 4))
    with get_context('spawn').Pool(workers) as pool:
        reqs = dict(pool.map(_make_request, range(nreq)))
    return [reqs[k] for k in range(nreq)]


def serving(reqs, steps_per_run=None):
    """Serving workload over the requests reqs.  (1) the plain path closed
    loop (one context per request: create, load from host, 200 steps, read to
    host) gives the rate r; (2) Poisson arrivals at 2r (default_rng(7)) are
    replayed in real time through the plain path (FIFO, one request at a time)
    and through the batch API (admit on arrival, advance all running requests
    steps_per_run steps per graph replay -- by default the autotuner's
    figure -- read and release on completion).
    (3) The batch's own capacity c (every request admitted at once), and a
    second batch replay with the same draws at 0.7c, where the queue stays
    short and the latency is the steady-state one.
    Latency = completion - arrival.  Returns the figures as a dict."""
    import numpy as np
    nreq = len(reqs)
    steps = reqs[0].steps

    import torch
    from paper_2001_01570_amd.cgks import Batch, Solver, SLOT_DONE, SLOT_FAILED, CgksError, CGKS_EBUSY, batch_tuning
    torch.cuda.init()
    if steps_per_run is None:        # the autotuner's steps per graph replay
        steps_per_run = batch_tuning()[2]

    def plain_solve(p):
        s = Solver(p)
        s.run_steps(steps)
        out = s.get_state()[0]
        s.close()
        return out

    plain_solve(reqs[0])                      # warm up
    log('[serving] closed loop, plain path')
    t0 = time.perf_counter()
    for p in reqs:
        plain_solve(p)
    closed = nreq / (time.perf_counter() - t0)
    rate = 2.0 * closed
    arrivals = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, size=nreq))
    log('[serving] closed loop %.2f solves/s; arrivals at %.2f /s over %.2f s' % (closed, rate, arrivals[-1]))

    def wait_until(t_abs):
        while True:
            d = t_abs - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 1e-3))

    # plain path, open loop
    log('[serving] replay: plain path')
    lat_plain = np.zeros(nreq)
    t0 = time.perf_counter()
    for k, p in enumerate(reqs):
        wait_until(t0 + arrivals[k])
        plain_solve(p)
        lat_plain[k] = time.perf_counter() - t0 - arrivals[k]
    span_plain = time.perf_counter() - t0

    # batch path, open loop
    def batch_replay(arr):
        b = Batch(48 << 30, max_slots=min(nreq, 1024))
        lat = np.full(nreq, np.nan)
        slot_of = {}
        nxt = 0
        done = 0
        pending = []
        t0 = time.perf_counter()
        while done < nreq:
            now = time.perf_counter() - t0
            while nxt < nreq and arr[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            still = []
            for k in pending:
                try:
                    slot_of[b.admit(reqs[k], max_steps=steps)] = k
                except CgksError as e:
                    if e.code != CGKS_EBUSY:
                        raise
                    still.append(k)
            pending = still
            if not slot_of:
                if nxt < nreq:
                    wait_until(t0 + arr[nxt])
                continue
            b.run(steps_per_run)
            for s in list(slot_of):
                st = b.poll(s)[0]
                if st in (SLOT_DONE, SLOT_FAILED):
                    if st == SLOT_FAILED:
                        raise RuntimeError('request %d failed' % slot_of[s])
                    b.read(s)
                    b.release(s)
                    k = slot_of.pop(s)
                    lat[k] = time.perf_counter() - t0 - arr[k]
                    done += 1
        span = time.perf_counter() - t0
        b.close()
        return lat, span

    log('[serving] replay: batch path')
    lat_batch, span_batch = batch_replay(arrivals)
    log('[serving] batch capacity (all requests at once)')
    _, span_cap = batch_replay(np.zeros(nreq))
    capacity = nreq / span_cap
    rate_low = 0.7 * capacity
    arrivals_low = arrivals * (rate / rate_low)
    log('[serving] replay: batch path at %.2f /s (0.7 x capacity %.2f)' % (rate_low, capacity))
    lat_low, span_low = batch_replay(arrivals_low)

    def pct(a, q):
        return float(np.percentile(a, q))
    cells = sum(p.nx * p.ny for p in reqs)
    return {
        'metric': 'solves/s (serving, Poisson arrivals at 2x the plain closed-loop rate)',
        'value': nreq / span_batch,
        'unit': 'solves/s',
        'higher_is_better': True,
        'config': {'workload': '%d serving requests (sides 64-512, pulse + vortex, %d steps each, default_rng(1000+k)),'
                               ' arrivals default_rng(7)' % (nreq, steps), 'cells_total': cells,
                   'steps_per_run': steps_per_run},
        'batched': {'solves_per_s': nreq / span_batch, 'p50_s': pct(lat_batch, 50), 'p99_s': pct(lat_batch, 99),
                    'span_s': span_batch},
        'batched_capacity_solves_per_s': capacity,
        'batched_at_70pct_capacity': {'arrival_rate_per_s': rate_low, 'solves_per_s': nreq / span_low,
                                      'p50_s': pct(lat_low, 50), 'p99_s': pct(lat_low, 99), 'span_s': span_low},
        'plain': {'closed_loop_solves_per_s': closed, 'solves_per_s': nreq / span_plain,
                  'p50_s': pct(lat_plain, 50), 'p99_s': pct(lat_plain, 99), 'span_s': span_plain},
        'arrival_rate_per_s': rate,
        'batched_over_plain': (nreq / span_batch) / (nreq / span_plain),
    }


def fp32_storage(args):
    """The headline workload with the 8 gradient fields stored in FP32
    (averages, arithmetic, accumulation and tau/exp in FP64): throughput, and
    the max-norm difference from the FP64 path after the same steps relative
    to the pulse amplitude (gradients as differences across a cell, i.e.
    times the cell width).  The FP64 path matches the oracle to 1e-12."""
    import numpy as np
    import torch
    from paper_2001_01570_amd import inputs as I
    from paper_2001_01570_amd.cgks import Solver, CGKS_FP32_STORAGE

    amp = 1e-3
    prob = I.acoustic_pulse_2d(args.n, seed=0, amp=amp, cfl=C3_CFL)
    fields = torch.from_numpy(prob.fields).to('cuda')
    runs = {}
    for name, storage in (('fp32', CGKS_FP32_STORAGE), ('fp64', 0)):
        s = Solver(prob, load_state=False, storage=storage)
        s.set_state(fields, 0.0)
        s.run_steps(args.warmup)
        s.set_state(fields, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run_steps(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs[name] = (prob.nx * prob.ny * args.steps / el, s.get_state()[0])
        log('[fp32-storage] %s: %.4e cell-updates/s' % (name, runs[name][0]))
        s.close()
    d = np.abs(runs['fp32'][1] - runs['fp64'][1]).reshape(12, -1).max(axis=1) / amp
    d[4:] *= prob.dx
    out = {
        'metric': 'cell-updates/s per MSMD step (2D FP64 arithmetic, FP32 gradient storage)',
        'value': runs['fp32'][0], 'unit': 'cell-updates/s', 'n_gpus': 1, 'steps': args.steps,
        'warmup': args.warmup, 'higher_is_better': True, 'dtype': 'f64', 'storage': 'fp32 gradients',
        'data': 'synthetic',
        'config': {'workload': 'acoustic_pulse_2d periodic %dx%d on [-1,1]^2, amp 1e-3, half-width 0.05, CFL %g'
                               % (prob.nx, prob.ny, C3_CFL), 'cells': prob.nx * prob.ny, 'seed': 0},
        'fp64_value': runs['fp64'][0],
        'error_vs_fp64_rel_amplitude': {'averages': float(d[:4].max()), 'gradients_times_dx': float(d[4:].max()),
                                        'per_field': [float(x) for x in d]},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=500)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--n', type=int, default=1024, help='grid side (the workload is defined at 1024)')
    ap.add_argument('--workload', choices=('pulse', 'shock_vortex'), default='pulse',
                    help='pulse: the headline 1024^2 acoustic pulse; shock_vortex: the 2048x1024 Mach 1.1 '
                         'shock-vortex case (throughput of its first steps; the work per step does not depend on t)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--copy-calibration', type=int, default=0, metavar='MIB',
                    help='also run one plain device copy of this many MiB (reference for HBM byte counters)')
    ap.add_argument('--serving', type=int, default=256, metavar='R',
                    help='serving requests measured after the headline (Poisson arrivals, batched vs per-request), '
                         'reported in the same JSON line; 0: none')
    ap.add_argument('--serving-only', action='store_true',
                    help='only the serving workload (its own JSON line)')
    ap.add_argument('--gauss-points', type=int, choices=(2, 4), default=2,
                    help='Gauss points per face segment in 2D (4: the eighth-order 2D assembly with the 7-segment '
                         'sextic; the headline uses 2)')
    ap.add_argument('--recon-vars', choices=('conservative', 'characteristic'), default='conservative',
                    help='variables of the WENO-Z states (the headline: conservative); the flop count covers '
                         'the conservative kernels only, so the roofline is left out for characteristic')
    ap.add_argument('--side-slopes', action='store_true',
                    help='the evaluated variant whose non-equilibrium sides take the WENO-weighted slopes of their '
                         'candidates (two Gauss points); like characteristic variables, without the roofline')
    ap.add_argument('--tang-weno', action='store_true',
                    help='the evaluated variant whose WENO-Z states are assembled along the face by a tangential '
                         'WENO-Z of five segments (two Gauss points); without the roofline')
    ap.add_argument('--fp32-storage', action='store_true',
                    help='instead: the same workload with FP32 storage of the gradients, and its error vs FP64')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py measures one GPU: the solver runs on a single MI355X (use --gpus 1).', file=sys.stderr)
        sys.exit(2)
    reqs = serving_requests(args.serving) if args.serving and not args.fp32_storage else None
    if args.serving_only:
        out = serving(reqs)
        out.update({'n_gpus': 1, 'dtype': 'f64', 'data': 'synthetic'})
        print(json.dumps(out), flush=True)
        return
    if args.fp32_storage:
        fp32_storage(args)
        return

    import torch
    from paper_2001_01570_amd import inputs as I
    from paper_2001_01570_amd.cgks import Solver

    if args.workload == 'pulse':
        log('[bench] building workload %dx%d' % (args.n, args.n))
        prob = I.acoustic_pulse_2d(args.n, seed=0, cfl=C3_CFL)
        workload = ('acoustic_pulse_2d periodic %dx%d on [-1,1]^2, amp 1e-3, half-width 0.05, CFL %g'
                    % (prob.nx, prob.ny, C3_CFL))
    else:
        log('[bench] building workload shock_vortex 2048x1024')
        prob = I.shock_vortex_2d(2048, 1024)
        workload = ('shock_vortex_2d 2048x1024 on [0,2]x[0,1], Mach 1.1 normal shock + vortex Mv 0.3, '
                    'walls, inflow, free outflow, CFL %g' % prob.cfl)
    if args.gauss_points != 2:
        prob = dataclasses.replace(prob, gauss_points=args.gauss_points)
        workload += ', %d Gauss points per face segment' % args.gauss_points
    charv = args.recon_vars == 'characteristic'
    if charv:
        prob = dataclasses.replace(prob, recon_vars=1)
        workload += ', WENO-Z states in characteristic variables'
    if args.side_slopes:
        prob = dataclasses.replace(prob, side_slopes=1)
        workload += ', WENO-weighted side slopes'
    if args.tang_weno:
        prob = dataclasses.replace(prob, tang_weno=1)
        workload += ', tangential WENO-Z of the WENO-Z states'
    # the flop count covers the scheme as read with conservative variables:
    # no roofline for the options
    variant = charv or args.side_slopes or args.tang_weno
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

    # a short pass with every kernel kind bracketed by events names the
    # dominant kernel; the timed region brackets only that one (fewer events
    # in the stream, less perturbation of the throughput)
    s.set_profiling(True)
    s.run_steps(20)
    torch.cuda.synchronize()
    probe = s.kernel_times()
    s.set_profiling(False)
    dominant = max(probe.items(), key=lambda kv: kv[1][0])[0]
    log('[bench] probe kernel ms/step: %s; dominant %s'
        % ({k: round(v[0] / max(v[1], 1), 4) for k, v in probe.items()}, dominant))

    log('[bench] timing %d steps' % args.steps)
    s.set_profiling(True, kinds=[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_steps(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ktimes = s.kernel_times()
    s.set_profiling(False)
    cells = prob.nx * prob.ny
    value = cells * args.steps / el
    log('[bench] %.3f s, %.4e cell-updates/s; %s %.4f ms/launch' % (el, value, dominant,
                                                                    ktimes[dominant][0] / ktimes[dominant][1]))

    # roofline of the dominant kernel
    name = dominant
    ms, calls = ktimes[dominant]
    avg_s = ms / max(calls, 1) / 1e3
    flops = load_flops()
    roof = None
    units_key = 'per_launch_units' if args.gauss_points == 2 else 'per_launch_units_4pt'
    if flops is not None and name in flops.get(units_key, {}) and not variant:
        unit = flops[units_key][name]
        nunits = launch_units(name, prob.nx, prob.ny)
        alg = unit['flops_per_unit'] * nunits
        achieved = alg / avg_s / 1e12
        roof = {'bound': 'alu', 'kernel': name, 'achieved': achieved, 'peak': FP64_VECTOR_PEAK_TFLOPS,
                'unit': 'TFLOP/s', 'frac': achieved / FP64_VECTOR_PEAK_TFLOPS,
                # the committed counter summary covers the two-point kernels of the pulse
                'traffic': measured_traffic(name, prob.nx, prob.ny) if args.gauss_points == 2 else None,
                'avg_ms': avg_s * 1e3, 'flops_per_launch': alg}

    # the whole step: algorithmic flops per cell and step times the rate
    step = None
    if flops is not None and args.gauss_points == 2 and not variant:
        fc = flops['flops_per_cell_step']
        step = {'flops_per_cell_step': fc, 'tflops': fc * value / 1e12,
                'frac_of_fp64_peak': fc * value / 1e12 / FP64_VECTOR_PEAK_TFLOPS}

    s.close()
    serv = None
    if reqs:
        log('[bench] serving: %d requests' % len(reqs))
        serv = serving(reqs)
        log('[bench] serving: batched %.2f solves/s (p50 %.3f s, p99 %.3f s), plain %.2f solves/s'
            % (serv['batched']['solves_per_s'], serv['batched']['p50_s'], serv['batched']['p99_s'],
               serv['plain']['solves_per_s']))

    cpu = None
    if not args.no_cpu_baseline:
        log('[bench] oracle CPU baseline (all cores, then one thread)')
        cpu = cpu_baseline(prob)
        log('[bench] cpu', cpu)
        one = cpu_baseline(prob, threads=1)
        log('[bench] cpu 1 thread', one)
        cpu['single_thread'] = {'value': one['value'], 'cores': 1, 'sample': one['sample']}

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
        'config': {'workload': workload, 'cells': cells, 'seed': 0},
        'roofline': roof,
        'kernel_ms_per_launch_probe': {k: v[0] / max(v[1], 1) for k, v in probe.items()},
        'whole_step': step,
        'cpu_baseline': cpu,
        'serving': serv,
    }
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
