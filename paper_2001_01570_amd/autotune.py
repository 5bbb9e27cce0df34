"""Autotuner of the face kernels' tile shape per direction and grid size, and
of the batch (serving) launches.

    python -m paper_2001_01570_amd.autotune [--sizes 64,128,256,512,1024,2048] [--steps 20]
                                            [--batch-requests 48]

For each grid size it times every tile shape (HIP events around each face
launch, two stages, over a few steps of the acoustic-pulse workload) and
keeps the fastest shape per direction.  For the batch it runs the first
requests of the serving workload (inputs.serving_request) admitted at once
through the serving loop (run, poll, read, release) and keeps the tile pair
of the two-point slots with the highest rate, then the number of steps per
graph replay (5, 10, 20 or 40) with the highest rate, a smaller one when
within 2 % (a shorter replay admits new requests sooner).  It writes
tuning.json (the timings, with the digest of the HIP sources they were
measured on) and csrc/tuning_table.h, the table the library compiles in:
every 2D context (and every step without allocation) takes the entry nearest
in cell count, every batch the batch entry.  Rebuild the library after
tuning.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, 'tuning.json')
SHAPES = {0: '8x16', 1: '4x32', 2: '2x64'}

def tune(n: int, steps: int = 20, rounds: int = 3):
    """Fastest shape per direction on an n x n grid: every shape is timed in
    each of `rounds` interleaved rounds (clock and cache warm-up affect all
    shapes alike) and keeps its best round."""
    import torch
    from . import inputs as I
    from .cgks import Solver
    p = I.acoustic_pulse_2d(n, seed=0, cfl=0.15)
    s = Solver(p)
    s.run_steps(10)
    ms = {k: {'x': float('inf'), 'y': float('inf')} for k in SHAPES}
    for _ in range(rounds):
        for shape in SHAPES:
            s.set_tiles(shape, shape)
            s.run_steps(2)
            s.set_profiling(True, kinds=['xfaces1', 'yfaces1', 'xfaces2', 'yfaces2'])
            s.run_steps(steps)
            torch.cuda.synchronize()
            t = s.kernel_times()
            s.set_profiling(False)
            ms[shape]['x'] = min(ms[shape]['x'], (t['xfaces1'][0] + t['xfaces2'][0]) / steps)
            ms[shape]['y'] = min(ms[shape]['y'], (t['yfaces1'][0] + t['yfaces2'][0]) / steps)
    best_x = min(ms, key=lambda k: ms[k]['x'])
    best_y = min(ms, key=lambda k: ms[k]['y'])
    s.close()
    return {'nx': n, 'ny': n, 'x': best_x, 'y': best_y,
            'ms_per_step': {SHAPES[k]: v for k, v in ms.items()}}


def _request(k):
    from . import inputs as I
    return I.serving_request(k)


def batch_requests(n):
    """The first n serving requests, generated in worker processes (call
    before anything touches the GPU: the workers are started by spawn)."""
    from multiprocessing import get_context
    with get_context('spawn').Pool(max(1, min(16, n))) as pool:
        return pool.map(_request, range(n))


def tune_batch(reqs, steps: int = 40, rounds: int = 2):
    """Tile pair of the two-point slots, then steps per replay, for the
    serving loop with every request admitted at once (cell-updates/s)."""
    import torch
    from .cgks import Batch, SLOT_DONE, SLOT_FAILED
    cells = sum(p.nx * p.ny for p in reqs)

    def rate(tiles, spr):
        b = Batch(48 << 30, max_slots=len(reqs))
        b.set_tiles(*tiles)
        live = {b.admit(p, max_steps=steps) for p in reqs}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while live:
            b.run(spr)
            for s in list(live):
                if b.poll(s)[0] in (SLOT_DONE, SLOT_FAILED):
                    b.read(s)
                    b.release(s)
                    live.discard(s)
        el = time.perf_counter() - t0
        b.close()
        return cells * steps / el

    rate((1, 2), 10)                         # warm-up
    pairs = [(x, y) for x in SHAPES for y in SHAPES]
    tile_rate = {pr: 0.0 for pr in pairs}
    for _ in range(rounds):
        for pr in pairs:
            tile_rate[pr] = max(tile_rate[pr], rate(pr, 10))
    best = max(pairs, key=lambda pr: tile_rate[pr])
    spr_rate = {}
    for _ in range(rounds):
        for spr in (5, 10, 20, 40):
            spr_rate[spr] = max(spr_rate.get(spr, 0.0), rate(best, spr))
    top = max(spr_rate.values())
    spr = min(k for k, v in spr_rate.items() if v >= 0.98 * top)
    return {'x': best[0], 'y': best[1], 'steps': spr, 'requests': len(reqs), 'steps_per_request': steps,
            'cell_updates_per_s_by_tiles': {'%s/%s' % (SHAPES[x], SHAPES[y]): v for (x, y), v in tile_rate.items()},
            'cell_updates_per_s_by_steps_per_run': spr_rate}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--sizes', default='64,128,256,512,1024,2048')
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--out', default=TABLE)
    ap.add_argument('--header', default=HEADER, help='where to write the C table (default: the library source)')
    ap.add_argument('--batch-requests', type=int, default=48)
    a = ap.parse_args(argv)
    from .build import source_digest
    reqs = batch_requests(a.batch_requests) if a.batch_requests > 0 else None
    entries = []
    for n in [int(x) for x in a.sizes.split(',')]:
        e = tune(n, a.steps)
        print('[autotune] %d^2: x %s, y %s  %s' % (n, SHAPES[e['x']], SHAPES[e['y']], e['ms_per_step']),
              file=sys.stderr, flush=True)
        entries.append(e)
    batch = {'x': 1, 'y': 2, 'steps': 10}
    if reqs:
        batch = tune_batch(reqs)
        print('[autotune] batch: x %s, y %s, %d steps per run  %s' % (SHAPES[batch['x']], SHAPES[batch['y']],
              batch['steps'], batch['cell_updates_per_s_by_steps_per_run']), file=sys.stderr, flush=True)
    digest = source_digest()
    with open(a.out + '.tmp', 'w') as f:
        json.dump({'source_digest': digest, 'shapes': SHAPES, 'entries': entries, 'batch': batch}, f, indent=1)
    os.replace(a.out + '.tmp', a.out)
    write_header(entries, digest, batch, a.header)


HEADER = os.path.join(PKG, 'csrc', 'tuning_table.h')


def write_header(entries, digest, batch, path=HEADER):
    rows = '\n'.join('    {%d, %d, %d, %d},' % (e['nx'], e['ny'], e['x'], e['y']) for e in entries)
    text = ('// Face tile shapes per direction by grid size, written by the autotuner\n'
            '// (python -m paper_2001_01570_amd.autotune) from its timings on the GPU;\n'
            '// the library applies the entry nearest in cell count (log scale) when a 2D\n'
            '// context is created.  Shapes: 0 = 8x16, 1 = 4x32, 2 = 2x64.\n'
            '// Sources digest the timings were taken on: %s\n'
            '#pragma once\n'
            'namespace cgks {\n'
            'struct TuneEntry { int nx, ny, x, y; };\n'
            '// Batch: face tile shapes of the two-point FP64 slots and the steps per graph\n'
            '// replay that gave the serving mix its highest rate.\n'
            'struct BatchTune { int x, y, steps; };\n'
            'constexpr BatchTune kBatchTune = {%d, %d, %d};\n'
            'constexpr TuneEntry kTuneTable[] = {\n%s\n};\n'
            '}  // namespace cgks\n' % (digest, batch['x'], batch['y'], batch['steps'], rows))
    with open(path + '.tmp', 'w') as f:
        f.write(text)
    os.replace(path + '.tmp', path)


if __name__ == '__main__':
    main()
