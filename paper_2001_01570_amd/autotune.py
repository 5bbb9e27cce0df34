"""Autotuner of the face kernels' tile shape per direction and grid size.

    python -m paper_2001_01570_amd.autotune [--sizes 64,128,256,512,1024,2048] [--steps 20]

For each grid size it times every tile shape (HIP events around each face
launch, two stages, over a few steps of the acoustic-pulse workload) and
keeps the fastest shape per direction.  It writes tuning.json (the timings,
with the digest of the HIP sources they were measured on) and
csrc/tuning_table.h, the table the library compiles in: every 2D context
(and every step without allocation) takes the entry nearest in cell count.
Rebuild the library after tuning.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    ap.add_argument('--sizes', default='64,128,256,512,1024,2048')
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--out', default=TABLE)
    a = ap.parse_args(argv)
    from .build import source_digest
    entries = []
    for n in [int(x) for x in a.sizes.split(',')]:
        e = tune(n, a.steps)
        print('[autotune] %d^2: x %s, y %s  %s' % (n, SHAPES[e['x']], SHAPES[e['y']], e['ms_per_step']),
              file=sys.stderr, flush=True)
        entries.append(e)
    digest = source_digest()
    with open(a.out + '.tmp', 'w') as f:
        json.dump({'source_digest': digest, 'shapes': SHAPES, 'entries': entries}, f, indent=1)
    os.replace(a.out + '.tmp', a.out)
    write_header(entries, digest)


HEADER = os.path.join(PKG, 'csrc', 'tuning_table.h')


def write_header(entries, digest, path=HEADER):
    rows = '\n'.join('    {%d, %d, %d, %d},' % (e['nx'], e['ny'], e['x'], e['y']) for e in entries)
    text = ('// Face tile shapes per direction by grid size, written by the autotuner\n'
            '// (python -m paper_2001_01570_amd.autotune) from its timings on the GPU;\n'
            '// the library applies the entry nearest in cell count (log scale) when a 2D\n'
            '// context is created.  Shapes: 0 = 8x16, 1 = 4x32, 2 = 2x64.\n'
            '// Sources digest the timings were taken on: %s\n'
            '#pragma once\n'
            'namespace cgks {\n'
            'struct TuneEntry { int nx, ny, x, y; };\n'
            'constexpr TuneEntry kTuneTable[] = {\n%s\n};\n'
            '}  // namespace cgks\n' % (digest, rows))
    with open(path + '.tmp', 'w') as f:
        f.write(text)
    os.replace(path + '.tmp', path)


if __name__ == '__main__':
    main()
