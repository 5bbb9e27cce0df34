"""Short text summaries of rocprofv3 output for the committed profiles.

    python -m paper_2001_01570_amd.profsum stats  KERNEL_STATS_CSV --cmd "..."
    python -m paper_2001_01570_amd.profsum fp64   COUNTER_CSV --nx N --ny N --cmd "..."
    python -m paper_2001_01570_amd.profsum counters COUNTER_CSV --cmd "..."
    python -m paper_2001_01570_amd.profsum traffic FETCH_CSV WRITE_CSV --copy-mib M --nx N --ny N
                                                   --cmd-fetch "..." --cmd-write "..."

`stats` and `fp64` print text; `traffic` prints JSON (bytes per launch of each
kernel: FETCH_SIZE and WRITE_SIZE, each divided by the ratio the same counter
shows for one plain device copy of M MiB, i.e. M MiB read and M MiB written).
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# kernel name patterns (template arguments after the leading ones, such as the
# storage type and the tile shape, do not change the short name)
SHORT = [
    (r'k_faces2<0, 1\b', 'xfaces1'), (r'k_faces2<1, 1\b', 'yfaces1'), (r'k_faces2<0, 2\b', 'xfaces2'),
    (r'k_faces2<1, 2\b', 'yfaces2'), (r'k_update2<1\b', 'update1'), (r'k_update2<2\b', 'update2'),
    (r'k_faces1<1\b', 'faces1'), (r'k_faces1<2\b', 'faces2'), (r'k_update1<1\b', 'update1_1d'),
    (r'k_update1<2\b', 'update2_1d'), (r'k_begin\b', 'begin'), (r'k_end\b', 'end'), (r'k_scan<4\b', 'scan'),
    (r'k_scan<3\b', 'scan_1d'), (r'kb_faces<0, 1\b', 'b_xfaces1'), (r'kb_faces<1, 1\b', 'b_yfaces1'),
    (r'kb_faces<0, 2\b', 'b_xfaces2'), (r'kb_faces<1, 2\b', 'b_yfaces2'), (r'kb_update<1\b', 'b_update1'),
    (r'kb_update<2\b', 'b_update2'), (r'kb_begin\b', 'b_begin'), (r'kb_end\b', 'b_end'),
    (r'k_to_storage32\b', 'to_fp32'), (r'k_from_storage32\b', 'from_fp32'), (r'k_steps1\b', 'steps_1d'),
]
COPY_KERNEL = '__amd_rocclr_copyBuffer'


def short_name(full: str) -> str:
    for pat, v in SHORT:
        if re.search(pat, full):
            return v
    return full.split('(')[0][:60]


def units(kernel: str, nx: int, ny: int) -> int:
    return {'xfaces1': ny * (nx + 1), 'xfaces2': ny * (nx + 1), 'yfaces1': (ny + 1) * nx,
            'yfaces2': (ny + 1) * nx, 'update1': nx * ny, 'update2': nx * ny}.get(kernel, 0)


def algorithmic_bytes(kernel: str, nx: int, ny: int) -> int:
    """Bytes a launch must move at least: face kernels read the 4 averages and
    the 4 normal gradients of every cell once and write 16 (stage 1) or 8
    (stage 2) values per face segment; the updates read their cell inputs and
    the face results of both directions once and write their outputs."""
    c = nx * ny
    if kernel in ('xfaces1', 'yfaces1'):
        return 8 * (8 * c + 16 * units(kernel, nx, ny))
    if kernel in ('xfaces2', 'yfaces2'):
        return 8 * (8 * c + 8 * units(kernel, nx, ny))
    if kernel == 'update1':   # averages (4), FX and FY stage 1 (16 each) in; W* (12) and P (12) out
        return 8 * (4 * c + 16 * (units('xfaces1', nx, ny) + units('yfaces1', nx, ny)) + 24 * c)
    if kernel == 'update2':   # P (12), FX and FY stage 2 (8 each) in; the new state (12) out
        return 8 * (12 * c + 8 * (units('xfaces2', nx, ny) + units('yfaces2', nx, ny)) + 12 * c)
    return 0


def read_counters(path):
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(path) as f:
        for r in csv.DictReader(f):
            per[r['Kernel_Name']][r['Counter_Name']].append(float(r['Counter_Value']))
    return per


def cmd_stats(a):
    rows = list(csv.DictReader(open(a.csv)))
    print('# rocprofv3 kernel trace statistics')
    print('# command: %s' % a.cmd)
    print('%-10s %7s %14s %12s %7s  %s' % ('kernel', 'calls', 'total_ns', 'avg_ns', 'pct', 'name'))
    for r in rows:
        print('%-10s %7s %14.0f %12.1f %7.2f  %s' % (short_name(r['Name']), r['Calls'], float(r['TotalDurationNs']),
                                                   float(r['AverageNs']), float(r['Percentage']), r['Name'][:70]))


def cmd_fp64(a):
    per = read_counters(a.csv)
    flops = json.load(open(os.path.join(ROOT, 'paper_2001_01570_amd', 'flops.json')))
    print('# rocprofv3 FP64 VALU counters per dispatch (mean over dispatches)')
    print('# command: %s' % a.cmd)
    print('# executed FP64 flops = 64 x SQ_INSTS_VALU_FLOPS_FP64 (ADD + MUL + TRANS + 2 FMA wave instructions,')
    print('# every lane counted); algorithmic flops from the operation counter (flops.json)')
    names = sorted(set(c for k in per.values() for c in k))
    print('%-10s ' % 'kernel' + ' '.join('%14s' % n.replace('SQ_INSTS_', '')[:14] for n in names)
          + ' %14s %14s %7s' % ('exec_flops', 'alg_flops', 'ratio'))
    for full, cs in per.items():
        k = short_name(full)
        if k == COPY_KERNEL or not k:
            continue
        mean = {n: sum(v) / len(v) for n, v in cs.items()}
        ex = 64 * mean.get('SQ_INSTS_VALU_FLOPS_FP64', 0.0)
        unit = flops['per_launch_units'].get(k)
        alg = unit['flops_per_unit'] * units(k, a.nx, a.ny) if unit else 0
        print('%-10s ' % k + ' '.join('%14.4g' % mean.get(n, float('nan')) for n in names)
              + ' %14.4g %14.4g %7.3f' % (ex, alg, ex / alg if alg else float('nan')))


def cmd_counters(a):
    per = read_counters(a.csv)
    print('# rocprofv3 counters per dispatch (mean over dispatches)')
    print('# command: %s' % a.cmd)
    names = sorted(set(c for k in per.values() for c in k))
    print('%-10s ' % 'kernel' + ' '.join('%16s' % n.replace('SQ_', '')[:16] for n in names))
    for full, cs in per.items():
        k = short_name(full)
        if k == COPY_KERNEL or not k:
            continue
        mean = {n: sum(v) / len(v) for n, v in cs.items()}
        print('%-10s ' % k + ' '.join('%16.4g' % mean.get(n, float('nan')) for n in names))


def cmd_traffic(a):
    fetch = read_counters(a.fetch)
    write = read_counters(a.write)
    copy_bytes = a.copy_mib * (1 << 20)

    def copy_factor(per, counter):
        # the calibration copy is the largest plain copy of the run
        vals = [v for k, c in per.items() if COPY_KERNEL in k for v in c.get(counter, [])]
        if not vals:
            raise SystemExit('no %s dispatch in the counter file' % COPY_KERNEL)
        return max(vals) * 1024.0 / copy_bytes

    ff = copy_factor(fetch, 'FETCH_SIZE')
    fw = copy_factor(write, 'WRITE_SIZE')
    sys.path.insert(0, ROOT)
    import bench
    out = {'nx': a.nx, 'ny': a.ny, 'source_digest': bench.source_digest(),
           'copy_mib': a.copy_mib, 'fetch_factor': ff, 'write_factor': fw,
           'commands': {'fetch': a.cmd_fetch, 'write': a.cmd_write}, 'kernels': {}}
    for full in fetch:
        k = short_name(full)
        if COPY_KERNEL in full or units(k, a.nx, a.ny) == 0:
            continue
        fk = fetch[full].get('FETCH_SIZE', [])
        wk = write.get(full, {}).get('WRITE_SIZE', [])
        if not fk or not wk:
            continue
        fb = sum(fk) / len(fk) * 1024.0 / ff
        wb = sum(wk) / len(wk) * 1024.0 / fw
        alg = algorithmic_bytes(k, a.nx, a.ny)
        out['kernels'][k] = {'fetch_kib_raw': sum(fk) / len(fk), 'write_kib_raw': sum(wk) / len(wk),
                             'fetch_bytes': fb, 'write_bytes': wb, 'bytes_per_launch': fb + wb,
                             'algorithmic_bytes': alg, 'ratio_to_algorithmic': (fb + wb) / alg if alg else None}
    print(json.dumps(out, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split('\n')[0])
    sub = ap.add_subparsers(dest='what', required=True)
    s = sub.add_parser('stats')
    s.add_argument('csv')
    s.add_argument('--cmd', required=True)
    s.set_defaults(fn=cmd_stats)
    s = sub.add_parser('fp64')
    s.add_argument('csv')
    s.add_argument('--cmd', required=True)
    s.add_argument('--nx', type=int, default=1024)
    s.add_argument('--ny', type=int, default=1024)
    s.set_defaults(fn=cmd_fp64)
    s = sub.add_parser('counters')
    s.add_argument('csv')
    s.add_argument('--cmd', required=True)
    s.set_defaults(fn=cmd_counters)
    s = sub.add_parser('traffic')
    s.add_argument('fetch')
    s.add_argument('write')
    s.add_argument('--copy-mib', type=int, required=True)
    s.add_argument('--nx', type=int, default=1024)
    s.add_argument('--ny', type=int, default=1024)
    s.add_argument('--cmd-fetch', required=True)
    s.add_argument('--cmd-write', required=True)
    s.set_defaults(fn=cmd_traffic)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == '__main__':
    main()
