"""Host checks of the measurement tooling: short names for every kernel the
library defines, the HBM-traffic scaling by a plain copy's counters on a
synthetic counter file, the algorithmic flop and byte bookkeeping, and the
benchmark's refusal of more than one GPU."""
import csv
import io
import json
import os
import subprocess
import sys
from contextlib import redirect_stdout

from paper_2001_01570_amd import profsum as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_short_names_cover_the_library_kernels():
    cases = {
        'void cgks::k_faces2<0, 1, double, cgks::Tile<4, 32> >(cgks::Geom, cgks::Bufs)': 'xfaces1',
        'void cgks::k_faces2<1, 1, double, cgks::Tile<2, 64> >(cgks::Geom, cgks::Bufs)': 'yfaces1',
        'void cgks::k_faces2<0, 2, float, cgks::Tile<8, 16> >(cgks::Geom, cgks::Bufs)': 'xfaces2',
        'void cgks::k_faces2<1, 2, float, cgks::Tile<2, 64> >(cgks::Geom, cgks::Bufs)': 'yfaces2',
        'void cgks::k_update2<1, double>(cgks::Geom, cgks::Bufs)': 'update1',
        'void cgks::k_update2<2, float>(cgks::Geom, cgks::Bufs)': 'update2',
        'void cgks::k_faces1<1>(cgks::Geom, cgks::Bufs)': 'faces1',
        'void cgks::k_update1<2>(cgks::Geom, cgks::Bufs)': 'update2_1d',
        'cgks::k_steps1(cgks::Geom, cgks::Bufs, int, int)': 'steps_1d',
        'cgks::k_begin(cgks::Scalars*, double const*, int)': 'begin',
        'cgks::k_end(cgks::Scalars*)': 'end',
        'void cgks::k_scan<4>(cgks::Geom, cgks::Bufs)': 'scan',
        'void cgks::kb_faces<0, 1>(cgks::SlotDev const*, cgks::BatchTable const*)': 'b_xfaces1',
        'void cgks::kb_faces<1, 2>(cgks::SlotDev const*, cgks::BatchTable const*)': 'b_yfaces2',
        'void cgks::kb_update<2>(cgks::SlotDev const*, cgks::BatchTable const*)': 'b_update2',
        'cgks::kb_begin(cgks::SlotDev const*, cgks::BatchTable const*)': 'b_begin',
        'cgks::kb_end(cgks::SlotDev const*, cgks::BatchTable const*)': 'b_end',
        'cgks::k_to_storage32(double const*, double*, unsigned long)': 'to_fp32',
    }
    for full, short in cases.items():
        assert P.short_name(full) == short, full


def _counters(path, rows):
    with open(path, 'w', newline='') as f:
        w = csv.writer(f)
        w.writerow(['Dispatch_Id', 'Kernel_Name', 'Counter_Name', 'Counter_Value'])
        for k, (name, counter, value) in enumerate(rows):
            w.writerow([k, name, counter, value])


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    nx = ny = 64
    copy = '__amd_rocclr_copyBuffer'
    xf = 'void cgks::k_faces2<0, 1, double, cgks::Tile<4, 32> >(cgks::Geom, cgks::Bufs)'
    mib = 8
    # the copy of 8 MiB reads 0.5x and writes 1.0x the bytes it moves (in KiB per dispatch)
    fetch, write = tmp_path / 'f.csv', tmp_path / 'w.csv'
    _counters(fetch, [(copy, 'FETCH_SIZE', 0.5 * mib * 1024), (copy, 'FETCH_SIZE', 3.0),
                      (xf, 'FETCH_SIZE', 100.0), (xf, 'FETCH_SIZE', 300.0)])
    _counters(write, [(copy, 'WRITE_SIZE', 1.0 * mib * 1024), (xf, 'WRITE_SIZE', 50.0)])
    buf = io.StringIO()
    with redirect_stdout(buf):
        P.main(['traffic', str(fetch), str(write), '--copy-mib', str(mib), '--nx', str(nx), '--ny', str(ny),
                '--cmd-fetch', 'f', '--cmd-write', 'w'])
    out = json.loads(buf.getvalue())
    assert out['fetch_factor'] == 0.5 and out['write_factor'] == 1.0
    k = out['kernels']['xfaces1']
    assert k['fetch_bytes'] == 200.0 * 1024 / 0.5          # mean of the dispatches, scaled
    assert k['write_bytes'] == 50.0 * 1024
    alg = 8 * (8 * nx * ny + 16 * ny * (nx + 1))           # 8 input fields per cell, 16 results per face
    assert k['algorithmic_bytes'] == alg and abs(k['ratio_to_algorithmic'] - (k['bytes_per_launch'] / alg)) < 1e-15


def test_flop_bookkeeping_adds_up():
    f = json.load(open(os.path.join(ROOT, 'paper_2001_01570_amd', 'flops.json')))
    u = f['units']
    per_launch = {k: v['flops_per_unit'] for k, v in f['per_launch_units'].items()}
    assert per_launch['xfaces1'] == per_launch['yfaces1'] == u['face_segment_stage1']['flops']
    assert per_launch['xfaces2'] == per_launch['yfaces2'] == u['face_segment_stage2']['flops']
    # per cell and step: one x and one y face segment per stage, and both updates
    assert f['flops_per_cell_step'] == (2 * (u['face_segment_stage1']['flops'] + u['face_segment_stage2']['flops'])
                                       + u['cell_update_stage1']['flops'] + u['cell_update_stage2']['flops'])
    for v in u.values():
        assert v['flops'] == v['add'] + v['mul'] + v['div']


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and 'one GPU' in r.stderr and r.stdout == ''
