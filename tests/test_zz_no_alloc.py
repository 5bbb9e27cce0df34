"""The step without allocation (cgks_step_noalloc) against the context's step
(cgks_step_dt) on the same input and step size, through the C ABI: two calls
in a row, the second on a smaller grid (the shared scratch keeps the first
call's contents), 2D and 1D, four Gauss points, the queued (no wait) form,
characteristic variables, and its error paths."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(prob, dt=0.0, wait=True):
    """(context result, no-alloc result, dt used by each)"""
    import torch
    from paper_2001_01570_amd.cgks import Solver, step_noalloc
    s = Solver(prob)
    dt_ctx = s.step(dt)
    ref = s.state
    s.close()
    fin = torch.from_numpy(np.ascontiguousarray(prob.fields)).to('cuda')
    fout = torch.full_like(fin, float('nan'))
    torch.cuda.synchronize()
    dt_na = step_noalloc(prob, fin, fout, dt=dt, wait=wait)
    torch.cuda.synchronize()
    return ref, fout.cpu().numpy(), dt_ctx, dt_na


def _check(prob, dt=0.0, wait=True):
    ref, got, dt_ctx, dt_na = _pair(prob, dt, wait)
    nf = ref.shape[0]
    worst = 0.0
    for f in range(nf):
        scale = max(np.abs(ref[f]).max(), 1e-300)
        worst = max(worst, np.abs(got[f] - ref[f]).max() / scale)
    say(prob.name, prob.nx, prob.ny, 'dt', dt_ctx, dt_na, 'worst field error', worst,
        'bitwise' if np.array_equal(got, ref) else '')
    assert worst <= 1e-12, worst
    if wait:
        assert dt_na == dt_ctx
    return worst


def test_two_calls_in_a_row_second_smaller():
    big = I.serving_request(3)                        # a pulse + vortex request
    if big.nx * big.ny > 65536:
        big = I.acoustic_pulse_2d(128, seed=5, amp=1e-2, half_width=0.1)
    _check(big)
    small = I.acoustic_pulse_2d(40, seed=0, amp=1e-2, half_width=0.25, ny=24)
    _check(small)


def test_walls_inflow_viscous_and_four_points():
    p = I.shock_vortex_2d(96, 48)
    _check(p)
    _check(dataclasses.replace(I.shock_vortex_2d(64, 32), mu=1e-3))
    _check(dataclasses.replace(I.diagonal_wave_2d(24), gauss_points=4))
    # WENO-Z states in characteristic variables (the kernel instances of their own)
    _check(dataclasses.replace(I.shock_vortex_2d(64, 32), recon_vars=1))
    _check(dataclasses.replace(I.shock_vortex_2d(48, 24), recon_vars=1, gauss_points=4))
    _check(dataclasses.replace(I.shock_tube_1d(100), recon_vars=1))
    # the side-slope variant (2D: kernel instances of their own; 1D)
    _check(dataclasses.replace(I.shock_vortex_2d(64, 32), side_slopes=1))
    _check(dataclasses.replace(I.shock_vortex_2d(48, 24), side_slopes=1, gauss_points=4))
    _check(dataclasses.replace(I.shock_tube_1d(100), side_slopes=1))
    # the tangential-WENO variant (the 5-segment halo)
    _check(dataclasses.replace(I.shock_vortex_2d(64, 32), tang_weno=1))


def test_one_dimensional_and_fixed_step():
    _check(I.sine_wave_1d(100))
    p = I.sine_wave_1d(400)
    _check(p, dt=1e-3)


def test_queued_form_without_wait():
    _check(I.acoustic_pulse_2d(64, seed=2, amp=1e-2, half_width=0.2), wait=False)


def test_largest_grid_and_rejections():
    import torch
    from paper_2001_01570_amd.cgks import CgksError, step_noalloc, CGKS_EINVAL, CGKS_ENONPHYS
    p = I.acoustic_pulse_2d(256, seed=1, amp=1e-3, half_width=0.1)    # 65536 cells: the maximum
    _check(p)
    q = I.acoustic_pulse_2d(257, seed=1)
    fin = torch.from_numpy(q.fields).to('cuda')
    fout = torch.empty_like(fin)
    with pytest.raises(CgksError) as e:
        step_noalloc(q, fin, fout)
    assert e.value.code == CGKS_EINVAL
    s = I.acoustic_pulse_2d(32, seed=1)
    fin = torch.from_numpy(s.fields).to('cuda')
    with pytest.raises(CgksError) as e:
        step_noalloc(s, fin, fin)                         # in place
    assert e.value.code == CGKS_EINVAL
    bad = s.fields.copy()
    bad[0, 3, 5] = -1.0                                   # negative density
    fin = torch.from_numpy(bad).to('cuda')
    fout = torch.empty_like(fin)
    with pytest.raises(CgksError) as e:
        step_noalloc(s, fin, fout)
    assert e.value.code == CGKS_ENONPHYS
    # the scratch is usable again after the rejected calls
    _check(I.acoustic_pulse_2d(48, seed=4, amp=1e-2, half_width=0.2))
