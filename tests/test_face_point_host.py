"""Host check of the phase-by-phase face-point evaluation of the 2D face
kernels: the device header compiled for the CPU, face_point (one Gauss point,
tangential quantities re-read per phase, mirrored line order for the second
point) against the direct composition tangential_point -> gks_point ->
face_accumulate (the second point with its own weights), for both face
directions, both stages, Euler and Navier-Stokes collision times and the
fallbacks; and the kernels' tangential weight tables against polynomials
(the three-segment quintic and quadratic at the 2- and 4-point nodes)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_face_point_matches_direct_composition(tmp_path):
    exe = str(tmp_path / 'face_point_check')
    subprocess.check_call(['g++', '-std=c++17', '-O1', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
                           '-I', os.path.join(ROOT, 'paper_2001_01570_amd', 'csrc'), '-I', os.path.join(ROOT, 'include'),
                           os.path.join(ROOT, 'tests', 'host', 'face_point_check.cpp'), '-o', exe],
                          stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True)
    lines = out.stdout.strip().splitlines()
    assert lines[-1] == 'fails 0', '\n'.join(l for l in lines if 'FAIL' in l or 'weights' in l)[:2000]
    assert out.returncode == 0
    assert lines[0].startswith('weights ') and float(lines[0].split()[1]) < 1e-13
    rows = [l.split() for l in lines[1:-1]]
    assert len(rows) == 2 * 40 * 8
    # fallbacks were exercised: right WENO state and equilibrium state
    assert any(r[7] == '1' for r in rows) and any(r[5] == '1' for r in rows)
