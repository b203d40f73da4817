"""The compulsory bytes per launch that the benchmark divides by each kernel's
duration (its roofline position), rebuilt here from the shapes of the arrays
each kernel reads and writes at 48x65x48 (FP64): canonical fields are
complex128 [3][nx][nz/2+1][ny], y-valued spectral fields complex [ny][nz/2][nx],
x-physical fields complex [ny][3nx/2][nz/2]. The solve is charged the phase
traffic 9 S (S = one spectral field [nx][nz/2+1][ny] complex128): it reads the
three product fields and u and writes Phi; its mode records (6(N+1)+12
doubles per mode, rounded up to even, for every mode outside the Nyquist row
and column) and the Chebyshev weights are reported apart."""
import math

import numpy as np


def _nbytes(shape, itemsize):
    return int(np.prod(shape)) * itemsize


def test_algorithmic_bytes_48x65x48():
    import bench
    w = bench.WORKLOADS["couette_48x65x48_re1000_dt100"]
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    ab = bench.algorithmic_bytes(w)
    canon = _nbytes((3, nx, nz // 2 + 1, ny), 16)
    yv = _nbytes((ny, nz // 2, nx), 16)
    xp = _nbytes((ny, 3 * nx // 2, nz // 2), 16)
    record = 6 * ny + 12
    record += record % 2
    modes = nx * (nz // 2 + 1)
    assert ab["k_synth_y"] == _nbytes((3, nx, nz // 2, ny), 16) + 5 * yv
    assert ab["k_fft_x_inv"] == 5 * yv + 6 * xp
    assert ab["k_z_product"] == 9 * xp
    assert ab["k_fft_x_fwd"] == 3 * xp + 3 * yv
    S = _nbytes((nx, nz // 2 + 1, ny), 16)
    assert ab["k_stokes_solve"] == 9 * S
    assert 9 * S == 3 * canon
    nonnyq = (nx - 1) * (nz // 2)
    assert bench.solve_modes(w) == nonnyq == 1128
    assert bench.record_bytes(w) == nonnyq * record * 8 + 3 * ny * 8
    # the figures quoted with the benchmark's roofline line
    assert ab["k_stokes_solve"] == 11_232_000
    assert bench.record_bytes(w) == 3_629_208
    assert ab["k_synth_y"] == 9_584_640
    assert math.isclose(ab["k_fft_x_inv"] / 1e6, 16.77, abs_tol=0.005)
    # the z-line kernel that takes the inverse x transforms reads the five
    # y-valued fields and writes the three product fields; no x-inverse launch
    abf = bench.algorithmic_bytes(w, fused=True)
    assert "k_fft_x_inv" not in abf
    assert abf["k_z_product"] == 5 * yv + 3 * xp
    assert {k: v for k, v in abf.items() if k != "k_z_product"} == \
        {k: v for k, v in ab.items() if k not in ("k_z_product", "k_fft_x_inv")}


def test_mixed_path_halves_transform_bytes():
    import bench
    w = bench.WORKLOADS["couette_48x65x48_re1000_dt100"]
    ab64, ab32 = bench.algorithmic_bytes(w), bench.algorithmic_bytes(w, fp32=True)
    for k in ("k_fft_x_inv", "k_z_product", "k_fft_x_fwd"):
        assert 2 * ab32[k] == ab64[k]
