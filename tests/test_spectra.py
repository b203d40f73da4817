"""Host helpers of the spectra tool against the paper's 1-D model (Sec. 3.5,
eq. model): advection-diffusion u_t = u_xx / Re - U u_x on a periodic line,
eigenvalues lambda_k = -k^2/Re - i k U. BEFE with the diffusion implicit and
the advection explicit gives B_T - I with eigenvalues
T lambda_k / (1 + T k^2 / Re), which Beaume's rescaling maps to lambda_k for
small T and to -1 - i U Re / k for large T."""
import numpy as np

from paper_1804_05087_amd import spectra


def _model_operator(n, L, re, U, T):
    """Dense B_T - I on n periodic grid points (Fourier differentiation)."""
    k = 2 * np.pi / L * np.fft.fftfreq(n, 1.0 / n)
    F = np.fft.fft(np.eye(n), axis=0)
    Finv = np.linalg.inv(F)
    ka = k.copy()
    ka[n // 2] = 0.0  # the real first derivative of the Nyquist mode vanishes
    D1 = (Finv @ np.diag(1j * ka) @ F).real
    D2 = (Finv @ np.diag(-k * k) @ F).real
    I = np.eye(n)
    B = np.linalg.solve(I - T * D2 / re, I - T * U * D1)
    return B - I, k, ka


def test_model_spectrum_and_beaume_limits():
    n, L, re, U = 32, 2 * np.pi, 500.0, 0.3
    for T in (1e-4, 0.1, 100.0, 1e6):
        A, k, ka = _model_operator(n, L, re, U, T)
        lam = spectra.eigenvalues(A)
        exact = T * (-k * k / re - 1j * ka * U) / (1 + T * k * k / re)
        for e in exact:
            assert np.min(np.abs(lam - e)) < 1e-10 * max(1.0, abs(e))
        scaled = spectra.beaume_scale(exact, T)
        model = -k * k / re - 1j * ka * U
        if T == 1e-4:
            assert np.allclose(scaled, model * (1 + T) / (1 + T * k * k / re))
            assert np.max(np.abs(scaled - model)) < 1e-3 * np.max(np.abs(model))
        if T == 1e6:   # T k^2 / Re >> 1 for every k != 0
            nz = ka != 0
            lim = -1 - 1j * U * re / k[nz]
            assert np.max(np.abs(scaled[nz] - lim) / np.abs(lim)) < 1e-3


def test_radius_and_band_statistics():
    rng = np.random.default_rng(0)
    r = rng.random(1000)
    th = rng.random(1000) * 2 * np.pi
    lam = -1 + r * np.exp(1j * th)
    rad = spectra.radius_containing(lam, 0.95)
    assert abs(rad - np.sort(r)[949]) < 1e-15
    assert np.mean(np.abs(lam + 1) <= rad) >= 0.95
    assert spectra.fraction_in_band(np.array([-1.1, -0.85, -1.3, 0.0]), 0.2) == 0.5
    s = spectra.summary(lam)
    assert s["n"] == 1000 and s["radius95_about_-1"] == rad


def test_admissible_restriction_removes_the_minus_one_block():
    """J = P A P - I with P an orthogonal projector of rank m: the restriction
    to range(P) has the eigenvalues of the m x m block, the rest is -1."""
    rng = np.random.default_rng(1)
    n, m = 40, 23
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Qm = Q[:, :m]
    A = rng.standard_normal((m, m))
    J = Qm @ A @ Qm.T - np.eye(n)
    Ja, Qa = spectra.admissible_restriction(J)
    assert Qa.shape == (n, m)
    ev = np.sort_complex(spectra.eigenvalues(Ja))
    ref = np.sort_complex(np.linalg.eigvals(A - np.eye(m)))
    assert np.allclose(ev, ref, atol=1e-10)
