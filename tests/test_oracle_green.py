"""Pins of the oracle's Green's functions against closed forms and the paper's
stated identities (Sec. 1 Eqs. 1-2, Sec. 3 ansatz and its expansions, Eq. 9)."""
import numpy as np
import pytest

from oracle import green as g


def test_s1_closed_form_equals_ansatz_a1_minus_one_eighth():
    # Sec. 3: a_1 = -1/8 gives G_S1; Eq. 9 prints the same map in closed form
    rng = np.random.default_rng(0)
    x = rng.uniform(-2, 2, (1000, 3))
    np.testing.assert_allclose(g.green_s(x, (-0.125,)), g.green_s1(x), rtol=1e-14)


def test_xi_third_order_cancellation():
    # Sec. 3: 9/8 sin t - 1/8 sin(3t)/3 = t + O(t^5); the t^5 coefficient of
    # xi(t) = t - 3 pi^4 t^5 / 40 + ... follows from the sine series
    for t in [1e-2, 2e-2, 4e-2]:
        c5 = (g.xi(t) - t) / t ** 5
        assert abs(c5 / (-3 * np.pi ** 4 / 40) - 1) < 0.05 * (t / 1e-2) ** 2


def test_xi_fifth_order_variant():
    # Sec. 3: 75/64 sin t - 25/128 sin(3t)/3 + 3/128 sin(5t)/5 = t + O(t^7),
    # i.e. xi_2 with a_1 = -25/128, a_2 = 3/128
    a = (-25 / 128, 3 / 128)
    for t in [1e-2, 2e-2]:
        r = (g.xi(t, a) - t) / t ** 7
        assert np.isfinite(r) and abs(r) < 100.0
    assert abs(g.xi(0.05, a) - 0.05) < abs(g.xi(0.05) - 0.05) / 10


def test_xi_half_box_value_and_flat_derivative():
    # x_hat is differentiable at half the box (Sec. 3): xi'(1/2) = 0, xi(1/2) = 7/(6 pi)
    assert abs(g.xi(0.5) - 7 / (6 * np.pi)) < 1e-15
    eps = 1e-5
    d = (g.xi(0.5 + eps) - g.xi(0.5 - eps)) / (2 * eps)
    assert abs(d) < 1e-9
    # the wrap in G_S1 never acts: max |xi| < 1/2
    t = np.linspace(-1, 1, 20001)
    assert np.max(np.abs(g.xi(t))) < 0.5


def test_gx_periodic_and_newtonian_inside_half_box():
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.49, 0.49, (500, 3))
    r = np.linalg.norm(x, axis=1)
    np.testing.assert_allclose(g.green_x(x), -1 / (4 * np.pi * r), rtol=1e-14)
    for sh in ([1, 0, 0], [0, -1, 0], [3, 2, -5]):
        np.testing.assert_allclose(g.green_x(x + np.asarray(sh)), g.green_x(x), rtol=1e-12)


def test_gx_kink_at_half_box():
    # Eq. 2 remark: continuous but not differentiable at |x| = L/2
    y = np.array([0.1, 0.05])
    def f(t):
        return g.green_x(np.array([t, y[0], y[1]]))
    eps = 1e-6
    assert abs(f(0.5 - eps) - f(0.5 + eps)) < 1e-6
    left = (f(0.5 - eps) - f(0.5 - 2 * eps)) / eps
    right = (f(0.5 + 2 * eps) - f(0.5 + eps)) / eps
    assert left > 0 > right and abs(left + right) < 1e-3 * abs(left)


def test_gs1_smooth_at_half_box():
    def f(t):
        return g.green_s1(np.array([t, 0.1, 0.05]))
    eps = 1e-5
    left = (f(0.5) - f(0.5 - eps)) / eps
    right = (f(0.5 + eps) - f(0.5)) / eps
    assert abs(left) < 1e-3 and abs(right) < 1e-3


def test_self_cell_constant_by_quadrature():
    # c0 = integral over the unit cube of 1/|u|; midpoint rule, error ~ 3e-6
    n = 200
    u = (np.arange(n) + 0.5) / n - 0.5
    X, Y, Z = np.meshgrid(u, u, u, indexing="ij")
    q = np.mean(1 / np.sqrt(X ** 2 + Y ** 2 + Z ** 2))
    assert abs(q / g.self_cell_constant() - 1) < 1e-5


def test_gk_lattice_equals_explicit_fourier_sum():
    # Eq. 1: G_K(x) = sum over n_i in [-N/2+1, N/2], n != 0 of -exp(i k.x)/k^2
    N = 8
    gl = g.gk_lattice(N)
    n1 = np.arange(-N // 2 + 1, N // 2 + 1)
    for j in [(0, 0, 0), (1, 0, 0), (3, 2, 1), (4, 4, 4), (7, 5, 2)]:
        s = 0.0
        for a in n1:
            for b in n1:
                for c in n1:
                    if a == b == c == 0:
                        continue
                    k2 = (2 * np.pi) ** 2 * (a * a + b * b + c * c)
                    s += -np.cos(2 * np.pi * (a * j[0] + b * j[1] + c * j[2]) / N) / k2
        assert abs(gl[j] - s) < 1e-13 * max(1, abs(s))


def test_gk_series_matches_lattice_at_lattice_points():
    for N in (8, 16):
        c = np.arange(N) / N
        np.testing.assert_allclose(g.gk_series(N, c, c, c), g.gk_lattice(N), atol=1e-13)


def test_gk_zero_mean_and_newtonian_limit():
    N = 128
    gl = g.gk_lattice(N)
    assert abs(gl.sum()) < 1e-9 * np.abs(gl).sum()
    # away from the origin (r >> h), well inside the box, G_K ~ -1/(4 pi r) plus
    # the smooth part -r^2/6 + const (lap G_K = delta - 1 in the unit box).
    # Differences between radii r and 2r along a face diagonal isolate them
    # (along an axis the Nyquist cut-off leaves percent-level ripples).
    for j in (4, 6, 8):
        d = gl[j, j, 0] - gl[2 * j, 2 * j, 0]
        r = np.sqrt(2) * j / N
        expect = -1 / (4 * np.pi * r) + 1 / (4 * np.pi * 2 * r) + 0.5 * r ** 2
        assert abs(d / expect - 1) < 1e-3


def _fourier_interpolate_2x(lat):
    """Band-limited interpolation of an N^3 periodic lattice function onto
    the 2N^3 lattice of half-cell steps, by zero padding its discrete
    spectrum.  The Nyquist coefficient of each axis is split equally between
    +N/2 and -N/2 of the wider spectrum, so that the interpolant is real and
    even wherever the lattice function is.  Independent of gk_series: FFTs of
    the lattice values only."""
    N = lat.shape[0]
    A = np.fft.fftn(lat)
    for axis in range(3):
        shape = list(A.shape)
        shape[axis] = 2 * N
        B = np.zeros(shape, complex)
        lo = [slice(None)] * 3
        src = [slice(None)] * 3
        lo[axis], src[axis] = slice(0, N // 2), slice(0, N // 2)
        B[tuple(lo)] = A[tuple(src)]
        lo[axis], src[axis] = slice(2 * N - N // 2 + 1, 2 * N), slice(N // 2 + 1, N)
        B[tuple(lo)] = A[tuple(src)]
        nyq = [slice(None)] * 3
        nyq[axis] = slice(N // 2, N // 2 + 1)
        half = 0.5 * A[tuple(nyq)]
        lo[axis] = slice(N // 2, N // 2 + 1)
        B[tuple(lo)] = half
        lo[axis] = slice(2 * N - N // 2, 2 * N - N // 2 + 1)
        B[tuple(lo)] = half
        A = B
    out = np.fft.ifftn(A) * 8.0
    assert np.max(np.abs(out.imag)) < 1e-12 * np.max(np.abs(out.real))
    return out.real


def test_gk_series_off_mesh_equals_fourier_interpolation_of_the_lattice():
    # Off the mesh G_K is the real even trigonometric interpolant of the
    # lattice values of Eq. 1 (Nyquist term split between +-N/2).  An
    # independent route to it: zero-pad the lattice function's FFT onto a
    # twice finer lattice and transform back.  Every second point of the fine
    # lattice lies half a cell off the mesh along one, two or three axes.
    for N in (8, 16):
        fine = _fourier_interpolate_2x(g.gk_lattice(N))
        c = np.arange(2 * N) / (2.0 * N)
        ser = g.gk_series(N, c, c, c)
        np.testing.assert_allclose(ser, fine, rtol=0, atol=1e-13 * np.max(np.abs(fine)))
        # the even sub-lattice is the mesh itself
        np.testing.assert_allclose(ser[::2, ::2, ::2], g.gk_lattice(N), atol=1e-13)


def test_gk_series_off_mesh_equals_explicit_symmetric_fourier_sum():
    # Eq. 1 summed term by term at arbitrary points, with the Nyquist
    # frequencies n_i = +-N/2 both present at half weight; the imaginary part
    # cancels exactly (the coefficients are even in n).
    N = 8
    n1 = np.arange(-N // 2, N // 2 + 1)
    w1 = np.where(np.abs(n1) == N // 2, 0.5, 1.0)
    pts = [(0.1234, 0.4567, 0.7891), (0.5 / N, 0.0, 0.0), (0.37, 0.37, 0.5), (1.5 / N, 2.5 / N, 3.25 / N)]
    ser = {p: g.gk_series(N, [p[0]], [p[1]], [p[2]])[0, 0, 0] for p in pts}
    for x in pts:
        s = 0.0 + 0.0j
        for ia, a in enumerate(n1):
            for ib, b in enumerate(n1):
                for ic, c in enumerate(n1):
                    if a == b == c == 0:
                        continue
                    k2 = (2 * np.pi) ** 2 * (a * a + b * b + c * c)
                    s += w1[ia] * w1[ib] * w1[ic] * (-1.0 / k2) * np.exp(
                        2j * np.pi * (a * x[0] + b * x[1] + c * x[2]))
        assert abs(s.imag) < 1e-14
        assert abs(ser[x] - s.real) < 1e-13 * max(1.0, abs(s.real))


def test_gk_off_mesh_pin_rejects_the_one_sided_nyquist_sum():
    # The pin above discriminates: the paper's one-sided frequency set
    # n_i in [-N/2+1, N/2], evaluated off the mesh along every axis, has a
    # different real part (and an imaginary part), so an interpolant that
    # dropped the Nyquist split would fail it.
    N = 8
    n1 = np.arange(-N // 2 + 1, N // 2 + 1)
    for x in ((0.5 / N, 0.5 / N, 0.5 / N), (0.37, 0.21, 0.05)):
        s = 0.0 + 0.0j
        for a in n1:
            for b in n1:
                for c in n1:
                    if a == b == c == 0:
                        continue
                    k2 = (2 * np.pi) ** 2 * (a * a + b * b + c * c)
                    s += (-1.0 / k2) * np.exp(2j * np.pi * (a * x[0] + b * x[1] + c * x[2]))
        ser = g.gk_series(N, [x[0]], [x[1]], [x[2]])[0, 0, 0]
        assert abs(s.imag) > 1e-4 and abs(s.real - ser) > 1e-4
