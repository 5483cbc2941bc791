"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method (no stencil, transfer or
smoother): it only draws random numbers and evaluates closed-form fields.
All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Grids are cell-centred with n cells per axis; arrays have shape (n, n) or
(n, n, n) with x the last (fastest) axis.  Cell i of an axis is centred at
(i + 1/2) h.
"""
import numpy as np


def cell_centres(n, length=1.0):
    h = length / n
    return (np.arange(n) + 0.5) * h, h


def _mesh(d, n, length=1.0):
    x, h = cell_centres(n, length)
    axes = np.meshgrid(*([x] * d), indexing="ij")  # axes[0] varies along array axis 0
    # array axis order is (z, y, x) / (y, x): the last axis is x
    return list(reversed(axes)), h


def manufactured_2d(n=128, seed=0, n_modes=8, amp=0.1):
    """Poisson source f = -Lap(u*) on the unit square, Dirichlet-0.

    u* = sin(pi x) sin(pi y) + amp * sum_m c_m sin(k_m pi x) sin(l_m pi y),
    (k_m, l_m) drawn without replacement from {1..8}^2 minus (1, 1),
    c_m ~ U[-1, 1].  f is the continuous negative Laplacian of u* sampled at
    the cell centres.  Returns dict(f, h, u_star, modes) where modes is a list
    of (coefficient of f, (kx, ky)) whose sum over sin(kx pi x) sin(ky pi y)
    gives f exactly.
    """
    rng = np.random.default_rng(seed)
    pairs = [(k, l) for k in range(1, 9) for l in range(1, 9) if (k, l) != (1, 1)]
    pick = rng.choice(len(pairs), size=n_modes, replace=False)
    c = rng.uniform(-1.0, 1.0, size=n_modes)
    (X, Y), h = _mesh(2, n)
    u = np.sin(np.pi * X) * np.sin(np.pi * Y)
    modes = [(2.0 * np.pi ** 2, (1, 1))]
    for m in range(n_modes):
        k, l = pairs[pick[m]]
        u = u + amp * c[m] * np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
        modes.append((amp * c[m] * np.pi ** 2 * (k * k + l * l), (k, l)))
    f = np.zeros_like(u)
    for coef, (k, l) in modes:
        f += coef * np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
    return dict(f=f, h=h, u_star=u, modes=modes)


def sine_rhs(d, n, seed=0, n_modes=8, kmax=8):
    """Smooth random source on the unit square/cube: f = sum_m c_m prod_a sin(k_ma pi x_a),
    k in {1..kmax}^d, c ~ U[-1, 1].  Returns dict(f, h, modes) with modes a list of
    (c_m, k_m tuple in (kx, ky[, kz]) order)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, kmax + 1, size=(n_modes, d))
    c = rng.uniform(-1.0, 1.0, size=n_modes)
    x, h = cell_centres(n)
    f = np.zeros((n,) * d)
    modes = []
    for m in range(n_modes):
        # separable product; array axis d-1-a carries coordinate a
        term = np.array(c[m])
        for a in reversed(range(d)):
            term = np.multiply.outer(term, np.sin(ks[m, a] * np.pi * x))
        f += term
        modes.append((float(c[m]), tuple(int(v) for v in ks[m])))
    return dict(f=f, h=h, modes=modes)


def _random_periodic_field(rng, d, n, kmax, power):
    """Real periodic field on the n^d grid of [0, 2pi)^d from integer wavevectors
    1 <= |k| <= kmax with amplitudes |k|^-power times a complex normal."""
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    K = np.meshgrid(*([k1] * d), indexing="ij")
    kk = np.sqrt(sum(k * k for k in K))
    mask = (kk >= 1.0) & (kk <= kmax)
    spec = np.zeros((n,) * d, dtype=np.complex128)
    cnt = int(mask.sum())
    z = rng.standard_normal(cnt) + 1j * rng.standard_normal(cnt)
    spec[mask] = z * kk[mask] ** (-power)
    return spec


def _to_real(spec, shift_axes, n):
    """Inverse DFT evaluated at positions shifted by half a cell along shift_axes
    (array axes), returning the real part."""
    d = spec.ndim
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    h = 2 * np.pi / n
    s = spec.copy()
    for ax in shift_axes:
        shape = [1] * d
        shape[ax] = n
        s = s * np.exp(1j * k1 * h / 2).reshape(shape)
    return np.real(np.fft.ifftn(s)) * n ** d


def divfree_velocity(d, n, seed=0, kmax=16):
    """Seeded divergence-free velocity on the periodic MAC grid of [0, 2pi)^d.

    2D: stream function psi at cell corners, spectrum |psi_k| ~ |k|^-3
    (kinetic energy spectrum ~ k^-3).  3D: vector potential on cell edges,
    |A_k| ~ |k|^-3.5.  Velocity is the discrete curl (exactly divergence-free
    under the face-difference divergence).  Scaled so that the largest
    component magnitude is 1.

    Layout: q[c] has shape (n,)*d; q[0][..., j, i] lives on the x-face between
    cells i and i+1, q[1] on the y-face between rows j and j+1, q[2] on the
    z-face.  Returns dict(q=[u, v(, w)], h, dt) with dt = 0.5 h / sum_c max|q_c|.
    """
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / n
    if d == 2:
        spec = _random_periodic_field(rng, 2, n, kmax, 3.0)
        psi = _to_real(spec, (0, 1), n)             # psi[j, i] at corner (i+1/2, j+1/2)
        u = (psi - np.roll(psi, 1, axis=0)) / h      # d psi / dy at x-face (i+1/2, j)
        v = -(psi - np.roll(psi, 1, axis=1)) / h     # -d psi / dx at y-face (i, j+1/2)
        q = [u, v]
    elif d == 3:
        # array axes: 0 = z, 1 = y, 2 = x
        Ax = _to_real(_random_periodic_field(rng, 3, n, kmax, 3.5), (0, 1), n)  # (i, j+1/2, k+1/2)
        Ay = _to_real(_random_periodic_field(rng, 3, n, kmax, 3.5), (0, 2), n)  # (i+1/2, j, k+1/2)
        Az = _to_real(_random_periodic_field(rng, 3, n, kmax, 3.5), (1, 2), n)  # (i+1/2, j+1/2, k)
        r = np.roll
        u = (Az - r(Az, 1, axis=1) - Ay + r(Ay, 1, axis=0)) / h
        v = (Ax - r(Ax, 1, axis=0) - Az + r(Az, 1, axis=2)) / h
        w = (Ay - r(Ay, 1, axis=2) - Ax + r(Ax, 1, axis=1)) / h
        q = [u, v, w]
    else:
        raise ValueError("d must be 2 or 3")
    s = max(float(np.abs(c).max()) for c in q)
    q = [np.ascontiguousarray(c / s) for c in q]
    dt = 0.5 * h / sum(float(np.abs(c).max()) for c in q)
    return dict(q=q, h=h, dt=dt)


def taylor_green_2d(n, t=0.0, nu=0.0):
    """Taylor-Green vortex on [0, 2pi)^2 sampled on the MAC grid:
    u = sin x cos y e^{-2 nu t} at x-faces, v = -cos x sin y e^{-2 nu t} at y-faces,
    p = (cos 2x + cos 2y)/4 e^{-4 nu t} at cell centres."""
    h = 2 * np.pi / n
    xc = (np.arange(n) + 0.5) * h
    xf = (np.arange(n) + 1.0) * h
    g = np.exp(-2 * nu * t)
    Yc, Xf = np.meshgrid(xc, xf, indexing="ij")
    u = np.sin(Xf) * np.cos(Yc) * g
    Yf, Xc = np.meshgrid(xf, xc, indexing="ij")
    v = -np.cos(Xc) * np.sin(Yf) * g
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    p = 0.25 * (np.cos(2 * X) + np.cos(2 * Y)) * g * g
    return dict(q=[u, v], p=p, h=h)


def gaussian_2d(n=301, gamma=40.0, spacing=1.0):
    """Gaussian exp(-(x^2 + y^2)/(2 gamma^2)) on n x n cells of width `spacing`
    whose centres are x = (i - (n-1)/2) * spacing (the middle cell sits at 0)."""
    x = (np.arange(n) - (n - 1) / 2.0) * spacing
    Y, X = np.meshgrid(x, x, indexing="ij")
    return np.exp(-(X ** 2 + Y ** 2) / (2 * gamma ** 2))


def gaussian_3d(n=64, gamma=10.0, spacing=1.0):
    """Gaussian exp(-(x^2 + y^2 + z^2)/(2 gamma^2)) on n^3 cells of width `spacing`,
    centres as gaussian_2d; array axes (z, y, x)."""
    x = (np.arange(n) - (n - 1) / 2.0) * spacing
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * gamma ** 2))


def explicit_ad_case(d, n):
    """Workload of the explicit advection-diffusion step: on n^d unit cells centred at
    the origin, a Gaussian of width n/10 offset by n/8 along x, advected by a solid-body
    rotation (2D: (-y, x) scaled to max speed 1) or by the divergence-free field
    (sin y cos z, sin z cos x, sin x cos y) on [-pi, pi)^3 (3D, max speed 1); nu = 0.5,
    dt = 0.1 (Courant number 0.1 as in the paper's explicit test).  Returns (T, a, h,
    dt, nu)."""
    h = 1.0
    x = (np.arange(n) - (n - 1) / 2.0) * h
    g = np.meshgrid(*([x] * d), indexing="ij")[::-1]  # [X, Y(, Z)], x fastest
    r2 = (g[0] - n / 8.0) ** 2 + sum(c ** 2 for c in g[1:])
    T = np.exp(-r2 / (2 * (n / 10.0) ** 2))
    if d == 2:
        R = (n - 1) / 2.0
        a = [-g[1] / R, g[0] / R]
    else:
        s = [c * (2 * np.pi / n) for c in g]
        a = [np.sin(s[1]) * np.cos(s[2]), np.sin(s[2]) * np.cos(s[0]), np.sin(s[0]) * np.cos(s[1])]
    return T, [np.ascontiguousarray(c) for c in a], h, 0.1, 0.5


def batched_sizes(count=512, seed=0, choices=(64, 128, 256, 512, 1024)):
    """Sizes of the batched workload: `count` draws, uniform over `choices`."""
    rng = np.random.default_rng(seed)
    return [int(choices[i]) for i in rng.integers(0, len(choices), size=count)]
