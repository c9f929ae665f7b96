"""Seeded synthetic initial states for the FAM workloads (shared by oracle and GPU tests).

This module holds no part of the scheme: it only turns an initial condition into
the evolved P1 moment state, i.e. the cell average and the scaled first moments

    u^(0) = (1/|I|) int_I u,   u^(1) = (1/|I|) int_I u (x - x_c)/dx,
    u^(2) = (1/|I|) int_I u (y - y_c)/dy                        (Sec. 2.1, 2.2)

computed either in closed form (piecewise-constant data) or with a 10-point
Gauss-Legendre rule per direction (smooth data; numpy's leggauss).

Arrays are numpy float64 with layout [component, moment, (ny,) nx], conservative
variables (rho, rho u, [rho v,] E) for the Euler equations.

Workloads (all synthetic; the paper uses no datasets):
* sine advection: u0 = sin x + cos(3x)/2 on [0, 2 pi] (linear advection, FAM3);
* Shu-Osher shock / density wave on [-5, 5] (Example 4.4, moved to 4000 cells);
* four-quadrant Riemann data on [0,1]^2, states drawn per quadrant from a seed;
* a batch of four-quadrant instances of uneven square sizes;
* a smooth periodic density-wave state for the adjoint;
* the smooth Euler and Burgers accuracy tests (Examples 4.1, 4.2).
"""
import math

import numpy as np

NQ = 10


def _gauss(n=NQ):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * x, 0.5 * w          # nodes on [-1/2, 1/2], weights sum to 1


# ----------------------------------------------------------------------------
# generic moment integration of smooth data
# ----------------------------------------------------------------------------
def moments_1d(func, x0, x1, n):
    """func(x) -> array [ncomp, ...]; returns [ncomp, 2, n]."""
    q, w = _gauss()
    dx = (x1 - x0) / n
    xc = x0 + (np.arange(n) + 0.5) * dx
    X = xc[None, :] + dx * q[:, None]                  # [Q, n]
    vals = np.asarray(func(X), dtype=np.float64)      # [C, Q, n]
    avg = np.einsum("q,cqn->cn", w, vals)
    mom = np.einsum("q,cqn->cn", w * q, vals)
    return np.stack([avg, mom], axis=1)


def moments_2d(func, x0, x1, y0, y1, nx, ny):
    """func(X, Y) -> array [ncomp, ...]; returns [ncomp, 3, ny, nx]."""
    q, w = _gauss()
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    acc0 = acc1 = acc2 = None
    for b in range(len(q)):
        Y = (yc + dy * q[b])[:, None, None]                  # [ny, 1, 1]
        X = (xc[None, :, None] + dx * q[None, None, :])      # [1, nx, Q]
        vals = np.asarray(func(np.broadcast_to(X, (ny, nx, len(q))),
                               np.broadcast_to(Y, (ny, nx, len(q)))), dtype=np.float64)
        s0 = np.einsum("a,cyxa->cyx", w, vals) * w[b]
        s1 = np.einsum("a,cyxa->cyx", w * q, vals) * w[b]
        s2 = s0 * q[b]
        if acc0 is None:
            acc0, acc1, acc2 = s0, s1, s2
        else:
            acc0, acc1, acc2 = acc0 + s0, acc1 + s1, acc2 + s2
    return np.stack([acc0, acc1, acc2], axis=1)


def euler_conservative(rho, u, p, v=None, gamma=1.4):
    """Primitive -> conservative (rho, rho u, [rho v,] E) for an ideal gas."""
    if v is None:
        return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def sine_advection(n, x0=0.0, x1=2.0 * math.pi):
    """u0 = sin x + cos(3x)/2, one component: [1, 2, n]."""
    return moments_1d(lambda x: (np.sin(x) + 0.5 * np.cos(3.0 * x))[None], x0, x1, n)


def fourier_mode_advection(n, omega, x0=0.0, x1=2.0 * math.pi, phase=0.0):
    """Real part of exp(i omega x + i phase) (closed form moments used by tests)."""
    return moments_1d(lambda x: np.cos(omega * x + phase)[None], x0, x1, n)


SHU_OSHER_LEFT = (3.857143, 2.629369, 10.33333)


def shu_osher(n, x0=-5.0, x1=5.0, gamma=1.4, split=-4.0):
    """Mach-3 shock meeting a density wave; left state for x < split."""
    dx = (x1 - x0) / n
    pos = (split - x0) / dx
    if abs(pos - round(pos)) > 1e-9:
        raise ValueError("the shock position must fall on a cell interface")
    rl, ul, pl = SHU_OSHER_LEFT

    def f(x):
        left = x < split
        rho = np.where(left, rl, 1.0 + 0.2 * np.sin(5.0 * x))
        u = np.where(left, ul, 0.0)
        p = np.where(left, pl, 1.0)
        return euler_conservative(rho, u, p, gamma=gamma)
    return moments_1d(f, x0, x1, n)


def draw_quadrants(seed):
    """Per-quadrant (rho, u, v, p) in the order NE, NW, SW, SE from numpy PCG64."""
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.02, 1.5)
        states.append((rho, u, v, p))
    return states


def _overlap_moments_1d(lo, hi, c, h):
    """For cell [c-h/2, c+h/2] and the interval [lo, hi]: (length fraction, first moment)."""
    a = np.clip(lo, c - h / 2, c + h / 2)
    b = np.clip(hi, c - h / 2, c + h / 2)
    frac = (b - a) / h
    mom = (((b - c) / h) ** 2 - ((a - c) / h) ** 2) / 2.0
    return frac, mom


def four_quadrant(n, seed, gamma=1.4, split=(0.5, 0.5), states=None, ny=None):
    """Four-quadrant piecewise-constant Euler data on [0,1]^2 (exact moments)."""
    nx = n
    ny = n if ny is None else ny
    if states is None:
        states = draw_quadrants(seed)
    dx, dy = 1.0 / nx, 1.0 / ny
    xc = (np.arange(nx) + 0.5) * dx
    yc = (np.arange(ny) + 0.5) * dy
    xs, ys = split
    U = np.zeros((4, 3, ny, nx))
    quads = {0: ((xs, 1.0), (ys, 1.0)), 1: ((0.0, xs), (ys, 1.0)),
             2: ((0.0, xs), (0.0, ys)), 3: ((xs, 1.0), (0.0, ys))}
    for qi, ((xl, xh), (yl, yh)) in quads.items():
        rho, u, v, p = states[qi]
        cons = euler_conservative(np.array(rho), np.array(u), np.array(p), np.array(v), gamma)
        fx, mx = _overlap_moments_1d(xl, xh, xc, dx)
        fy, my = _overlap_moments_1d(yl, yh, yc, dy)
        a0 = fy[:, None] * fx[None, :]
        a1 = fy[:, None] * mx[None, :]
        a2 = my[:, None] * fx[None, :]
        for c in range(4):
            U[c, 0] += cons[c] * a0
            U[c, 1] += cons[c] * a1
            U[c, 2] += cons[c] * a2
    return U


BATCH_SIZES = (64, 96, 128, 192, 256, 384, 512)


def batch_sizes(count=256, seed=1):
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(BATCH_SIZES, size=count)]


def batch_instance(i, n, gamma=1.4):
    """Instance i of the batched workload: four-quadrant data from seed 1000 + i."""
    return four_quadrant(n, 1000 + i, gamma)


def draw_density_waves(seed):
    """(a_m, k_m), m = 1..4: a_m ~ U[-1,1]/4, k_m integer vectors in [-3,3]^2 minus 0."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=4) / 4.0
    ks = []
    while len(ks) < 4:
        kv = rng.integers(-3, 4, size=2)
        if kv[0] != 0 or kv[1] != 0:
            ks.append((int(kv[0]), int(kv[1])))
    return a, ks


def _sincos_moments_1d(k, n):
    """Cell average and scaled first moment of sin(2 pi k x), cos(2 pi k x) on n cells of [0,1]."""
    q, w = _gauss()
    X = (np.arange(n) + 0.5)[:, None] / n + q[None, :] / n
    s, c = np.sin(2.0 * math.pi * k * X), np.cos(2.0 * math.pi * k * X)
    return s @ w, s @ (w * q), c @ w, c @ (w * q)


def density_waves(n, seed=2, gamma=1.4, ny=None):
    """rho = 1 + 0.2 sum_m a_m sin(2 pi k_m . x), u = v = 1/2, p = 1 on periodic [0,1]^2.

    Exact moments by the same Gauss rule as ``moments_2d``, evaluated in separable
    form: sin(a + b) = sin a cos b + cos a sin b, so each cell moment of a mode is a
    sum of products of 1D cell moments.  The state is linear in rho on this
    family: rho u = rho v = rho / 2 and E = p / (gamma - 1) + rho / 4.
    """
    a, ks = draw_density_waves(seed)
    ny = n if ny is None else ny
    r0 = np.ones((ny, n))
    r1 = np.zeros((ny, n))
    r2 = np.zeros((ny, n))
    for m in range(4):
        sx0, sx1, cx0, cx1 = _sincos_moments_1d(ks[m][0], n)
        sy0, sy1, cy0, cy1 = _sincos_moments_1d(ks[m][1], ny)
        amp = 0.2 * a[m]
        r0 = r0 + amp * (cy0[:, None] * sx0[None, :] + sy0[:, None] * cx0[None, :])
        r1 = r1 + amp * (cy0[:, None] * sx1[None, :] + sy0[:, None] * cx1[None, :])
        r2 = r2 + amp * (cy1[:, None] * sx0[None, :] + sy1[:, None] * cx0[None, :])
    rho = np.stack([r0, r1, r2])
    U = np.empty((4, 3, ny, n))
    U[0] = rho
    U[1] = 0.5 * rho
    U[2] = 0.5 * rho
    U[3] = 0.25 * rho
    U[3, 0] += 1.0 / (gamma - 1.0)
    return U


def smooth_euler_1d(n, gamma=1.4):
    """Example 4.2 (1D): (rho, u, p) = (1 + 0.2 sin(pi x), 1, 1) on [0, 2]."""
    return moments_1d(lambda x: euler_conservative(1.0 + 0.2 * np.sin(math.pi * x),
                                                   np.ones_like(x), np.ones_like(x), gamma=gamma),
                      0.0, 2.0, n)


def smooth_euler_1d_exact_density(n, t):
    """Exact density moments at time t (translation with unit speed)."""
    return moments_1d(lambda x: (1.0 + 0.2 * np.sin(math.pi * (x - t)))[None], 0.0, 2.0, n)


def smooth_euler_2d(n, gamma=1.4):
    """Example 4.2 (2D): (rho, u, v, p) = (1 + 0.2 sin(pi (x+y)), 1, 1, 1) on [0, 2]^2."""
    def f(X, Y):
        rho = 1.0 + 0.2 * np.sin(math.pi * (X + Y))
        one = np.ones_like(rho)
        return euler_conservative(rho, one, one, one, gamma)
    return moments_2d(f, 0.0, 2.0, 0.0, 2.0, n, n)


def smooth_euler_2d_exact_density(n, t):
    return moments_2d(lambda X, Y: (1.0 + 0.2 * np.sin(math.pi * (X + Y - 2.0 * t)))[None],
                      0.0, 2.0, 0.0, 2.0, n, n)


def burgers_smooth(n):
    """Example 4.1: u0 = 0.5 + sin(pi x) on [0, 2]."""
    return moments_1d(lambda x: (0.5 + np.sin(math.pi * x))[None], 0.0, 2.0, n)


def burgers_exact(x, t, iters=60):
    """Exact smooth Burgers solution via the characteristic relation u = u0(x - u t)."""
    u = 0.5 + np.sin(math.pi * x)
    for _ in range(iters):
        u = 0.5 + np.sin(math.pi * (x - u * t))
    return u


def burgers_exact_moments(n, t):
    return moments_1d(lambda x: burgers_exact(x, t)[None], 0.0, 2.0, n)


def random_state(shape, seed, lo=-1.0, hi=1.0):
    """Uniform random moments (for linear-operator tests)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def random_euler_state_2d(nx, ny, seed, amp=0.05):
    """A positive, mildly perturbed Euler moment state (for parity tests of the nonlinear path)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    u = 0.3 + amp * rng.uniform(-1, 1, (ny, nx))
    v = -0.2 + amp * rng.uniform(-1, 1, (ny, nx))
    p = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    U = np.zeros((4, 3, ny, nx))
    U[:, 0] = euler_conservative(rho, u, p, v)
    U[:, 1:] = amp * 0.1 * rng.uniform(-1, 1, (4, 2, ny, nx))
    return U


def density_wave_direction(n, rng, ny=None, gamma=1.4):
    """A random perturbation of the density-wave state that keeps u = v = 1/2 and p = 1.

    Perturbs the density moments by a random field and the momenta and energy
    consistently: d(rho u) = d(rho v) = d(rho)/2, dE = d(rho)/4 (E = p/(gamma-1) +
    rho |u|^2 / 2 with |u|^2 = 1/2).  Returns an array of the state's shape.
    """
    ny = n if ny is None else ny
    drho = rng.standard_normal((3, ny, n))
    d = np.zeros((4, 3, ny, n))
    d[0] = drho
    d[1] = 0.5 * drho
    d[2] = 0.5 * drho
    d[3] = 0.25 * drho
    return d


def smooth_density_wave_direction(n, rng, ny=None):
    """A random smooth perturbation of the density-wave state keeping u = v = 1/2, p = 1.

    d(rho) = sum_{m=1..4} b_m sin(2 pi k_m . x + phi_m) with b_m ~ N(0, 1),
    k_m integer vectors in [-3,3]^2 minus 0 and phi_m ~ U[0, 2 pi), as exact cell
    moments; d(rho u) = d(rho v) = d(rho)/2 and dE = d(rho)/4 as for
    ``density_wave_direction``.  Being smooth, it changes the interface jumps of
    the reconstruction only at the truncation-error level.
    """
    ny = n if ny is None else ny
    b = rng.standard_normal(4)
    ks = []
    while len(ks) < 4:
        kv = rng.integers(-3, 4, size=2)
        if kv[0] != 0 or kv[1] != 0:
            ks.append((int(kv[0]), int(kv[1])))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=4)

    def f(X, Y):
        drho = sum(b[m] * np.sin(2.0 * math.pi * (ks[m][0] * X + ks[m][1] * Y) + phi[m]) for m in range(4))
        return np.stack([drho, 0.5 * drho, 0.5 * drho, 0.25 * drho])
    return moments_2d(f, 0.0, 1.0, 0.0, 1.0, n, ny)


def double_mach(nx, ny, gamma=1.4, x1=3.0, y1=1.0):
    """Double Mach reflection initial data on [0, x1] x [0, y1] (Sec. 4 example): the state
    (rho, u, v, p) = (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5) behind the incident shock
    x = 1/6 + y / sqrt(3) (to its left) and (1.4, 0, 0, 1) ahead of it; moments by Gauss
    quadrature of the piecewise-constant data."""
    prim = ((8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5), (1.4, 0.0, 0.0, 1.0))
    cons = [euler_conservative(np.array(r), np.array(u), np.array(p), np.array(v), gamma) for r, u, v, p in prim]

    def f(X, Y):
        behind = X < 1.0 / 6.0 + Y / math.sqrt(3.0)
        return np.stack([np.where(behind, float(cons[0][c]), float(cons[1][c])) for c in range(4)])

    return moments_2d(f, 0.0, x1, 0.0, y1, nx, ny)
