"""Pins of the FP64 oracle against what the mathematics fixes.

Each test ties one part of the oracle (Sec. 2, Eq. (1), forward Euler,
five-node Laplacian, stimulation) to something other than the oracle itself:
a closed form, a textbook special case, brute force on tiny inputs, an
invariant, or an independent integrator.  The cases are chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1901_06535_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P = dict(inputs.PARAMS_WORKLOAD)          # eps=0.022, D_u=1.0, rest of Table 1
P1 = dict(inputs.PARAMS_TABLE1)           # Table 1


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def _rest_state(params, phi):
    """Homogeneous rest state u* = v* of Eq. (1).

    With v = u and the Laplacian zero, du/dt = 0 reads
        (u - u^2)(u + q) = (f u + phi)(u - q)
    i.e.  u^3 + (f + q - 1) u^2 + (phi - q(1 + f)) u - phi q = 0,
    whose single positive root is the rest state (numpy.roots solves it)."""
    f, q = params["f"], params["q"]
    roots = np.roots([1.0, f + q - 1.0, phi - q * (1.0 + f), -phi * q])
    pos = [r.real for r in roots if abs(r.imag) < 1e-14 and r.real > 0]
    assert len(pos) == 1
    return pos[0]


# ---------------------------------------------------------------- Table 1

def test_table1_constants_match_paper():
    g = _read_golden("table1_params.txt")
    for k in ("eps", "f", "q", "D_u", "dt", "dx"):
        assert inputs.PARAMS_TABLE1[k] == g[k]
    assert inputs.PHI_ACTIVE_TABLE1 == g["phi_active"]
    assert inputs.PHI_PASSIVE_TABLE1 == g["phi_passive"]


# ---------------------------------------------------------------- P1 rest state

@pytest.mark.parametrize("params,phi", [(P, 0.04), (P, 0.054), (P, 0.08), (P1, 0.054),
                                        (P1, 0.0975)])
def test_rest_state_is_fixed(params, phi):
    us = _rest_state(params, phi)
    n = 12
    u = np.full((n, n), us)
    r = oracle.Run(u, u, np.full((n, n), phi), params)
    r.advance(1000)
    assert np.max(np.abs(r.u - us)) < 1e-12
    assert np.max(np.abs(r.v - us)) < 1e-12


def test_rest_state_moves_when_reaction_is_perturbed():
    """The fixed point above is not generic: shifting q by 1% moves it."""
    p = dict(P); p["q"] = P["q"] * 1.01
    us = _rest_state(P, 0.054)
    u = np.full((4, 4), us)
    r = oracle.Run(u, u, np.full((4, 4), 0.054), p)
    r.advance(50)
    assert np.max(np.abs(r.u - us)) > 1e-7


# ---------------------------------------------------------------- linearisation

@pytest.mark.parametrize("params,phi", [(P, 0.054), (P1, 0.0975), (P, 0.08)])
def test_linearisation_about_rest(params, phi):
    """A small homogeneous perturbation of the rest state obeys the Jacobian
    of the Euler map, derived by hand from Eq. (1):
        du'/du = 1 + (dt/eps) [1 - 2u - (f v + phi) 2q/(u+q)^2]
        du'/dv =   - (dt/eps) f (u - q)/(u + q)
        dv'/du = dt,   dv'/dv = 1 - dt."""
    eps, f, q, dt = params["eps"], params["f"], params["q"], params["dt"]
    us = _rest_state(params, phi)
    j_uu = 1 + dt / eps * (1 - 2 * us - (f * us + phi) * 2 * q / (us + q) ** 2)
    j_uv = -dt / eps * f * (us - q) / (us + q)
    h = 1e-7
    shape = (3, 5)
    phis = np.full(shape, phi)
    un, vn = oracle.step(np.full(shape, us + h), np.full(shape, us), phis, params)
    assert abs((un[0, 0] - us) / h - j_uu) < 1e-4 * max(1.0, abs(j_uu))
    assert abs((vn[0, 0] - us) / h - dt) < 1e-6
    un, vn = oracle.step(np.full(shape, us), np.full(shape, us + h), phis, params)
    assert abs((un[0, 0] - us) / h - j_uv) < 1e-4 * max(1.0, abs(j_uv))
    assert abs((vn[0, 0] - us) / h - (1 - dt)) < 1e-6


def test_euler_factor_matches_finite_difference_of_step():
    """The oracle's stability factor equals the numerical derivative of its own
    step map with diffusion off (two independent code paths)."""
    p = dict(P); p["D_u"] = 0.0
    rng = np.random.default_rng(3)
    for _ in range(20):
        u, v, phi = rng.uniform(0, 1), rng.uniform(0, 0.3), rng.uniform(0.04, 0.2)
        h = 1e-6 * max(u, 1e-3)
        up, _ = oracle.step(np.full((1, 1), u + h), np.full((1, 1), v), np.full((1, 1), phi), p)
        um, _ = oracle.step(np.full((1, 1), u - h), np.full((1, 1), v), np.full((1, 1), phi), p)
        fd = (up[0, 0] - um[0, 0]) / (2 * h)
        assert abs(fd - oracle.euler_factor(p, u, v, phi)) < 1e-5 * max(1, abs(fd))


# ---------------------------------------------------------------- Euler convergence

def test_forward_euler_converges_at_first_order_to_eq1():
    """Homogeneous field (no diffusion): the oracle is forward Euler on the
    reaction ODE of Eq. (1).  Written here in the equivalent form
        du/dt = [u(1-u) - (f v + phi)(1 - 2q/(u+q))]/eps,  dv/dt = u - v
    and solved by a stiff high-accuracy integrator, the error of the oracle at
    t = 0.2 (on the excited plateau, before the collapse into the refractory
    tail, where dt = 1e-3 is no longer Euler-stable) must halve when dt halves
    (first order), and be small."""
    eps, f, q, phi = P["eps"], P["f"], P["q"], 0.054

    def rhs(_t, y):
        u, v = y
        return [(u * (1 - u) - (f * v + phi) * (1 - 2 * q / (u + q))) / eps, u - v]

    t_end = 0.2
    ref = solve_ivp(rhs, (0, t_end), [0.6, 0.05], method="Radau", rtol=1e-12, atol=1e-14)
    ue, ve = ref.y[0, -1], ref.y[1, -1]
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        p = dict(P); p["dt"] = dt
        n = int(round(t_end / dt))
        r = oracle.Run(np.full((2, 2), 0.6), np.full((2, 2), 0.05), np.full((2, 2), phi), p)
        r.advance(n)
        errs.append(max(abs(r.u[0, 0] - ue), abs(r.v[0, 0] - ve)))
    assert errs[0] < 1e-3
    assert 1.95 < errs[0] / errs[1] < 2.05
    assert 1.95 < errs[1] / errs[2] < 2.05


# ---------------------------------------------------------------- P4 heat equation

def _no_reaction(params=P):
    p = dict(params); p["eps"] = math.inf      # c1 = dt/eps = 0: reaction off
    return p


@pytest.mark.parametrize("k,l", [(3, 2), (0, 1), (1, 0), (23, 15), (5, 7)])
def test_neumann_cosine_modes_decay_exactly(k, l):
    """With the reaction off, u follows the discrete heat equation with
    zero-flux (cell-centred) edges.  Its eigenvectors are
    cos(pi k (i+1/2)/nx) cos(pi l (j+1/2)/ny) with per-step factor
        lam = 1 - 4 r [sin^2(pi k/(2 nx)) + sin^2(pi l/(2 ny))],  r = dt D_u/dx^2.
    v then obeys v' = (1-dt) v + dt u, which sums in closed form:
        v_n = rho^n v0 + B (1 - rho^n) + A m dt (rho^n - lam^n)/(rho - lam),  rho = 1-dt.
    nx != ny so that a transposed index fails."""
    p = _no_reaction()
    nx, ny = 24, 16
    A, B, v0 = 0.3, 0.5, 0.1
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    m = np.cos(np.pi * k * (i + 0.5) / nx) * np.cos(np.pi * l * (j + 0.5) / ny)
    r_ = p["dt"] * p["D_u"] / p["dx"] ** 2
    lam = 1 - 4 * r_ * (np.sin(np.pi * k / (2 * nx)) ** 2 + np.sin(np.pi * l / (2 * ny)) ** 2)
    rho = 1 - p["dt"]
    n = 600
    run = oracle.Run(B + A * m, np.full((ny, nx), v0), np.full((ny, nx), 0.054), p)
    run.advance(n)
    assert np.max(np.abs(run.u - (B + A * m * lam ** n))) < 1e-13
    if abs(rho - lam) > 1e-12:
        coef = (rho ** n - lam ** n) / (rho - lam)
    else:
        coef = n * rho ** (n - 1)
    v_exp = rho ** n * v0 + B * (1 - rho ** n) + A * m * p["dt"] * coef
    assert np.max(np.abs(run.v - v_exp)) < 1e-13


def test_heat_equation_mass_is_conserved():
    """Zero-flux edges conserve the sum of u when the reaction is off."""
    u, v, phi = inputs.random_state(17, 11, seed=5)
    run = oracle.Run(u, v, phi, _no_reaction())
    s0 = run.u.sum()
    run.advance(300)
    assert abs(run.u.sum() - s0) < 1e-10 * abs(s0)


# ---------------------------------------------------------------- P5 Laplacian

def _laplacian_via_step(u):
    """L(u) read off one step with the reaction off and c2 = dt D/dx^2 = 2^-10
    (exact for small-integer fields)."""
    p = dict(eps=math.inf, f=1.4, q=0.002, D_u=1.0, dt=2.0 ** -10, dx=1.0)
    ny, nx = u.shape
    un, _ = oracle.step(u, np.zeros_like(u), np.zeros_like(u), p)
    return (un - u) * 2.0 ** 10


def test_laplacian_of_constant_is_zero():
    assert np.all(_laplacian_via_step(np.full((9, 13), 7.0)) == 0.0)


@pytest.mark.parametrize("a,b", [(3, 0), (0, -5), (2, 7)])
def test_laplacian_of_linear_field(a, b):
    """L(a x + b y) = 0 inside; on an edge cell the missing neighbour equals
    the cell itself, leaving +a at x=0, -a at x=nx-1, +b at y=0, -b at y=ny-1."""
    ny, nx = 9, 13
    y, x = np.mgrid[0:ny, 0:nx]
    L = _laplacian_via_step((a * x + b * y + 100).astype(np.float64))
    exp = np.zeros((ny, nx))
    exp[:, 0] += a
    exp[:, -1] -= a
    exp[0, :] += b
    exp[-1, :] -= b
    assert np.array_equal(L, exp)


def test_laplacian_sums_to_zero_on_integer_field():
    rng = np.random.default_rng(11)
    u = rng.integers(-50, 50, size=(10, 14)).astype(np.float64)
    assert _laplacian_via_step(u).sum() == 0.0


# ---------------------------------------------------------------- P7 brute force

def _dense_neumann_laplacian(nx, ny):
    """Explicit (nx*ny)^2 matrix of the five-node operator: for each cell and
    each of its four directions, +1 on the neighbour (or on the cell itself
    when the neighbour lies outside the grid), and -4 on the cell."""
    n = nx * ny
    M = np.zeros((n, n))
    for y in range(ny):
        for x in range(nx):
            c = y * nx + x
            M[c, c] -= 4
            for dx_, dy_ in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                xx, yy = x + dx_, y + dy_
                if 0 <= xx < nx and 0 <= yy < ny:
                    M[c, yy * nx + xx] += 1
                else:
                    M[c, c] += 1
    return M


def test_brute_force_8x8_matrix_form():
    """The whole step as a dense-matrix update on an 8x8 grid, 200 steps.
    The state is drawn where the Euler step is stable (v < 0.05, phi <= 0.1),
    so differences of summation order stay at rounding level."""
    nx = ny = 8
    M = _dense_neumann_laplacian(nx, ny)
    u, v, phi = inputs.random_state(nx, ny, seed=21, umax=0.9, vmax=0.05, phi_lo=0.04,
                                    phi_hi=0.1)
    p = P
    c1 = p["dt"] / p["eps"]
    c2 = p["dt"] * p["D_u"] / p["dx"] ** 2
    uu = u.astype(np.float64).ravel(); vv = v.astype(np.float64).ravel()
    ph = phi.astype(np.float64).ravel()
    run = oracle.Run(u, v, phi, p)
    for _ in range(200):
        react = uu - uu ** 2 - (p["f"] * vv + ph) * (uu - p["q"]) / (uu + p["q"])
        uu, vv = uu + c1 * react + c2 * (M @ uu), vv + p["dt"] * (uu - vv)
    run.advance(200)
    assert np.max(np.abs(run.u.ravel() - uu)) < 1e-12
    assert np.max(np.abs(run.v.ravel() - vv)) < 1e-12


def test_no_diffusion_cells_are_independent():
    """D_u = 0: each cell follows its own scalar recurrence, so permuting the
    cells of the input permutes the output identically (bitwise)."""
    p = dict(P); p["D_u"] = 0.0
    u, v, phi = inputs.random_state(9, 7, seed=4, vmax=0.05, phi_hi=0.1)
    perm = np.random.default_rng(1).permutation(63)
    a = oracle.Run(u, v, phi, p); a.advance(300)
    b = oracle.Run(u.ravel()[perm].reshape(7, 9), v.ravel()[perm].reshape(7, 9),
                   phi.ravel()[perm].reshape(7, 9), p)
    b.advance(300)
    assert np.array_equal(a.u.ravel()[perm], b.u.ravel())
    assert np.array_equal(a.v.ravel()[perm], b.v.ravel())


# ---------------------------------------------------------------- P6 symmetry

@pytest.mark.parametrize("sym", ["xflip", "yflip", "transpose"])
def test_d4_symmetry_is_bitwise(sym):
    """A mirror-symmetric start (symmetric phi, disks placed symmetrically)
    stays bitwise symmetric through waves, collisions and refractory tails."""
    n = 32
    _, _, phi = inputs.random_state(n, n, seed=8)
    def symmetrise(a):
        if sym == "xflip":
            return np.concatenate([a[:, : n // 2], a[:, : n // 2][:, ::-1]], axis=1)
        if sym == "yflip":
            return np.concatenate([a[: n // 2], a[: n // 2][::-1]], axis=0)
        return np.triu(a) + np.triu(a, 1).T
    phi = symmetrise(phi)
    disks = {"xflip": [(5, 9, 4), (n - 6, 9, 4), (12, 25, 3), (n - 13, 25, 3)],
             "yflip": [(9, 5, 4), (9, n - 6, 4), (25, 12, 3), (25, n - 13, 3)],
             "transpose": [(5, 20, 4), (20, 5, 4), (9, 9, 3)]}[sym]
    run = oracle.Run(np.zeros((n, n)), np.zeros((n, n)), phi, P)
    run.stimulate(disks)
    run.advance(1500)
    assert np.isfinite(run.u).all() and np.isfinite(run.v).all()
    assert run.v.max() > 0.05          # waves have passed
    op = {"xflip": lambda a: a[:, ::-1], "yflip": lambda a: a[::-1],
          "transpose": lambda a: a.T}[sym]
    assert np.array_equal(run.u, op(run.u))
    assert np.array_equal(run.v, op(run.v))


# ---------------------------------------------------------------- P2 period two

def test_inhibitory_background_settles_on_period_two_orbit():
    """phi = 0.2 at eps = 0.022: the rest state's Euler factor is below -1, so
    the homogeneous field leaves it and settles on a stable 2-cycle."""
    us = _rest_state(P, 0.2)
    assert oracle.euler_factor(P, us, us, 0.2) < -1
    assert oracle.euler_factor(P1, _rest_state(P1, 0.0975), _rest_state(P1, 0.0975), 0.0975) > -1
    run = oracle.Run(np.zeros((2, 2)), np.zeros((2, 2)), np.full((2, 2), 0.2), P)
    run.advance(25000)                 # v relaxes on the O(1/dt) step scale
    seq = []
    for _ in range(4):
        run.advance(1)
        seq.append(run.u[0, 0])
    assert abs(seq[0] - seq[2]) < 1e-9 and abs(seq[1] - seq[3]) < 1e-9
    assert abs(run.v[0, 0] - run.v[1, 1]) == 0.0
    assert abs(seq[0] - seq[1]) > 1e-3
    assert min(seq) < us < max(seq)


def _cell_map(params, phi, u, v):
    """One forward-Euler step of Eq. (1) for a cell of a homogeneous field
    (the five-node Laplacian of a constant is zero), written out here."""
    q = params["q"]
    react = (u - u * u - (params["f"] * v + phi) * (u - q) / (u + q)) / params["eps"]
    return u + params["dt"] * react, v + params["dt"] * (u - v)


def _two_cycle_newton(params, phi, guess):
    """A period-2 point of the cell map: Newton's method on F(F(x)) - x with
    a central-difference Jacobian."""
    def g(x):
        return np.array(_cell_map(params, phi, *_cell_map(params, phi, *x))) - x
    x = np.array(guess, dtype=np.float64)
    for _ in range(60):
        jac = np.empty((2, 2))
        for j in range(2):
            h = 1e-9 * max(1e-3, abs(x[j]))
            e = np.zeros(2)
            e[j] = h
            jac[:, j] = (g(x + e) - g(x - e)) / (2 * h)
        dx = np.linalg.solve(jac, -g(x))
        x = x + dx
        if np.abs(dx).max() < 1e-17:
            break
    return x


@pytest.mark.parametrize("eps", [0.022, 0.02, 0.0243])
def test_period_two_orbit_values_on_inhibitory_background(eps):
    """The 2-cycle the oracle settles on from u = v = 0 on phi = 0.2 is the
    one Newton's method finds for the cell map (to 1e-9 in u and v, with the
    phase the run reaches), a true 2-cycle (not the fixed point), and it
    meets the invariant the v-equation alone fixes: over one period v
    changes by dt (u1 - v1) + dt (u2 - v2) = 0, so u1 + u2 = v1 + v2."""
    p = dict(P, eps=eps)
    x1 = _two_cycle_newton(p, 0.2, (0.0011, 0.00247))
    x2 = np.array(_cell_map(p, 0.2, *x1))
    assert np.abs(x1 - x2).max() > 1e-4                         # not the fixed point
    assert abs((x1[0] + x2[0]) - (x1[1] + x2[1])) < 1e-15
    run = oracle.Run(np.zeros((2, 2)), np.zeros((2, 2)), np.full((2, 2), 0.2), p)
    run.advance(25000)
    a = np.array([run.u[0, 0], run.v[0, 0]])
    run.advance(1)
    b = np.array([run.u[0, 0], run.v[0, 0]])
    if np.abs(a - x1).max() > np.abs(a - x2).max():
        a, b = b, a
    assert np.abs(a - x1).max() < 1e-9 and np.abs(b - x2).max() < 1e-9
    assert abs((a[0] + b[0]) - (a[1] + b[1])) < 1e-12


# ---------------------------------------------------------------- timelapse

@pytest.mark.parametrize("rate,chunks", [(1, [7, 5]), (3, [1, 1, 10, 4]), (7, [20, 2])])
def test_timelapse_is_the_max_over_frames_every_rate_steps(rate, chunks):
    """Run.track_timelapse against a step-by-step record of every frame: the
    first frame is the state at attach time, then one frame after each step
    that leaves an index divisible by rate, however advance() is split."""
    u, v, phi = inputs.random_state(23, 17, seed=9)
    run = oracle.Run(u, v, phi, P)
    run.stimulate([(11, 8, 3)])
    run.advance(2)
    run.track_timelapse(rate)
    frames = [run.u.copy()]
    uu, vv = run.u.copy(), run.v.copy()
    t = run.step_index
    for n in chunks:
        run.advance(n)
        for _ in range(n):
            uu, vv = oracle.step(uu, vv, phi, P)
            t += 1
            if t % rate == 0:
                frames.append(uu.copy())
    assert np.array_equal(run.u, uu)
    assert np.array_equal(run.timelapse, np.max(frames, axis=0))
    assert len(frames) == 1 + (t // rate - 2 // rate)


# ---------------------------------------------------------------- Euler pole bound

def _one_cell_step(u, c, params):
    """One oracle step of a uniform field (no diffusion) at u with f v + phi = c."""
    v = (c - 0.054) / params["f"]
    un, _ = oracle.step(np.full((2, 2), u), np.full((2, 2), v), np.full((2, 2), 0.054), params)
    return un[0, 0]


def test_euler_step_from_nonnegative_u_stays_above_the_pole_iff_a_below_8q():
    """With a = dt (f v + phi) / eps, the reaction term's part of one Euler
    step maps u to u - a (u - q)/(u + q); over u >= 0 its minimum, at
    u + q = sqrt(2 a q), is 2 sqrt(2 a q) - a - q, above the pole -q iff
    a < 8 q.  The oracle's step (which adds dt (u - u^2) / eps >= 0) agrees:
    below the bound no u >= 0 steps past -q, and 10% above it the minimising
    u does.  The coarse stepper caps f v + phi of its outputs from this."""
    from paper_1901_06535_amd import surrogate
    q, eps, dt = P["q"], P["eps"], P["dt"]
    c8 = 8 * q * eps / dt
    assert surrogate.euler_safe_c(P, margin=0.0) == pytest.approx(c8, rel=1e-15)
    for frac in (0.5, 0.9, 0.99):
        c = frac * c8
        us = np.concatenate([np.linspace(0, 0.05, 2001), np.geomspace(1e-9, 1.0, 400)])
        lo = min(_one_cell_step(x, c, P) for x in us)
        assert lo > -q, (frac, lo)
    a = dt * 1.1 * c8 / eps
    ustar = np.sqrt(2 * a * q) - q
    assert _one_cell_step(ustar, 1.1 * c8, P) < -q


# ---------------------------------------------------------------- stimulation

def test_disk_cell_counts_match_gauss_circle():
    counts = _read_golden("gauss_circle.txt")
    for r, cnt in counts.items():
        r = int(r)
        n = 2 * r + 5
        u = np.zeros((n, n))
        oracle.stimulate(u, [(n // 2, n // 2, r)])
        assert int((u == 1.0).sum()) == int(cnt)


def test_stimulation_sets_u_only_and_clips():
    u = np.full((12, 10), 0.25)
    v = np.full((12, 10), 0.125)
    oracle.stimulate(u, [(0, 0, 5), (9, 11, 2)])
    # brute force: cells with (x-cx)^2 + (y-cy)^2 <= r^2
    y, x = np.mgrid[0:12, 0:10]
    inside = ((x ** 2 + y ** 2) <= 25) | (((x - 9) ** 2 + (y - 11) ** 2) <= 4)
    assert np.array_equal(u == 1.0, inside)
    assert np.all(u[~inside] == 0.25)
    assert np.all(v == 0.125)


# ---------------------------------------------------------------- trackers

def test_arrival_tracker_matches_brute_force_history():
    wl = inputs.single_disk(n=40, seed=3, steps=300)
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params, track_arrival=True, theta=0.5)
    run.run_schedule(wl.stimuli, 300)
    # brute force: keep every state, take the first index with u >= 0.5
    hist = []
    u = wl.u0.astype(np.float64); v = wl.v0.astype(np.float64)
    oracle.stimulate(u, [(s.cx, s.cy, s.r) for s in wl.stimuli])
    hist.append(u.copy())
    for _ in range(300):
        u, v = oracle.step(u, v, wl.phi, wl.params)
        hist.append(u)
    h = np.stack(hist) >= 0.5
    exp = np.where(h.any(0), h.argmax(0), oracle.NEVER)
    assert np.array_equal(run.arrival, exp)
    assert (run.arrival < oracle.NEVER).sum() > 81


def test_unstable_tracker_matches_brute_force():
    wl = inputs.single_disk(n=24, seed=9, steps=60)
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params, track_unstable=True, unstable_from=5)
    run.run_schedule(wl.stimuli, 60)
    u = wl.u0.astype(np.float64); v = wl.v0.astype(np.float64)
    phi = wl.phi.astype(np.float64)
    oracle.stimulate(u, [(s.cx, s.cy, s.r) for s in wl.stimuli])
    mask = np.zeros(u.shape, dtype=bool)
    first = -1
    for n in range(60):
        if n >= 5:
            fac = np.array([[oracle.euler_factor(wl.params, u[j, i], v[j, i], phi[j, i])
                             for i in range(24)] for j in range(24)])
            bad = fac < -1
            if bad.any() and first < 0:
                first = n
            mask |= bad
        u, v = oracle.step(u, v, phi, wl.params)
    assert np.array_equal(run.unstable.astype(bool), mask)
    assert run.first_unstable == first


def _front_speed(params, phi, nx=700, ny=3, steps=30000, x1=150, x2=550):
    """Cells per step of a planar wave in a strip of excitable medium (phi
    uniform), started from the settled rest state by a disk at the west end;
    from the arrival times (first step with u >= 0.5) at two columns."""
    z = np.zeros((ny, nx))
    ph = np.full((ny, nx), phi)
    rest = oracle.Run(z, z, ph, params)
    rest.advance(3000)
    run = oracle.Run(rest.u, rest.v, ph, params, track_arrival=True)
    run.stimulate([(0, ny // 2, 4)])
    run.advance(steps)
    a = run.arrival
    assert (a[:, x2] < oracle.NEVER).all()
    # planar: every row of the strip arrives at the same step
    assert (a[:, x1] == a[0, x1]).all() and (a[:, x2] == a[0, x2]).all()
    return (x2 - x1) / float(a[0, x2] - a[0, x1])


def test_front_speed_sanity():
    """Sanity (not a paper value): a planar front moves at a steady 0.021-0.022
    cells per step at the workload parameters, about 46 steps per cell, the
    figure the circuit generator's space-time spacing rule bounds from above
    (0.03); at Table 1 (smaller D_u, larger eps) it is slower."""
    c = _front_speed(P, inputs.PHI_ACTIVE_TABLE1)
    c_half = _front_speed(P, inputs.PHI_ACTIVE_TABLE1, x1=150, x2=350)
    print("  front speed %.5f cells/step (first half %.5f)" % (c, c_half))
    assert 0.020 <= c <= 0.023
    assert abs(c_half - c) <= 0.02 * c              # steady, not accelerating
    c1 = _front_speed(inputs.PARAMS_TABLE1, inputs.PHI_ACTIVE_TABLE1, steps=45000)
    print("  Table 1: %.5f cells/step" % c1)
    assert 0.010 <= c1 < 0.8 * c
