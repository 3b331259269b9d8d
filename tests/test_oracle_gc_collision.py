"""Pin of the oracle's guiding-centre collision point (Sec. 3.1 "Drift mover" and
"Comparison": between interactions the particle moves on the exact helix around its guiding
centre; at an interaction the new guiding centre follows from the particle's position and new
velocity).

Inside the transport loop the oracle keeps only the guiding centre, the direction at the
last interaction and the path flown since then; at a collision it turns the direction by the
gyration angle of that path and places the particle on its gyro circle.  Nothing else pins
this: the helix tests call a separate restatement of the helix, and the flight tests have no
collision.  Here an off-axis electron beam in a uniform axial field makes exactly one
collision per history, an excitation that removes 90 % of its energy without turning it, so
the new guiding centre is x_c + (v'/v)(X - x_c) with x_c the particle's position at the
collision.  The r-faces crossed by that jump are tallied.  The expected tallies come from an
independent integration of m dv/dt = q v x B from the birth point over the exponential
distribution of the flown path (the free path redrawn at every z-face is still exponential
by memorylessness).  A reversed gyration, a collision point on the wrong side of the guiding
centre or a path that restarts at every z-face each moves the tallies by far more than their
statistical error (checked below).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2503_10263_amd import workloads as W

B = 0.01            # T
E0 = 100.0          # eV
E_X = 90.0          # eV: excitation energy; 10 eV is left, below every threshold
SIGMA = 1.0e-20     # m^2, constant
N_GAS = 1.67e22     # m^-3: mean free path 6 mm against 21 mm of helix per gyration
THETA = math.radians(60.0)
X0 = 3.0e-3         # m: birth point (X0, 0, 0), moving radially outward and along +z
RADIUS, N_R = 10.0e-3, 40
LENGTH, N_Z = 0.1, 100   # 1 mm z-cells: about three z-faces per flight before the collision
N = 20000


def _workload():
    proc = [W.Process(W.EXCITATION, W.ELECTRON, W.TARGET_GAS, E_X, np.full(256, SIGMA), "exc 90 eV")]
    return W.beam_problem(E0, proc, np.full(N_Z, N_GAS), LENGTH, radius=RADIUS, n_r=N_R, bz=B,
                          t_gas=0.0, n_primaries=N, seed=41,
                          beam_pos=(X0, 0.0, 0.0),
                          beam_dir=(math.sin(THETA), 0.0, math.cos(THETA)))


def _gc(pos, vel, q, m):
    """Guiding centre of a charge in a uniform axial field: x + (m / (q B)) (v x z_hat)."""
    return pos[:2] + (m / (q * B)) * np.array([vel[1], -vel[0]])


def _expected(gyration=+1.0, restart_at_faces=False, wrong_side=False):
    """Expected crossings per r-face (outward, inward) per history, from the Lorentz ODE.
    gyration=-1 integrates with the opposite sense of rotation, restart_at_faces=True counts
    the gyration angle from the last z-face only, wrong_side=True puts the collision point
    opposite the guiding centre: the mistakes the pin must reject."""
    m, q = W.M_E, -W.QE
    v = math.sqrt(2.0 * E0 * W.QE / m)
    vp = math.sqrt(2.0 * (E0 - E_X) * W.QE / m)
    d0 = np.array([math.sin(THETA), 0.0, math.cos(THETA)])
    y0 = np.concatenate([[X0, 0.0, 0.0], v * d0])
    # E_xs = E M/(m+M) only decides the threshold; the rate is n sigma at 100 eV
    rate = N_GAS * SIGMA
    s_max = 40.0 / rate

    def rhs(_, y):
        vv = y[3:]
        return np.concatenate([vv, gyration * (q / m) * np.array([vv[1] * B, -vv[0] * B, 0.0])])

    sol = integrate.solve_ivp(rhs, (0.0, s_max / v), y0, method="DOP853", rtol=1e-12,
                              atol=1e-15 * v, dense_output=True)
    s = np.linspace(0.0, s_max, 400001)
    if restart_at_faces:
        # the helix phase as if the path restarted at every z-face crossed
        dz_path = (LENGTH / N_Z) / math.cos(THETA)
        s_phase = np.mod(s, dz_path)
    else:
        s_phase = s
    y = sol.sol(s_phase / v)
    pos, vel = y[:3], y[3:]
    gc_old = _gc(np.array([X0, 0.0]), v * d0, q, m)
    if wrong_side:
        pos = pos.copy()
        pos[:2] = 2.0 * gc_old[:, None] - pos[:2]
    rho_old = float(np.hypot(*gc_old))
    gc_new = pos[:2] + (m / (q * B)) * (vp / v) * np.array([vel[1], -vel[0]])
    rho_new = np.hypot(gc_new[0], gc_new[1])
    faces = RADIUS * np.arange(N_R + 1) / N_R
    ir_old = int(np.sum(faces[1:N_R] <= rho_old))
    ir_new = np.searchsorted(faces[1:N_R], rho_new, side="right")
    # weights of the exponential path density on the grid (exact per interval)
    cdf = 1.0 - np.exp(-rate * s)
    wgt = np.diff(cdf)
    irm = ir_new[:-1]
    out = np.zeros(N_R + 1)
    inn = np.zeros(N_R + 1)
    for f in range(ir_old + 1, N_R):
        out[f] = np.sum(wgt[irm >= f])
    for f in range(1, ir_old + 1):
        inn[f] = np.sum(wgt[irm < f])
    return out, inn, ir_old


@pytest.fixture(scope="module")
def tallies(oracle_lib):
    import oracle
    return oracle.run(_workload(), 0, N)


def test_one_collision_per_history(tallies):
    """Every history makes its one excitation well inside the tube and leaves through the far
    end: the tallies below are those of one guiding-centre jump per history."""
    import oracle
    c = tallies["counters"]
    assert int(c[oracle.C_COLL]) == N
    exit_high, wall = oracle.C_DEATH + 1, oracle.C_DEATH + 2      # electrons, reasons 1 and 2
    assert int(c[exit_high]) == N and int(c[wall]) == 0


def test_gc_collision_crossings_match_lorentz_ode(tallies):
    jr = tallies["jr"]            # [S][n_r+1][n_z][2], dir 1 outward
    got_out = jr[0, :, :, 1].sum(axis=1).astype(float)
    got_in = jr[0, :, :, 0].sum(axis=1).astype(float)
    p_out, p_in, ir_old = _expected()
    assert got_out[N_R] == 0       # no wall loss: rho' + r_L' <= rho + r_L < R
    worst = 0.0
    n_checked = 0
    for f in range(1, N_R):
        for got, p in ((got_out[f], p_out[f]), (got_in[f], p_in[f])):
            sd = math.sqrt(max(N * p * (1.0 - p), 1.0))
            worst = max(worst, abs(got - N * p) / sd)
            n_checked += p > 0.01
    assert n_checked >= 6, n_checked    # the jump spreads over several faces
    assert worst < 5.0, worst


@pytest.mark.parametrize("mistake", ["reversed gyration", "path restarted at z-faces",
                                     "collision point opposite the guiding centre"])
def test_gc_pin_rejects_mistakes(tallies, mistake):
    """The same comparison against the two plausible mistakes fails by a wide margin, so the
    pin above has the power to see them."""
    jr = tallies["jr"]
    got_out = jr[0, :, :, 1].sum(axis=1).astype(float)
    got_in = jr[0, :, :, 0].sum(axis=1).astype(float)
    if mistake == "reversed gyration":
        p_out, p_in, _ = _expected(gyration=-1.0)
    elif mistake == "path restarted at z-faces":
        p_out, p_in, _ = _expected(restart_at_faces=True)
    else:
        p_out, p_in, _ = _expected(wrong_side=True)
    worst = 0.0
    for f in range(1, N_R):
        for got, p in ((got_out[f], p_out[f]), (got_in[f], p_in[f])):
            sd = math.sqrt(max(N * p * (1.0 - p), 1.0))
            worst = max(worst, abs(got - N * p) / sd)
    assert worst > 15.0, worst
