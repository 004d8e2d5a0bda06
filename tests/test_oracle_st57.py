"""Pins of the oracle's ST57 model (the 57-state Shorten-type stand-in).

The real Shorten model is not available, so these pins check the oracle
against properties its written specification fixes:
  * the resting state is a fixed point with the seven prescribed conserved
    sums (four probability chains sum to 1, total Ca 2200 uM, total Mg
    1500 uM);
  * Heun steps preserve every linear invariant of the model to rounding
    (a dropped or mis-signed flux term in any block breaks one of them);
  * with both membrane voltages frozen (huge capacitance) the voltage-
    sensor chain relaxes to its closed-form Boltzmann distribution
    P_{i+1}/P_i = k_f,i/k_b,i = exp(2 (V_t - V_i) / 25);
  * the model is second order in time under Strang splitting, fires and
    propagates an action potential of the Hodgkin-Huxley shape, and keeps
    concentrations and probabilities non-negative;
  * every kinetic block (sensor chain, pump cycle, thin-filament chain,
    cross-bridge cycle) is first order in its own states, so the block's
    Jacobian is its kinetic generator: its off-diagonal entries are
    non-zero exactly on the edges the specification draws (chain or cycle,
    both directions), and positive there, and its columns sum to zero; the
    thin-filament chain's links share one forward and one backward rate.
    A mis-indexed, mis-signed or dropped transition in a block fails this
    without the test restating any rate formula;
  * the signs and zeros of Jacobian entries that the modelled processes fix
    (which way a flux moves a state, which states an equation involves),
    and the SR uptake's Hill coefficient of 2 from its low-calcium slope.
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module")
def rest():
    return O.rest_state(O.MODEL_ST57)


def test_rest_is_a_fixed_point_with_prescribed_sums(rest):
    G = O.st57_rhs(rest)
    scale = np.maximum(np.abs(rest), 1.0)
    assert np.max(np.abs(G) / scale) < 1e-10
    inv = O.st57_invariants(rest)
    np.testing.assert_allclose(inv, [1, 1, 1, 1, 2200, 1500], rtol=1e-13)
    # membrane near the Hodgkin-Huxley resting potential, gates in [0, 1]
    assert -80 < rest[0] < -70 and -80 < rest[4] < -70
    assert np.all(rest[1:4] > 0) and np.all(rest[1:4] < 1)
    assert np.all(rest[8:] >= 0)


def test_invariants_are_preserved_by_heun_steps(rest):
    rng = np.random.default_rng(1)
    y = rest[:, None] * (1 + 0.05 * rng.standard_normal((57, 6)))
    y[0] += np.array([0, 10, 30, 60, 90, 110])  # from rest to strongly depolarized
    inv0 = np.array([O.st57_invariants(y[:, i]) for i in range(6)])
    cfg = O.Config(model=O.MODEL_ST57, dt_0D=1e-4)
    I = np.array([0, 0, 500.0, 0, 0, 1200.0])
    for _ in range(50):
        y = O.reaction(cfg, y, 5e-4, I)
    inv1 = np.array([O.st57_invariants(y[:, i]) for i in range(6)])
    np.testing.assert_allclose(inv1, inv0, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Vt", [-90.0, -60.0, -30.0, 0.0, 25.0])
def test_sensor_chain_reaches_boltzmann_distribution(rest, Vt):
    y = rest.copy()
    y[4] = Vt
    y[8:18] = 0.1
    cfg = O.Config(model=O.MODEL_ST57, Cm=1e300, dt_0D=2e-3)
    yy = y[:, None]
    for _ in range(60):
        yy = O.reaction(cfg, yy, 1.0)  # 60 ms with frozen V and V_t
    P = yy[8:18, 0]
    Vi = -70.0 + 7.5 * np.arange(9)
    w = np.concatenate([[1.0], np.cumprod(np.exp(2 * (Vt - Vi) / 25.0))])
    np.testing.assert_allclose(P, w / w.sum(), rtol=1e-6, atol=1e-9)


def test_time_order_and_action_potential(rest):
    n = [120]
    y0 = np.tile(rest[:, None], (1, 120))
    stims = [dict(fiber=0, node=60, half_width=1, step_on=0, n_steps=200, period=0, amp=1200.0)]
    cfg = O.Config(model=O.MODEL_ST57, dt_0D=1e-4, dt_1D=5e-4, dt_split=5e-4)
    y, s, ta = O.run(cfg, n, y0, stims, 3000, sample_every=100)
    assert 15.0 < np.nanmax(s) < 45.0           # HH-shaped upstroke
    assert np.all(np.isfinite(ta[45:76]))       # propagated over +-15 nodes
    assert np.all(y[8:55] >= -1e-12)            # probabilities, concentrations
    # second order in time, continuing from the propagating state
    def solve(dt):
        c = O.Config(model=O.MODEL_ST57, dt_0D=dt / 2, dt_1D=dt, dt_split=dt)
        return O.run(c, n, y, [], int(round(0.2 / dt)))[0]
    ref = solve(0.2 / 3200)
    errs = np.array([np.max(np.abs(solve(dt)[0] - ref[0])) for dt in (2e-3, 1e-3, 5e-4)])
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(order - 2.0) < 0.2), order


def _block_generator(y, lo, n):
    """d G[lo:lo+n] / d y[lo:lo+n] by central differences (exact up to
    rounding for a block that is first order in its own states)."""
    J = np.zeros((n, n))
    for c in range(n):
        h = 1e-3
        yp, ym = y.copy(), y.copy()
        yp[lo + c] += h
        ym[lo + c] -= h
        J[:, c] = (O.st57_rhs(yp)[lo:lo + n] - O.st57_rhs(ym)[lo:lo + n]) / (2 * h)
    return J


def _chain(n):
    return {(i, i + 1) for i in range(n - 1)} | {(i + 1, i) for i in range(n - 1)}


def _cycle(n):
    return _chain(n) | {(n - 1, 0), (0, n - 1)}


@pytest.mark.parametrize("name,lo,n,edges", [
    ("sensor chain P", 8, 10, _chain(10)),
    ("pump cycle Q", 35, 4, _cycle(4)),
    ("thin-filament chain R", 39, 8, _chain(8)),
    ("cross-bridge cycle X", 47, 8, _cycle(8))])
def test_kinetic_blocks_have_the_specified_generators(rest, name, lo, n, edges):
    # a state away from rest, so that every rate takes a generic value
    rng = np.random.default_rng(7)
    y = rest * (1.0 + 0.2 * rng.random(57))
    y[4] = -35.0                      # tubular voltage: sensor rates far from rest's
    y[21] = 90.0                      # b_T: thin-filament activation theta = 0.64
    y[46] = 0.2                       # R_7: the cross-bridge attachment rate
    for x0, x1 in ((8, 18), (35, 39), (39, 47), (47, 55)):
        y[x0:x1] /= y[x0:x1].sum()    # each chain a distribution again
    J = _block_generator(y, lo, n)
    scale = np.max(np.abs(J))
    # A non-linear term in the block would make the generator depend on the
    # point: the same generator at a second point of the block.
    y2 = y.copy()
    y2[lo:lo + n] = rng.random(n)
    np.testing.assert_allclose(_block_generator(y2, lo, n), J, rtol=1e-6, atol=1e-9 * scale)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            if (j, i) in edges:       # transition j -> i feeds state i
                assert J[i, j] > 1e-6 * scale, (name, j, i, J[i, j])
            else:
                assert abs(J[i, j]) <= 1e-9 * scale, (name, j, i, J[i, j])
    assert np.all(np.diag(J) < 0)
    np.testing.assert_allclose(J.sum(axis=0), 0.0, atol=1e-9 * scale)
    if name.startswith("thin"):
        fwd = np.array([J[i + 1, i] for i in range(n - 1)])
        bwd = np.array([J[i, i + 1] for i in range(n - 1)])
        np.testing.assert_allclose(fwd, fwd[0], rtol=1e-7)
        np.testing.assert_allclose(bwd, bwd[0], rtol=1e-7)


def _jacobian_entries(y, pairs):
    """dG_i / dy_j by central differences for (i, j) in pairs."""
    out = {}
    for j in sorted({j for _, j in pairs}):
        h = 1e-4 * max(1.0, abs(y[j]))
        yp, ym = y.copy(), y.copy()
        yp[j] += h
        ym[j] -= h
        g = (O.st57_rhs(yp) - O.st57_rhs(ym)) / (2 * h)
        for i, jj in pairs:
            if jj == j:
                out[(i, j)] = g[i]
    return out


# (derivative of state i, state j, sign) fixed by what the specification
# models, not by its formulas: +1 the flux raises state i when state j
# grows, -1 it lowers it, 0 state i's equation does not involve state j.
_SIGNS = [
    # electrical coupling of surface (0) and tubular (4) membranes
    (0, 4, +1), (4, 0, +1),
    # each membrane's currents use its own gates only
    (0, 5, 0), (0, 6, 0), (0, 7, 0), (4, 1, 0), (4, 2, 0), (4, 3, 0),
    # pump turnover (J_p grows with Q_1): outward pump current, Na out of
    # the cell into the tubule, K from the tubule into the cell
    (0, 36, -1), (29, 36, -1), (32, 36, +1), (30, 36, +1), (33, 36, -1),
    # an outward chloride current carries Cl into the cell: the surface
    # current with V, the tubular one with V_t takes Cl from the tubule
    (31, 0, +1), (34, 4, -1),
    # SR: uptake from the myoplasm, transfer network -> junctional SR,
    # release through open channels (the junctional SR is loaded)
    (19, 18, +1), (20, 19, +1), (19, 20, +1), (18, 17, +1), (20, 17, -1),
    # unbinding from troponin, parvalbumin, ATP releases Ca; Mg likewise
    (18, 21, +1), (18, 22, +1), (18, 24, +1), (26, 23, +1), (26, 25, +1),
    # sensor chain: depolarization of the tubule moves sensors forward
    (8, 4, -1),
    # thin filament: Ca-bound troponin speeds activation
    (39, 21, -1),
    # cross-bridges: attachment driven by the last thin-filament state,
    # detachment from the last cross-bridge state speeded by Mg-free ATP
    (47, 46, -1), (48, 46, +1), (54, 25, -1), (47, 25, +1),
    # force: the strongly bound states X_4..X_7 only; it shortens L_s
    (56, 47, 0), (56, 48, 0), (56, 49, 0), (56, 50, 0),
    (56, 51, +1), (56, 52, +1), (56, 53, +1), (56, 54, +1), (55, 54, -1),
]


def test_jacobian_signs_follow_what_the_model_describes(rest):
    rng = np.random.default_rng(11)
    y = rest * (1.0 + 0.1 * rng.random(57))
    for x0, x1 in ((8, 18), (35, 39), (39, 47), (47, 55)):
        y[x0:x1] /= y[x0:x1].sum()
    J = _jacobian_entries(y, [(i, j) for i, j, _ in _SIGNS])
    scale = {i: max(abs(v) for (ii, _), v in J.items() if ii == i) for i, _, _ in _SIGNS}
    for i, j, sgn in _SIGNS:
        v = J[(i, j)]
        if sgn == 0:
            # a state that does not enter an equation leaves it bit for bit
            assert v == 0.0, (i, j, v)
        else:
            # well above the differences' rounding floor, with the sign
            assert v * sgn > 1e-10 * scale[i], (i, j, v)


def test_sr_uptake_is_cooperative_with_hill_coefficient_two(rest):
    # the network SR gains Ca only through uptake from the myoplasm, so
    # d(dc_s/dt)/dc_m is the uptake's slope, 8 c_m / (1 + c_m^2)^2 times a
    # constant: proportional to c_m at small c_m for a Hill coefficient of 2
    y = rest.copy()
    slope = []
    for c in (1e-3, 2e-3, 4e-3):
        y[18] = c
        J = _jacobian_entries(y, [(19, 18)])
        slope.append(J[(19, 18)])
    np.testing.assert_allclose(np.array(slope[1:]) / np.array(slope[:-1]), 2.0, rtol=2e-3)
