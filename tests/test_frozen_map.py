"""CPU checks of the fixed-step Rosenbrock map used as the adjoint's
finite-difference reference (tests/frozen_map.py): with the oracle's
right-hand side it converges to the oracle's converged solution at order 4
(the derived tableau's order, seen on a real nonlinear reactor), and its
central-difference gradient agrees with a one-step closed form."""
import numpy as np

from frozen_map import fd_gradient, fixed_map, step


def test_fixed_map_converges_at_order_four():
    from oracle.oracle import Oracle
    from synth.cells import make_cells
    c = make_cells("C1")
    o = Oracle(c["mech"].to_text())
    i = 100
    y0 = np.append(c["Y"][i], c["T"][i])
    dt = c["dt"][i] * 1e-2
    ref = o.integrate(c["T"][i:i + 1], c["p"][i:i + 1], c["Y"][i:i + 1], np.array([dt]), rtol=1e-12,
                      atol=1e-18)
    yref = np.append(ref["Y"][0], ref["T"][0])
    errs = []
    for ns in (8, 16, 32):
        y = fixed_map(o, y0, c["p"][i], dt, dt / ns)
        errs.append(np.max(np.abs(y - yref) / np.maximum(np.abs(yref), 1e-6)))
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(12.0 < r < 20.0 for r in ratios), (errs, ratios)


def test_linear_step_is_the_stability_function():
    """For y' = lam y the step multiplies by R(h lam) of the tableau."""
    from paper_2311_14941_amd.tableau import stability

    class Lin:
        lam = -3.0e3

        def rhs(self, y, p, dlnA=None):
            return self.lam * y

        def jac_cs(self, y, p, dlnA=None):
            return np.array([[self.lam]])

    o = Lin()
    for h in (1e-5, 1e-3, 1e-1):
        y1 = step(o, np.array([1.0]), 0.0, h)
        assert abs(y1[0] - stability(h * o.lam).real) < 1e-13 * max(1.0, abs(y1[0]))
    # and the central-difference gradient of the map is R(h lam)^n
    g, _ = fd_gradient(o, np.array([2.0]), 0.0, 1e-3, 2.5e-4, np.array([1.0]), np.zeros(1), [])
    assert abs(g[0] - stability(2.5e-4 * o.lam).real ** 4) < 1e-8
