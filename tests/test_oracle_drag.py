"""Pins of the oracle's pressure drag coefficient (the functional of the
adjoint study) and of its gradient: closed bodies in uniform pressure feel no
force, a linear pressure field gives the force of the divergence theorem, the
1/q_inf scaling, and the gradient against central differences of the whole
functional."""

import math

import numpy as np

import oracle
from eg_inputs import ogrid, cubed_sphere_shell
from tests.test_oracle_solver import perturbed


def _fit_state(O, p, fn):
    """Level-p coefficients whose expansion equals fn(x) (a function in the
    span of the element basis) at (p+1)^d points per element, by least
    squares on basis values obtained by evaluating unit coefficient vectors."""
    N, V = O.N(p), O.V
    u = O.zeros(p)
    g = np.linspace(-0.8, 0.8, p + 1)
    pts = np.array(np.meshgrid(*([g] * O.dim), indexing="ij")).reshape(O.dim, -1).T
    for e in range(O.ne):
        A = np.zeros((len(pts), N))
        rhs = np.zeros((len(pts), V))
        for k, xi in enumerate(pts):
            for i in range(N):
                unit = O.zeros(p)
                unit[e, 0, i] = 1.0
                Ui, x = O.eval_point(p, e, unit, xi)
                A[k, i] = Ui[0]
            rhs[k] = fn(x)
        u[e] = np.linalg.lstsq(A, rhs, rcond=None)[0].T
    return u


def test_uniform_pressure_no_drag():
    for mesh, p in ((ogrid(24, 3), 2), (cubed_sphere_shell(2, 1), 1)):
        O = oracle.Oracle(mesh, p, alpha_deg=4.0)
        assert abs(O.drag(p, O.freestream(p))) < 1e-13


def test_linear_pressure_divergence_theorem():
    """rho = 1, v = 0, p = p0 + a . x: the pressure force on the body B is
    -int_B grad p dV = -a |B|, so C_D = (a . d) |B| / (q_inf S_ref) with |B|
    the area of the faceted cylinder (a regular 24-gon of radius 0.5)."""
    n_th, p, gam, ma = 24, 1, 1.4, 0.3
    O = oracle.Oracle(ogrid(n_th, 2, r_out=3.0), p, mach=ma, alpha_deg=30.0)
    a = np.array([0.07, -0.05])
    d = O.freestream_direction()
    u = _fit_state(O, p, lambda x: np.array([1.0, 0.0, 0.0, (1.0 / gam + a @ x) / (gam - 1.0)]))
    area = 0.5 * n_th * 0.25 * math.sin(2 * math.pi / n_th)
    sref = 1.0
    ref = (a @ d) * area / (0.5 * ma * ma * sref)
    assert abs(O.drag(p, u, sref=sref) - ref) < 1e-12 * abs(ref) + 1e-14


def test_drag_scales_with_inverse_dynamic_pressure():
    mesh = ogrid(16, 3)
    O1 = oracle.Oracle(mesh, 2, mach=0.3)
    O2 = oracle.Oracle(mesh, 2, mach=0.2)
    u = perturbed(O1, 2, 5)
    assert abs(O2.drag(2, u) - O1.drag(2, u) * (0.3 / 0.2) ** 2) < 1e-12 * abs(O2.drag(2, u))


def test_drag_gradient_matches_central_differences():
    """dC_D/du along random directions against central differences of the
    whole functional (step 1e-5: truncation ~1e-10 relative)."""
    for mesh, p in ((ogrid(12, 3), 2), (cubed_sphere_shell(1, 1), 1)):
        O = oracle.Oracle(mesh, p, alpha_deg=2.0)
        u = perturbed(O, p, 7)
        c, g = O.drag(p, u, grad=True)
        rng = np.random.default_rng(8)
        for _ in range(3):
            du = rng.standard_normal(u.shape) * 1e-2
            h = 1e-5
            fd = (O.drag(p, u + h * du) - O.drag(p, u - h * du)) / (2 * h)
            an = float(np.sum(g * du))
            assert abs(fd - an) < 1e-7 * max(abs(an), 1e-12), (fd, an)
        # only the elements touching the wall carry a gradient
        tags = mesh.bface_tag
        wall = np.any(tags == 1, axis=1)
        assert np.all(g[~wall] == 0.0) and np.any(g[wall] != 0.0)
