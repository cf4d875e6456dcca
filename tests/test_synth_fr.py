"""Input checks of the node-level (solution + flux point) generator: the flux
points sit on the element faces, neighbours list the same physical points,
and the face values are the element polynomial on the face."""

import numpy as np

import synth
from synth.workloads import _admissible


def test_fr_stencil_shape_and_admissibility():
    wl = synth.make_quad_fr_workload(N=6, seed=5)
    assert wl.n_sol == 16 and wl.n_flux == 16 and wl.n_v == 32
    assert np.all(np.diff(wl.rowptr) == 48)
    assert wl.cols.min() >= 0 and wl.cols.max() < wl.n_state_nodes
    assert _admissible(wl.gamma, wl.states).all()
    assert np.all(wl.v_weights[16:] == 0) and np.all(wl.v_weights[:16] > 0)
    # each element lists its own 16 solution points and 16 flux points once
    for e in (0, 7, 35):
        row = wl.cols[wl.rowptr[e]:wl.rowptr[e + 1]]
        assert np.array_equal(row[:16], e * 16 + np.arange(16))
        assert len(np.unique(row)) == 48


def test_fr_face_values_interpolate_polynomials_exactly():
    """A field that is a polynomial of degree <= 3 per element has its face
    values reproduced by the interpolant: target flux points of an element
    equal the target's polynomial on the face (checked with a cubic)."""
    from synth.workloads import _lagrange_at
    xi, _ = np.polynomial.legendre.leggauss(4)
    f = lambda x: 1.0 + 0.3 * x - 0.2 * x ** 2 + 0.05 * x ** 3
    vals = f(xi)
    assert abs(_lagrange_at(xi, -1.0) @ vals - f(-1.0)) < 1e-14
    assert abs(_lagrange_at(xi, 1.0) @ vals - f(1.0)) < 1e-14


def test_fr_target_mean_is_the_solution_point_mean():
    wl = synth.make_quad_fr_workload(N=6, seed=6)
    T = wl.target.reshape(4, wl.n_elem, wl.n_v)
    S = wl.states[:, :wl.n_elem * 16].reshape(4, wl.n_elem, 16)
    c = wl.v_weights / wl.v_weights.sum()
    np.testing.assert_allclose((T * c).sum(2), (S * c[:16]).sum(2), rtol=1e-13, atol=1e-13)
