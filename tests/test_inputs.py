"""Checks of the seeded input generators (no GPU; torch on the CPU).

The generators hold none of the method's arithmetic; these tests only make
sure that the advective-product operands are what their names say: unit-RMS
velocity components and their derivatives along the named axis.
"""
import numpy as np

import ttm_inputs as I


def _dense(cores, n):
    x = cores[0]
    for c in cores[1:]:
        x = np.tensordot(x, c, axes=([-1], [0]))
    L = len(cores)
    x = x.reshape((2, 2, 2) * L)
    order = [3 * s for s in range(L)] + [3 * s + 1 for s in range(L)] + [3 * s + 2 for s in range(L)]
    return x.transpose(order).reshape(n, n, n)


def _central_difference(u, axis):
    """Eighth-order central difference on the periodic grid x_i = 2 pi i / n."""
    n = u.shape[axis]
    h = 2.0 * np.pi / n
    coef = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)
    return sum(c * (np.roll(u, -(m + 1), axis) - np.roll(u, m + 1, axis)) for m, c in enumerate(coef)) / h


def test_advective_operands_are_velocity_and_its_derivative():
    n = 32
    prods = I.advective_qtts_device(n, 7, chis=[0] * 9, device="cpu")
    assert len(prods) == 9
    u = [_dense(prods[4 * c][0], n) for c in range(3)]   # product (c, c) has A = u_c
    for c in range(3):
        assert abs(np.sqrt(np.mean(u[c] ** 2)) - 1.0) < 1e-12
    assert np.linalg.norm(u[0] - u[1]) > 0.5 * np.linalg.norm(u[0])
    for p, (A, B, chi) in enumerate(prods):
        i, j = divmod(p, 3)
        assert chi == 0
        assert np.allclose(_dense(A, n), u[j], rtol=0, atol=1e-12)
        du = _dense(B, n)
        ref = _central_difference(u[i], j)
        # the band-limited spectrum leaves the difference scheme ~0.6% off;
        # a wrong axis or sign would be off by order one
        assert np.linalg.norm(du - ref) <= 0.02 * np.linalg.norm(ref), p
        # periodic: the mean of a derivative is zero
        assert abs(du.mean()) <= 1e-12 * np.abs(du).mean()
    # sum over the grid of u_i d_i u_i vanishes (it is half the integral of a derivative)
    for i in range(3):
        assert abs(np.sum(u[i] * _dense(prods[4 * i][1], n))) <= 1e-10 * np.sum(np.abs(u[i]) ** 2)


def test_advective_bond_caps():
    chis = (8, 4, 2, 8, 4, 2, 8, 4, 2)
    prods = I.advective_qtts_device(16, 3, chis=chis, device="cpu")
    for (A, B, chi), c in zip(prods, chis):
        assert chi == c
        assert max(x.shape[2] for x in A) <= c and max(x.shape[2] for x in B) <= c


def test_binary_qtt_is_the_same_field():
    """Uncapped, the binary QTT (three d = 2 sites per d = 8 site) and the
    d = 8 QTT of the same seed decompress to the same tensor."""
    import oracle as O
    q8 = I.turbulence_qtt_device(16, 5, [0], "cpu")[0]
    q2 = I.turbulence_qtt_binary_device(16, 5, 0, "cpu")
    assert len(q8) == 4 and len(q2) == 12
    assert all(c.shape[1] == 2 for c in q2)
    d8 = O.dense(q8).reshape(-1)
    d2 = O.dense(q2).reshape(-1)
    assert np.abs(d8 - d2).max() <= 1e-12 * np.abs(d8).max()
