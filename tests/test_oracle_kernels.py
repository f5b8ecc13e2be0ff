"""Pins of the oracle's kernel functions and dense direct sum.

The project-written log and exp (used so that CPU and GPU evaluate the 2D and
Gaussian kernels identically) are checked against numpy's libm; the direct
sum (the plain definition of A x, Sec. 1) is checked against an explicit dense
matrix product.
"""
import numpy as np
import pytest


def test_log_matches_libm(orc):
    rng = np.random.default_rng(0)
    xs = np.concatenate([10.0 ** rng.uniform(-300, 300, 2000), rng.uniform(0.5, 2.0, 2000),
                         [1.0, 2.0, 0.5, np.sqrt(2.0), np.nextafter(np.sqrt(2.0), 2), 1e-310, 1.7e308]])
    for x in xs:
        a, b = orc.log(x), np.log(x)
        # a few units in the last place of the larger of |log x| and 1
        assert abs(a - b) <= 4 * np.spacing(max(abs(b), 1.0)), (x, a, b)


def test_log_is_exact_at_powers_of_two(orc):
    for e in range(-20, 21):
        assert orc.log(2.0 ** e) == e * float.fromhex("0x1.62e42fefa39efp-1")


def test_exp_matches_libm(orc):
    rng = np.random.default_rng(1)
    xs = np.concatenate([-rng.uniform(0, 700, 3000), -rng.uniform(0, 1, 1000), [0.0, -1e-300, -0.5]])
    for x in xs:
        a, b = orc.exp(x), np.exp(x)
        assert abs(a - b) <= 4 * np.spacing(b), (x, a, b)
    assert orc.exp(-800.0) == 0.0
    assert orc.exp(0.0) == 1.0


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("inv_r", 2), ("log_r", 2), ("gauss", 3), ("exp_r", 2),
                                    ("exp_r", 4)])
def test_kernel_diagonal_and_symmetry(orc, kind, d):
    rng = np.random.default_rng(2)
    a, b = rng.uniform(-1, 1, d), rng.uniform(-1, 1, d)
    assert orc.kernel_eval(kind, a, b, 0.5) == orc.kernel_eval(kind, b, a, 0.5)
    diag = orc.kernel_eval(kind, a, a, 0.5)
    assert diag == (1.0 if kind in ("gauss", "exp_r") else 0.0)
    r = np.linalg.norm(a - b)
    ref = {"inv_r": 1 / r, "log_r": np.log(r), "gauss": np.exp(-r * r / 0.25), "exp_r": np.exp(-r / 0.5)}[kind]
    assert abs(orc.kernel_eval(kind, a, b, 0.5) - ref) <= 1e-15 * max(1.0, abs(ref))


def _dense(kind, p, h=1.0):
    diff = p[:, None, :] - p[None, :, :]
    r = np.sqrt((diff ** 2).sum(-1))
    with np.errstate(divide="ignore"):
        if kind == "inv_r":
            K = np.where(r > 0, 1.0 / np.where(r > 0, r, 1), 0.0)
        elif kind == "log_r":
            K = np.where(r > 0, np.log(np.where(r > 0, r, 1)), 0.0)
        elif kind == "exp_r":
            K = np.exp(-r / h)
        else:
            K = np.exp(-r * r / (h * h))
    return K


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 3), ("exp_r", 2)])
def test_direct_equals_dense_product(orc, kind, d):
    rng = np.random.default_rng(3)
    p = rng.uniform(-1, 1, (700, d))
    p[5] = p[17]  # a duplicate point: K = 0 (1/r, log) or 1 (Gaussian, exp(-r/h)) there
    x = rng.standard_normal((700, 2))
    y = orc.direct(p, x, kind, 0.5)
    yd = _dense(kind, p, 0.5) @ x
    assert np.linalg.norm(y - yd) <= 1e-14 * np.linalg.norm(yd)
    rows = np.array([0, 5, 17, 699])
    ys = orc.direct(p, x, kind, 0.5, rows=rows)
    np.testing.assert_array_equal(ys, y[rows])
