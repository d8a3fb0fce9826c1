"""Pins of the oracle's spectral Poisson solve: closed forms, a library DCT, convergence."""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import poisson
from oracle.geometry import Geometry


def _mode_map(geo, j, k, l, fx="c", fy="c", fz="c"):
    x = (np.arange(geo.nx) + 0.5) * geo.wb
    y = (np.arange(geo.ny) + 0.5) * geo.hb
    z = (np.arange(geo.nz) + 0.5) * geo.db
    f = {"c": np.cos, "s": np.sin}
    return (f[fz](l * np.pi * z / geo.dz)[:, None, None] * f[fy](k * np.pi * y / geo.die_y)[None, :, None]
            * f[fx](j * np.pi * x / geo.die_x)[None, None, :])


@pytest.mark.parametrize("jkl", [(1, 0, 0), (3, 2, 1), (0, 5, 1), (7, 1, 0)])
def test_single_cosine_mode_closed_form(jkl):
    geo = Geometry(40.0, 24.0, 16, 8, 2)
    j, k, l = jkl
    rho = _mode_map(geo, j, k, l)
    w = np.array([j * np.pi / geo.die_x, k * np.pi / geo.die_y, l * np.pi / geo.dz])
    w2 = float(np.sum(w ** 2))
    out = poisson.solve(rho, geo)
    np.testing.assert_allclose(out["phi"], rho / w2, atol=1e-12 * np.abs(rho / w2).max())
    np.testing.assert_allclose(out["ex"], w[0] / w2 * _mode_map(geo, j, k, l, fx="s"), atol=1e-12)
    np.testing.assert_allclose(out["ey"], w[1] / w2 * _mode_map(geo, j, k, l, fy="s"), atol=1e-12)
    np.testing.assert_allclose(out["ez"], w[2] / w2 * _mode_map(geo, j, k, l, fz="s"), atol=1e-12)


def test_constant_density_has_zero_potential_and_field():
    geo = Geometry(10.0, 10.0, 8, 8, 2)
    out = poisson.solve(np.full((2, 8, 8), 0.37), geo)
    for v in out.values():
        assert np.abs(v).max() < 1e-13


def test_round_trip_reproduces_density():
    rng = np.random.default_rng(3)
    geo = Geometry(16.0, 12.0, 16, 12, 4)
    rho = rng.random((4, 12, 16))
    a = poisson.coefficients(rho, geo)
    np.testing.assert_allclose(poisson.synthesize(a, geo), rho, atol=1e-13)


def test_potential_matches_scipy_dct_solution():
    """phi from an orthonormal DCT-II / DCT-III pair of a library, divided by |omega|^2."""
    rng = np.random.default_rng(11)
    geo = Geometry(30.0, 20.0, 12, 10, 4)
    rho = rng.random((4, 10, 12))
    X = sfft.dctn(rho, type=2, norm="ortho")
    l = np.arange(4)[:, None, None] * np.pi / geo.dz
    k = np.arange(10)[None, :, None] * np.pi / geo.die_y
    j = np.arange(12)[None, None, :] * np.pi / geo.die_x
    w2 = l ** 2 + k ** 2 + j ** 2
    Y = np.zeros_like(X)
    Y[w2 > 0] = X[w2 > 0] / w2[w2 > 0]
    phi_ref = sfft.idctn(Y, type=2, norm="ortho")
    phi = poisson.solve(rho, geo, want=("phi",))["phi"]
    np.testing.assert_allclose(phi, phi_ref, atol=1e-12 * np.abs(phi_ref).max())
    # the spectral Laplacian of phi is -(rho - mean rho)
    lap = sfft.idctn(-w2 * sfft.dctn(phi, type=2, norm="ortho"), type=2, norm="ortho")
    np.testing.assert_allclose(lap, -(rho - rho.mean()), atol=1e-12)


def _fd_laplacian_neumann(phi, geo):
    """7-point Laplacian with mirror (Neumann) ghost cells."""
    p = np.pad(phi, 1, mode="edge")
    c = p[1:-1, 1:-1, 1:-1]
    return ((p[1:-1, 1:-1, 2:] - 2 * c + p[1:-1, 1:-1, :-2]) / geo.wb ** 2
            + (p[1:-1, 2:, 1:-1] - 2 * c + p[1:-1, :-2, 1:-1]) / geo.hb ** 2
            + (p[2:, 1:-1, 1:-1] - 2 * c + p[:-2, 1:-1, 1:-1]) / geo.db ** 2)


def test_fd_laplacian_of_potential_converges_to_density_minus_mean():
    errs = []
    for n in (16, 32, 64):
        geo = Geometry(10.0, 10.0, n, n, n // 4)
        rho = 1.0 + _mode_map(geo, 1, 2, 1) + 0.5 * _mode_map(geo, 2, 1, 0)
        phi = poisson.solve(rho, geo, want=("phi",))["phi"]
        errs.append(np.abs(_fd_laplacian_neumann(phi, geo) + (rho - rho.mean())).max())
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5   # second order: 4x per halving


def test_field_is_minus_potential_gradient_by_central_differences():
    errs = []
    for n in (16, 32, 64):
        geo = Geometry(10.0, 8.0, n, n, n // 4)
        rho = _mode_map(geo, 1, 1, 1) + 0.3 * _mode_map(geo, 2, 3, 0)
        out = poisson.solve(rho, geo)
        phi, ex = out["phi"], out["ex"]
        # -dphi/dx between neighbouring centres against the mean of E at those centres
        dphi = -(phi[:, :, 1:] - phi[:, :, :-1]) / geo.wb
        eface = 0.5 * (ex[:, :, 1:] + ex[:, :, :-1])
        errs.append(np.abs(dphi - eface).max() / np.abs(ex).max())
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_field_points_away_from_a_density_peak():
    geo = Geometry(32.0, 32.0, 32, 32, 2)
    rho = np.zeros((2, 32, 32))
    rho[:, 14:18, 14:18] = 1.0
    out = poisson.solve(rho, geo)
    assert out["ex"][0, 16, 20] > 0 and out["ex"][0, 16, 11] < 0
    assert out["ey"][0, 20, 16] > 0 and out["ey"][0, 11, 16] < 0


def test_energy_gradient_with_respect_to_density_is_potential_times_bin_volume():
    rng = np.random.default_rng(2)
    geo = Geometry(12.0, 12.0, 6, 6, 2)
    rho = rng.random((2, 6, 6))
    phi = poisson.solve(rho, geo, want=("phi",))["phi"]
    for idx in [(0, 1, 2), (1, 5, 0), (1, 3, 3)]:
        e = np.zeros_like(rho)
        e[idx] = 1e-3
        up = poisson.energy(rho + e, poisson.solve(rho + e, geo, want=("phi",))["phi"], geo)
        dn = poisson.energy(rho - e, poisson.solve(rho - e, geo, want=("phi",))["phi"], geo)
        fd = (up - dn) / 2e-3
        assert abs(fd - phi[idx] * geo.vol_bin) < 1e-9 * max(1.0, abs(fd))


def test_potential_map_is_symmetric():
    """<phi(a), b> = <a, phi(b)>: the forward coefficients and the inverse sum share the cosine
    basis and the 1/|omega|^2 weights sit on the diagonal, so rho -> phi is a symmetric operator
    (what lets the autograd form reuse the solve as its own adjoint)."""
    rng = np.random.default_rng(3)
    geo = Geometry(30.0, 20.0, 12, 10, 4)
    a = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    b = rng.normal(size=(geo.nz, geo.ny, geo.nx))
    pa = poisson.solve(a, geo, want=("phi",))["phi"]
    pb = poisson.solve(b, geo, want=("phi",))["phi"]
    lhs, rhs = float(np.sum(pa * b)), float(np.sum(a * pb))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
