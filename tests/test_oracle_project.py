"""Pins of the oracle's projection (Eq. (1)-(3), Sec. 2.1) against things the
paper and the mathematics fix, not against a retyped copy of its code:

* the on-axis isotropic closed form of the EWA covariance;
* the EWA Jacobian as the numerical (central-difference) Jacobian of the
  pinhole map, with the 3D covariance built by scipy's quaternion routine;
* the real spherical-harmonic basis against scipy's complex harmonics and
  against orthonormality on the sphere (Gauss-Legendre quadrature).
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y
from scipy.spatial.transform import Rotation

from workloads.scenes import Camera


def _cam(w=64, h=48, fx=70.0, fy=55.0, R=None, t=None):
    return Camera(width=w, height=h, fx=fx, fy=fy, cx=w / 2, cy=h / 2,
                  R=np.eye(3) if R is None else R, t=np.zeros(3) if t is None else t)


def _one(orc, cam, mean, log_scale, quat, opacity=0.7, colors=None, sh_degree=-1):
    m = np.asarray([mean], np.float32)
    ls = np.asarray([log_scale], np.float32)
    q = np.asarray([quat], np.float32)
    op = np.asarray([opacity], np.float32)
    col = np.asarray([colors if colors is not None else [0.1, 0.2, 0.3]], np.float32)
    return orc.project(cam, m, ls, q, op, col, sh_degree)


@pytest.mark.parametrize("z,s", [(3.0, -2.0), (4.5, -1.2), (7.0, -3.0)])
def test_on_axis_isotropic_closed_form(orc, z, s):
    cam = _cam()
    rng = np.random.default_rng(1)
    q = rng.standard_normal(4)
    out = _one(orc, cam, [0.0, 0.0, z], [s, s, s], q / np.linalg.norm(q))
    sig = math.exp(float(np.float32(s)))
    s00 = cam.fx ** 2 * sig ** 2 / z ** 2 + 0.3
    s11 = cam.fy ** 2 * sig ** 2 / z ** 2 + 0.3
    np.testing.assert_allclose(out["cov2d"][0], [s00, 0.0, s11], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["conic_opacity"][0, :3], [1 / s00, 0.0, 1 / s11], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(out["means2D"][0], [cam.cx - 0.5, cam.cy - 0.5], rtol=0, atol=1e-12)
    assert out["depth"][0] == pytest.approx(z, rel=1e-14)
    ext = 3.0 * math.sqrt(max(s00, s11))
    assert out["extent"][0] == pytest.approx(ext, rel=1e-12)
    assert out["radius"][0] == math.ceil(ext)
    assert out["conic_opacity"][0, 3] == pytest.approx(0.7, rel=1e-7)


def _pinhole(cam, p):
    return np.array([cam.fx * p[0] / p[2] + cam.cx - 0.5, cam.fy * p[1] / p[2] + cam.cy - 0.5])


def _num_jacobian(cam, p):
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-5 * max(1.0, abs(p[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(cam, p + e) - _pinhole(cam, p - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_ewa_matches_numerical_jacobian(orc, seed):
    rng = np.random.default_rng(100 + seed)
    R = Rotation.from_rotvec(rng.normal(0, 0.15, 3)).as_matrix()
    t = rng.normal(0, 0.2, 3)
    cam = _cam(R=R, t=t)
    mean = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3), rng.uniform(3, 5)])
    ls = rng.normal(-2.0, 0.5, 3)
    q = rng.standard_normal(4)
    out = _one(orc, cam, mean, ls, q)
    mean32 = np.asarray(mean, np.float32).astype(np.float64)
    ls32 = np.asarray(ls, np.float32).astype(np.float64)
    q32 = np.asarray(q, np.float32).astype(np.float64)
    Rq = Rotation.from_quat([q32[1], q32[2], q32[3], q32[0]]).as_matrix()  # scipy: scalar last
    Sigma = Rq @ np.diag(np.exp(2 * ls32)) @ Rq.T
    p = R @ mean32 + t
    # no clamp is active: the mean is well inside 1.3 x the half field of view
    assert abs(p[0] / p[2]) < 1.3 * (cam.width / 2) / cam.fx
    J = _num_jacobian(cam, p)
    S2 = J @ R @ Sigma @ R.T @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(out["cov2d"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    inv = np.linalg.inv(S2)
    np.testing.assert_allclose(out["conic_opacity"][0, :3], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-6)
    np.testing.assert_allclose(out["means2D"][0], _pinhole(cam, p), rtol=1e-12)
    assert out["depth"][0] == pytest.approx(p[2], rel=1e-12)
    lmax = np.linalg.eigvalsh(S2).max()
    assert out["extent"][0] == pytest.approx(3 * math.sqrt(lmax), rel=1e-7)


def test_jacobian_clamp_far_off_screen(orc):
    """Off-screen means use the Jacobian at the ray clamped to 1.3 x the half
    field of view (reading: the 3DGS convention; the paper is silent)."""
    cam = _cam()
    mean = np.array([5.0, -4.0, 4.0])
    out = _one(orc, cam, mean, [-1.5, -1.7, -1.6], [1, 0, 0, 0])
    limx = 1.3 * (cam.width / 2) / cam.fx
    limy = 1.3 * (cam.height / 2) / cam.fy
    m32 = np.asarray(mean, np.float32).astype(np.float64)
    z = m32[2]
    pc = np.array([np.clip(m32[0] / z, -limx, limx) * z, np.clip(m32[1] / z, -limy, limy) * z, z])
    J = _num_jacobian(cam, pc)
    Sigma = np.diag(np.exp(2 * np.asarray([-1.5, -1.7, -1.6], np.float32).astype(np.float64)))
    S2 = J @ Sigma @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(out["cov2d"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    # the mean itself is not clamped
    np.testing.assert_allclose(out["means2D"][0], _pinhole(cam, m32), rtol=1e-12)


def test_near_plane_cull(orc):
    cam = _cam()
    out = _one(orc, cam, [0.0, 0.0, 0.15], [-2, -2, -2], [1, 0, 0, 0])
    assert out["radius"][0] == 0
    out = _one(orc, cam, [0.0, 0.0, -3.0], [-2, -2, -2], [1, 0, 0, 0])
    assert out["radius"][0] == 0


def _real_sh_scipy(l, m, d):
    d = np.asarray(d, np.float64)
    polar = math.acos(max(-1.0, min(1.0, d[2])))
    az = math.atan2(d[1], d[0])
    if m == 0:
        return float(np.real(sph_harm_y(l, 0, polar, az)))
    y = sph_harm_y(l, abs(m), polar, az)
    if m > 0:
        return float(math.sqrt(2) * (-1) ** m * np.real(y))
    return float(math.sqrt(2) * (-1) ** m * np.imag(y))


def test_sh_basis_matches_scipy(orc):
    rng = np.random.default_rng(7)
    for _ in range(40):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert orc.sh_basis(l, m, d) == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-12)


def test_sh_basis_orthonormal(orc):
    zs, wz = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phis = 2 * math.pi * np.arange(nphi) / nphi
    idx = [(l, m) for l in range(4) for m in range(-l, l + 1)]
    Y = np.zeros((len(idx), len(zs) * nphi))
    W = np.zeros(len(zs) * nphi)
    k = 0
    for zi, wzi in zip(zs, wz):
        s = math.sqrt(1 - zi * zi)
        for ph in phis:
            d = (s * math.cos(ph), s * math.sin(ph), zi)
            for r, (l, m) in enumerate(idx):
                Y[r, k] = orc.sh_basis(l, m, d)
            W[k] = wzi * 2 * math.pi / nphi
            k += 1
    G = (Y * W) @ Y.T
    np.testing.assert_allclose(G, np.eye(len(idx)), atol=1e-12)


def test_sh_colour_along_view_ray(orc):
    rng = np.random.default_rng(11)
    R = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix()
    t = np.array([0.3, -0.1, 0.4])
    cam = _cam(R=R, t=t)
    for deg in range(4):
        k = (deg + 1) ** 2
        coef = rng.normal(0, 0.4, (k, 3)).astype(np.float32)
        mean = np.array([0.2, -0.1, 4.0])
        out = _one(orc, cam, mean, [-2, -2, -2], [1, 0, 0, 0], colors=coef, sh_degree=deg)
        campos = -R.T @ t
        d = np.asarray(mean, np.float32).astype(np.float64) - campos
        d /= np.linalg.norm(d)
        want = np.full(3, 0.5)
        for l in range(deg + 1):
            for m in range(-l, l + 1):
                want += coef[l * l + l + m].astype(np.float64) * _real_sh_scipy(l, m, d)
        np.testing.assert_allclose(out["rgb"][0], np.maximum(want, 0.0), atol=1e-12)
