"""Physics helpers for validation tests (numpy, float64): not part of any compute path.

project_to_surface moves a filtered state along its own helix onto the cylinder of
its layer and maps its covariance with the surface projection
Pi = I - g a^T, where g = (t_x, t_y, cot(theta), 0, omega, 0) is the change of the
state per unit transverse arc along the helix and a = (r_hat, 0, 0, 0, 0) / (r_hat . t)
is the arc needed to return a position offset to the surface.  Only projected
states are comparable with the simulated truth at the crossing.
"""
import numpy as np


def helix_point(x, s, kB):
    w = -kB * x[3]
    u = w * s
    small = np.abs(u) < 1e-6
    us = np.where(small, 1.0, u)
    A = np.where(small, 1 - u * u / 6, np.sin(us) / us)
    Bn = np.where(small, u / 2, 2 * np.sin(0.5 * us) ** 2 / us)
    tx, ty = np.cos(x[4]), np.sin(x[4])
    px = x[0] + s * (A * tx - Bn * ty)
    py = x[1] + s * (A * ty + Bn * tx)
    pz = x[2] + s / np.tan(x[5])
    ph = x[4] + u
    return px, py, pz, ph


def project_to_surface(x, Cm, r, kB, cx=0.0, cy=0.0):
    """x [6, n], Cm [6, 6, n] -> projected (x, C)."""
    x = np.array(x, np.float64)
    s = np.zeros(x.shape[1])
    for _ in range(30):
        px, py, pz, ph = helix_point(x, s, kB)
        ex, ey = px - cx, py - cy
        f = ex * ex + ey * ey - r * r
        fp = 2 * (ex * np.cos(ph) + ey * np.sin(ph))
        s = s - f / fp
    px, py, pz, ph = helix_point(x, s, kB)
    xp = x.copy()
    xp[0], xp[1], xp[2], xp[4] = px, py, pz, (ph + np.pi) % (2 * np.pi) - np.pi
    n = x.shape[1]
    rx, ry = (px - cx) / r, (py - cy) / r
    tx, ty = np.cos(ph), np.sin(ph)
    ca = rx * tx + ry * ty
    g = np.stack([tx, ty, 1 / np.tan(x[5]), np.zeros(n), -kB * x[3], np.zeros(n)])
    a = np.stack([rx / ca, ry / ca, np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)])
    Pi = np.eye(6)[:, :, None] - g[:, None, :] * a[None, :, :]
    Cp = np.einsum('ijn,jkn,lkn->iln', Pi, Cm, Pi)
    return xp, Cp


def project_to_plane(x, Cm, zd, kB):
    """As project_to_surface for the plane z = zd of a disk: the arc to the plane is
    s = (zd - z) tan(theta), and a z offset returns to the plane with a = e_z / cot."""
    x = np.array(x, np.float64)
    zd = np.broadcast_to(np.asarray(zd, np.float64), x[2].shape)
    cot = 1 / np.tan(x[5])
    s = (zd - x[2]) / cot
    px, py, pz, ph = helix_point(x, s, kB)
    xp = x.copy()
    xp[0], xp[1], xp[2], xp[4] = px, py, zd, (ph + np.pi) % (2 * np.pi) - np.pi
    n = x.shape[1]
    z0 = np.zeros(n)
    g = np.stack([np.cos(ph), np.sin(ph), cot, z0, -kB * x[3], z0])
    a = np.stack([z0, z0, 1 / cot, z0, z0, z0])
    Pi = np.eye(6)[:, :, None] - g[:, None, :] * a[None, :, :]
    Cp = np.einsum('ijn,jkn,lkn->iln', Pi, Cm, Pi)
    return xp, Cp


def pulls(est, cov, truth, idx=(3, 4, 5)):
    """Pulls of state components; phi differences are wrapped."""
    out = {}
    for p in idx:
        d = est[p] - truth[p]
        if p == 4:
            d = (d + np.pi) % (2 * np.pi) - np.pi
        out[p] = d / np.sqrt(cov[p, p])
    return out


# determinants of the equilibrated S on both sides of the 1e-2 fallback threshold
FALLBACK_DETS = [0.5, 0.02, 0.0105, 0.0101, 0.0099, 0.0095, 0.002]


def correlated_seeds(geom, dets):
    """External seeds on layer 0 whose first update has an innovation covariance S of a
    chosen conditioning: for each target d, a radial track (phi = 0, theta = pi/2) at
    (r_0, 0, 0) with a prior whose (y, z) block gives the measured rows of S the
    correlation rho = sqrt(1 - d).  There the crossing-point projection is H = rows
    (y) and (z) of the position, so S = diag(sigma_r^2, C_yy + sigma_rphi^2,
    C_zz + sigma_z^2) + C_yz off the diagonal, and the determinant of S scaled to unit
    diagonal is exactly 1 - rho^2 = d.  Returns hits [L][3][n], mask [n] (layer 0 only),
    seed_state [6][n] and seed_cov [21][n] (packed lower triangle), float32."""
    d = np.asarray(dets, np.float64)
    n = d.size
    L = geom.n_layers
    r0 = float(geom.radius[0])
    vr, vz = geom.sigma_rphi ** 2, geom.sigma_z ** 2
    a, b = 999.0 * vr, 999.0 * vz          # |rho| can reach 999/1000
    rho = np.sqrt(1.0 - d)
    cyz = rho * np.sqrt((a + vr) * (b + vz))
    full = np.zeros((6, 6, n))
    for i, v in enumerate([1e-4, a, b, 1e-4, 1e-6, 1e-6]):
        full[i, i] = v
    full[1, 2] = full[2, 1] = cyz
    cov = np.zeros((21, n))
    k = 0
    for i in range(6):
        for j in range(i + 1):
            cov[k] = full[i, j]
            k += 1
    state = np.zeros((6, n))
    state[0] = r0
    state[3] = 0.5
    state[5] = 0.5 * np.pi
    hits = np.zeros((L, 3, n), np.float32)
    hits[0, 0] = r0
    hits[0, 1] = 0.003
    hits[0, 2] = -0.02
    mask = np.ones(n, np.uint32)
    return hits, mask, state.astype(np.float32), cov.astype(np.float32)
