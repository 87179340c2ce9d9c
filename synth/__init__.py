"""Seeded synthetic detector events for the Kalman fit and the combinatorial finder.

Stand-in for the simulated CMS events the paper measures on (Sec. 4 and Sec. 5:
ttbar at PU 50/70 with the Phase-I geometry), which are not available here.
This module only *simulates* particles: exact helix crossings with cylindrical
layers, Gaussian hit smearing, Highland multiple-scattering kicks, uniform noise
hits and the bookkeeping around them.  It contains none of the filter's
arithmetic (no propagation Jacobian, no covariance, no gain, no seed fit).
Both the GPU path and the oracle consume exactly the float32 arrays produced
here.

Conventions shared with the filter (inputs only):
  * units: cm, GeV, rad, tesla; B is uniform along +z;
  * transverse direction phi, polar angle theta, kappa = q / pT;
  * the signed turning rate per unit transverse arc is omega = -k_B * kappa with
    k_B = 0.299792458e-2 * B  (cm^-1 GeV);
  * a layer L is an infinite cylinder of radius r_L; its alignment
    (dx, dy, dz, dphi) is a rigid transform about its own axis: the axis moves
    to (dx, dy), hits move by dz along z and rotate by dphi about the axis.
    Hits are always reported in the *nominal* frame of their layer.

The random stream is numpy's Philox4x32-10 (Salmon et al., SC'11) keyed by
(1906117440 + workload index, event index).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 1906117440
K_B_PER_TESLA = 0.299792458e-2   # GeV / (cm T)
M_PION = 0.13957039              # GeV
HIGHLAND_A = 0.0136              # GeV
HIGHLAND_B = 0.038
# Mean ionisation loss of a minimum-ionising particle per radiation length of silicon:
# (dE/dx)_min = 1.664 MeV cm^2/g times X0 = 21.82 g/cm^2 (PDG tables of atomic and
# nuclear properties of materials).
ELOSS_SI_GEV_PER_X0 = 0.0363


@dataclasses.dataclass
class Geometry:
    """Ideal barrel: concentric cylinders plus per-layer material and alignment."""
    radius: np.ndarray            # [L] cm, strictly increasing
    zhalf: np.ndarray             # [L] cm, half length used for z binning
    B: float = 3.8                # tesla
    xX0: np.ndarray | None = None  # [L] radiation lengths per layer crossing at normal incidence
    sigma_rphi: float = 0.01      # cm
    sigma_z: float = 0.1          # cm
    sigma_r: float = 0.001        # cm, radial regulariser of the 3-D hit
    mass: float = M_PION          # GeV, used in beta of the Highland formula
    n_phi_bins: int = 128
    n_z_bins: int = 32
    # Endcap disks (Sec. 3): layer l is the plane z = disk_z[l] (!= 0), active for radii
    # disk_rmin[l] .. disk_rmax[l] (its finder bins run over that radial range); other
    # layers are cylinders, active for |z| <= cyl_zmax[l] (0: unbounded).
    disk_z: np.ndarray | None = None
    disk_rmin: np.ndarray | None = None
    disk_rmax: np.ndarray | None = None
    cyl_zmax: np.ndarray | None = None

    def __post_init__(self):
        self.radius = np.asarray(self.radius, dtype=np.float64)
        self.zhalf = np.asarray(self.zhalf, dtype=np.float64)
        if self.xX0 is None:
            self.xX0 = np.zeros_like(self.radius)
        self.xX0 = np.asarray(self.xX0, dtype=np.float64)
        for f in ("disk_z", "disk_rmin", "disk_rmax", "cyl_zmax"):
            v = getattr(self, f)
            setattr(self, f, np.zeros_like(self.radius) if v is None else np.asarray(v, dtype=np.float64))

    @property
    def is_disk(self) -> np.ndarray:
        return self.disk_z != 0.0

    @property
    def has_disks(self) -> bool:
        return bool(np.any(self.is_disk))

    @property
    def n_layers(self) -> int:
        return int(self.radius.shape[0])

    @property
    def k_B(self) -> float:
        return K_B_PER_TESLA * self.B


def barrel(n_layers: int, r_min: float, r_max: float, B: float = 3.8,
           xX0: float = 0.0, eta_max: float = 1.5, **kw) -> Geometry:
    """Evenly spaced radii r_L = r_min + (r_max - r_min) L / (n_layers - 1).

    The binning half length is Z_L = 1.1 r_L sinh(eta_max): every track
    generated with |eta| < eta_max crosses layer L inside it (hits that stray
    beyond it after scattering are clamped into the edge bins by the finder).
    """
    r = r_min + (r_max - r_min) * np.arange(n_layers) / (n_layers - 1)
    z = 1.1 * r * math.sinh(eta_max)
    return Geometry(radius=r, zhalf=z, B=B, xX0=np.full(n_layers, xX0), **kw)


# eta regions of the seeds (Sec. 2: seeds are processed in regions of pseudorapidity):
# barrel, transition and endcap on each side, by the seed's |eta| (of its third hit)
ETA_REGION_EDGES = (0.9, 1.7)


def barrel_endcap(n_barrel: int = 17, r_min: float = 4.0, r_max: float = 110.0, zmax: float = 120.0,
                  disk_z=(130.0, 155.0, 180.0, 205.0, 230.0, 255.0, 280.0), disk_rmin: float = 20.0,
                  disk_rmax: float = 110.0, B: float = 3.8, xX0: float = 0.0, **kw) -> Geometry:
    """Barrel cylinders at radii r_min..r_max (evenly spaced), active for |z| <= zmax,
    then endcap disks at +disk_z, then at -disk_z, active for disk_rmin <= r <= disk_rmax.
    The cylinders' finder bins in z run over [-zmax, zmax]; the disks' over their radii."""
    nd = len(disk_z)
    r = r_min + (r_max - r_min) * np.arange(n_barrel) / (n_barrel - 1)
    L = n_barrel + 2 * nd
    radius = np.concatenate([r, np.full(2 * nd, disk_rmax)])
    dz = np.concatenate([np.zeros(n_barrel), np.asarray(disk_z, float), -np.asarray(disk_z, float)])
    return Geometry(radius=radius, zhalf=np.full(L, zmax), B=B, xX0=np.full(L, xX0), disk_z=dz,
                    disk_rmin=np.where(dz != 0, disk_rmin, 0.0), disk_rmax=np.where(dz != 0, disk_rmax, 0.0),
                    cyl_zmax=np.where(dz == 0, zmax, 0.0), **kw)


def eta_region(eta) -> np.ndarray:
    """Region of each |eta|: 0 barrel, 1 transition, 2 endcap (ETA_REGION_EDGES)."""
    a = np.abs(np.asarray(eta, np.float64))
    return (a >= ETA_REGION_EDGES[0]).astype(np.int32) + (a >= ETA_REGION_EDGES[1]).astype(np.int32)


def rng_for(workload: int, event: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[BASE_SEED + workload, event]))


# --------------------------------------------------------------------------------------
# particle kinematics
# --------------------------------------------------------------------------------------

def sample_particles(rng, n, pt_range=(0.5, 10.0), pt_log=False, eta_max=1.0):
    """Prompt particles from the origin: (pT, phi, eta, q)."""
    u = rng.random(n)
    if pt_log:
        lo, hi = pt_range
        pt = lo * (hi / lo) ** u
    else:
        pt = pt_range[0] + (pt_range[1] - pt_range[0]) * u
    phi = rng.uniform(-math.pi, math.pi, n)
    eta = rng.uniform(-eta_max, eta_max, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return pt, phi, eta, q


def highland_theta0(p, beta, x):
    """Highland's width of the projected scattering angle (PDG review, passage of
    particles through matter), for x radiation lengths traversed."""
    return HIGHLAND_A / (beta * p) * np.sqrt(x) * (1.0 + HIGHLAND_B * np.log(x))


def first_crossing(px, py, phi, omega, cx, cy, r):
    """Transverse arc length from (px, py) to the first forward crossing of the helix
    with the circle |p - c| = r, and the crossing point.

    Route: intersection of the helix's circle (centre p + n/omega) with the layer
    circle; of the two intersection points the one reached first moving forward
    wins.  Straight lines (omega == 0) use the line-circle root.  Returns
    (s, qx, qy); NaN where the layer is never reached.
    """
    px = np.asarray(px, np.float64)
    n = px.shape[0]
    s = np.full(n, np.nan)
    qx = np.full(n, np.nan)
    qy = np.full(n, np.nan)
    tx, ty = np.cos(phi), np.sin(phi)
    ex, ey = px - cx, py - cy                     # start relative to the layer axis
    e2 = ex * ex + ey * ey
    straight = omega == 0.0
    if np.any(straight):
        i = straight
        a = ex[i] * tx[i] + ey[i] * ty[i]
        disc = a * a - (e2[i] - r * r)
        ok = disc >= 0
        root = np.where(ok, -a + np.sqrt(np.maximum(disc, 0)), np.nan)
        root = np.where(root > 0, root, np.nan)
        s[i] = root
        qx[i] = px[i] + root * tx[i]
        qy[i] = py[i] + root * ty[i]
    curved = ~straight
    if np.any(curved):
        i = curved
        w = omega[i]
        nx, ny = -ty[i], tx[i]
        R = 1.0 / np.abs(w)
        ccx = px[i] + nx / w                      # centre of curvature
        ccy = py[i] + ny / w
        dx = ccx - cx
        dy = ccy - cy
        d = np.sqrt(dx * dx + dy * dy)
        # d^2 - R^2 written without cancelling the two large squares
        d2mR2 = e2[i] + 2.0 * (ex[i] * nx + ey[i] * ny) / w
        a_ = (r * r + d2mR2) / (2.0 * d)          # distance from the layer axis to the chord
        h2 = r * r - a_ * a_
        ok = h2 >= 0
        h = np.sqrt(np.maximum(h2, 0.0))
        ux, uy = dx / d, dy / d
        mx, my = cx + a_ * ux, cy + a_ * uy
        cand = [(mx - h * uy, my + h * ux), (mx + h * uy, my - h * ux)]
        psi_p = np.arctan2(py[i] - ccy, px[i] - ccx)
        best = np.full(w.shape, np.inf)
        bx = np.full(w.shape, np.nan)
        by = np.full(w.shape, np.nan)
        for (kx, ky) in cand:
            psi_q = np.arctan2(ky - ccy, kx - ccx)
            du = np.mod((psi_q - psi_p) * np.sign(w), 2.0 * math.pi)
            sq = du * R
            take = ok & (sq > 1e-9) & (sq < best)
            best = np.where(take, sq, best)
            bx = np.where(take, kx, bx)
            by = np.where(take, ky, by)
        best = np.where(np.isfinite(best), best, np.nan)
        s[i], qx[i], qy[i] = best, bx, by
    return s, qx, qy


@dataclasses.dataclass
class TrackSample:
    """Simulated tracks of one or more events (structure of arrays over tracks)."""
    hits: np.ndarray        # [L][3][N] float32, nominal-frame hit positions (NaN if absent)
    hit_mask: np.ndarray    # [N] uint32, bit L set <=> a hit on layer L
    truth: np.ndarray | None  # [L][6][N] float64, post-scatter state at each crossing
    truth_hit: np.ndarray | None  # [L][3][N] float64, unsmeared crossing points (aligned frame)
    pt: np.ndarray
    phi: np.ndarray
    eta: np.ndarray
    q: np.ndarray


def simulate(geom: Geometry, rng, n, pt_range=(0.5, 10.0), pt_log=False, eta_max=1.0,
             align=None, smear=True, scatter=True, keep_truth=True, particles=None,
             hit_dtype=np.float32, material=None, field=None):
    """Simulate n prompt tracks through every layer in turn.

    At each layer: exact crossing (first_crossing), record the unsmeared point,
    smear it along the cylinder (sigma_rphi in r*phi, sigma_z in z), then apply a
    Gaussian multiple-scattering kick with the Highland width for the crossing's
    path length (x/X0 / cos psi, cos psi = sin(theta) |r_hat . t|).  Without
    `material` the layer's x/X0 is geom.xX0 and the momentum magnitude is conserved.
    With material = (xX0_map [L][nz], eloss) the layer's x/X0 is the map
    interpolated at the crossing's z (material_at), and after the kick the energy
    drops by the mean ionisation loss eloss * x_eff / beta^2 (x_eff the same path
    length, beta at the incoming momentum); a particle left without kinetic energy
    stops.  With field = (c_r, c_z) the field is B_z(r, z) = B (1 + c_r r^2 + c_z z^2)
    (cm, global frame) and each step from one layer to the next is the helix of the
    field at the step's starting point.  A track that cannot reach a layer stops there;
    later layers have no hit.
    """
    if geom.has_disks:
        return _simulate_with_disks(geom, rng, n, pt_range, pt_log, eta_max, align, smear, scatter, keep_truth,
                                    particles, hit_dtype)
    L = geom.n_layers
    if particles is None:
        pt, phi0, eta, q = sample_particles(rng, n, pt_range, pt_log, eta_max)
    else:
        pt, phi0, eta, q = (np.asarray(a, np.float64) for a in particles)
        n = pt.shape[0]
    if align is None:
        align = np.zeros((L, 4))
    align = np.asarray(align, np.float64)
    theta = 2.0 * np.arctan(np.exp(-eta))
    kappa = q / pt
    phi = phi0.copy()
    x = np.zeros(n)
    y = np.zeros(n)
    z = np.zeros(n)
    alive = np.ones(n, dtype=bool)
    hits = np.full((L, 3, n), np.nan, dtype=hit_dtype)
    mask = np.zeros(n, dtype=np.uint32)
    truth = np.full((L, 6, n), np.nan) if keep_truth else None
    truth_hit = np.full((L, 3, n), np.nan) if keep_truth else None
    kB = geom.k_B
    for l in range(L):
        dx, dy, dz, dphi = align[l]
        r = geom.radius[l]
        if field is None:
            omega = -kB * kappa
        else:
            omega = -kB * (1.0 + field[0] * (x * x + y * y) + field[1] * z * z) * kappa
        s, qx, qy = first_crossing(x, y, phi, omega, dx, dy, r)
        reach = alive & np.isfinite(s)
        alive = reach
        s = np.where(reach, s, 0.0)
        x = np.where(reach, qx, x)
        y = np.where(reach, qy, y)
        z = z + s * np.cos(theta) / np.sin(theta)
        phi = np.mod(phi + omega * s + math.pi, 2.0 * math.pi) - math.pi
        # smeared measurement in the layer's true frame, reported in its nominal frame
        g1 = rng.standard_normal(n)
        g2 = rng.standard_normal(n)
        if not smear:
            g1[:] = 0.0
            g2[:] = 0.0
        ang = np.arctan2(y - dy, x - dx) + g1 * geom.sigma_rphi / r
        zm = z + g2 * geom.sigma_z
        loc = ang - dphi
        hits[l, 0] = np.where(reach, r * np.cos(loc), np.nan)
        hits[l, 1] = np.where(reach, r * np.sin(loc), np.nan)
        hits[l, 2] = np.where(reach, zm - dz, np.nan)
        mask |= np.where(reach, np.uint32(1) << np.uint32(l), np.uint32(0)).astype(np.uint32)
        if keep_truth:
            truth_hit[l] = np.where(reach, np.stack([x, y, z]), np.nan)
        # multiple scattering (and, with a material model, energy loss) at the crossing
        k1 = rng.standard_normal(n)
        k2 = rng.standard_normal(n)
        if material is None:
            xx = np.full(n, geom.xX0[l])
            eloss = 0.0
        else:
            xx = material_at(geom, material[0], l, z - dz)
            eloss = float(material[1])
        if scatter and np.any(xx > 0):
            st, ct = np.sin(theta), np.cos(theta)
            rhx, rhy = (x - dx) / r, (y - dy) / r
            cpsi = st * np.abs(rhx * np.cos(phi) + rhy * np.sin(phi))
            p = np.abs(1.0 / kappa) / st
            beta = p / np.sqrt(p * p + geom.mass ** 2)
            xe = np.where(xx > 0, xx / cpsi, 1.0)
            th0 = np.where(xx > 0, highland_theta0(p, beta, xe), 0.0)
            a = k1 * th0
            b = k2 * th0
            cp, sp = np.cos(phi), np.sin(phi)
            d0 = np.stack([st * cp, st * sp, ct])
            e1 = np.stack([ct * cp, ct * sp, -st])
            e2 = np.stack([-sp, cp, np.zeros(n)])
            dn = d0 + a * e1 + b * e2
            dn /= np.linalg.norm(dn, axis=0)
            th_new = np.arccos(np.clip(dn[2], -1.0, 1.0))
            ph_new = np.arctan2(dn[1], dn[0])
            p_new = p
            if eloss > 0:
                m2 = geom.mass ** 2
                e_new = np.sqrt(p * p + m2) - np.where(xx > 0, eloss * xe / (beta * beta), 0.0)
                stopped = reach & (e_new * e_new <= m2)
                p_new = np.sqrt(np.maximum(e_new * e_new - m2, 1e-300))
                alive = alive & ~stopped
            pt_new = p_new * np.sin(th_new)
            theta = np.where(reach, th_new, theta)
            phi = np.where(reach, ph_new, phi)
            kappa = np.where(reach, q / pt_new, kappa)
        if keep_truth:
            truth[l] = np.where(reach, np.stack([x, y, z, kappa, phi, theta]), np.nan)
    return TrackSample(hits=hits, hit_mask=mask, truth=truth, truth_hit=truth_hit,
                       pt=pt, phi=phi0, eta=eta, q=q)


def helix_step(x, y, phi, omega, s):
    """Transverse position and azimuth after a transverse arc s along the helix (the
    chord of the circle of curvature omega, written to stay exact as omega -> 0)."""
    u = omega * s
    small = np.abs(u) < 1e-6
    us = np.where(small, 1.0, u)
    A = np.where(small, 1.0 - u * u / 6.0, np.sin(us) / us)       # sin(u)/u
    Bn = np.where(small, 0.5 * u, (1.0 - np.cos(us)) / us)       # (1 - cos u)/u
    tx, ty = np.cos(phi), np.sin(phi)
    return x + s * (A * tx - Bn * ty), y + s * (A * ty + Bn * tx), phi + u


def _simulate_with_disks(geom, rng, n, pt_range, pt_log, eta_max, align, smear, scatter, keep_truth, particles,
                         hit_dtype):
    """simulate() for a geometry with endcap disks.  A particle visits the cylinders in
    turn, then the disks on its side of z (the sign of cot theta) in turn.  A surface it
    crosses outside its active area (|z| > cyl_zmax of a bounded cylinder; a radius
    outside a disk's range), or does not reach within half a turn, is passed over: no
    hit, no material.  An unbounded cylinder that is not reached stops the particle.
    A disk hit is smeared along the disk: sigma_z in r, sigma_rphi in r*phi; the
    scattering path length on a disk is x/X0 / |cos theta|.  Uniform field, one x/X0
    per layer."""
    L = geom.n_layers
    if particles is None:
        pt, phi0, eta, q = sample_particles(rng, n, pt_range, pt_log, eta_max)
    else:
        pt, phi0, eta, q = (np.asarray(a, np.float64) for a in particles)
        n = pt.shape[0]
    if align is None:
        align = np.zeros((L, 4))
    align = np.asarray(align, np.float64)
    theta = 2.0 * np.arctan(np.exp(-eta))
    kappa = q / pt
    phi = phi0.copy()
    x = np.zeros(n)
    y = np.zeros(n)
    z = np.zeros(n)
    alive = np.ones(n, dtype=bool)
    hits = np.full((L, 3, n), np.nan, dtype=hit_dtype)
    mask = np.zeros(n, dtype=np.uint32)
    truth = np.full((L, 6, n), np.nan) if keep_truth else None
    truth_hit = np.full((L, 3, n), np.nan) if keep_truth else None
    kB = geom.k_B
    for l in range(L):
        dx, dy, dz, dphi = align[l]
        omega = -kB * kappa
        cot = np.cos(theta) / np.sin(theta)
        if geom.is_disk[l]:
            zp = geom.disk_z[l] + dz
            side = np.sign(geom.disk_z[l]) == np.sign(cot)
            s = np.where(side & (cot != 0), (zp - z) / np.where(cot != 0, cot, 1.0), -1.0)
            ok = alive & side & (s > 0) & (np.abs(omega * s) < math.pi)
            s = np.where(ok, s, 0.0)
            qx, qy, qphi = helix_step(x, y, phi, omega, s)
            rr = np.hypot(qx - dx, qy - dy)
            reach = ok & (rr >= geom.disk_rmin[l]) & (rr <= geom.disk_rmax[l])
            znew = np.full(n, zp)
        else:
            r = geom.radius[l]
            s, qx, qy = first_crossing(x, y, phi, omega, dx, dy, r)
            got = alive & np.isfinite(s)
            s = np.where(got, s, 0.0)
            znew = z + s * cot
            qphi = phi + omega * s
            if geom.cyl_zmax[l] > 0:
                reach = got & (np.abs(znew - dz) <= geom.cyl_zmax[l])
            else:
                reach = got
                alive = got
        x = np.where(reach, qx, x)
        y = np.where(reach, qy, y)
        z = np.where(reach, znew, z)
        phi = np.where(reach, np.mod(qphi + math.pi, 2.0 * math.pi) - math.pi, phi)
        g1 = rng.standard_normal(n)
        g2 = rng.standard_normal(n)
        if not smear:
            g1[:] = 0.0
            g2[:] = 0.0
        ang = np.arctan2(y - dy, x - dx)
        if geom.is_disk[l]:
            rr = np.hypot(x - dx, y - dy)
            rm = rr + g2 * geom.sigma_z
            loc = ang + g1 * geom.sigma_rphi / np.maximum(rr, 1e-9) - dphi
            hx, hy, hz = rm * np.cos(loc), rm * np.sin(loc), np.full(n, geom.disk_z[l])
        else:
            r = geom.radius[l]
            loc = ang + g1 * geom.sigma_rphi / r - dphi
            hx, hy, hz = r * np.cos(loc), r * np.sin(loc), z + g2 * geom.sigma_z - dz
        hits[l, 0] = np.where(reach, hx, np.nan)
        hits[l, 1] = np.where(reach, hy, np.nan)
        hits[l, 2] = np.where(reach, hz, np.nan)
        mask |= np.where(reach, np.uint32(1) << np.uint32(l), np.uint32(0)).astype(np.uint32)
        if keep_truth:
            truth_hit[l] = np.where(reach, np.stack([x, y, z]), np.nan)
        k1 = rng.standard_normal(n)
        k2 = rng.standard_normal(n)
        xx = geom.xX0[l]
        if scatter and xx > 0:
            st, ct = np.sin(theta), np.cos(theta)
            cp, sp = np.cos(phi), np.sin(phi)
            if geom.is_disk[l]:
                cpsi = np.abs(ct)
            else:
                r = geom.radius[l]
                cpsi = st * np.abs((x - dx) / r * cp + (y - dy) / r * sp)
            p = np.abs(1.0 / kappa) / st
            beta = p / np.sqrt(p * p + geom.mass ** 2)
            th0 = highland_theta0(p, beta, xx / np.maximum(cpsi, 1e-12))
            a = k1 * th0
            b = k2 * th0
            d0 = np.stack([st * cp, st * sp, ct])
            e1 = np.stack([ct * cp, ct * sp, -st])
            e2 = np.stack([-sp, cp, np.zeros(n)])
            dn = d0 + a * e1 + b * e2
            dn /= np.linalg.norm(dn, axis=0)
            th_new = np.arccos(np.clip(dn[2], -1.0, 1.0))
            ph_new = np.arctan2(dn[1], dn[0])
            theta = np.where(reach, th_new, theta)
            phi = np.where(reach, ph_new, phi)
            kappa = np.where(reach, q / (p * np.sin(th_new)), kappa)
        if keep_truth:
            truth[l] = np.where(reach, np.stack([x, y, z, kappa, phi, theta]), np.nan)
    return TrackSample(hits=hits, hit_mask=mask, truth=truth, truth_hit=truth_hit,
                       pt=pt, phi=phi0, eta=eta, q=q)


def endcap_workload(n: int = 100_000, event: int = 0, eta_max: float = 2.5, workload: int = 11):
    """Tracks through the barrel-and-endcap geometry (barrel_endcap, x/X0 = 0.02 per
    layer), pT log-uniform 0.5-50 GeV, |eta| < eta_max, hits smeared and scattered.
    Tracks with hits on layers 0-2 can be fitted from three-hit seeds."""
    geom = barrel_endcap(xX0=0.02)
    ts = simulate(geom, rng_for(workload, event), n, (0.5, 50.0), True, eta_max)
    return geom, ts


# --------------------------------------------------------------------------------------
# material beyond one x/X0 per layer
# --------------------------------------------------------------------------------------

def material_map(geom: Geometry, nz: int = 16, workload: int = 7):
    """x/X0 at normal incidence at nz equally spaced z-bin centres of every layer,
    [L][nz]: the layer's own geom.xX0 (0.02 if it has none) rising as (1 + 1.5 (z/Z_L)^2)
    towards the ends (cables and supports), 0.01 more in the central bin (a service
    ring), and a seeded +-20% variation per bin."""
    rng = np.random.Generator(np.random.Philox(key=[BASE_SEED + workload, 2 ** 31 - 2]))
    L = geom.n_layers
    zc = (np.arange(nz) + 0.5) / nz * 2.0 - 1.0          # bin centres in units of Z_L
    base = np.where(geom.xX0 > 0, geom.xX0, 0.02)
    m = base[:, None] * (1.0 + 1.5 * zc[None, :] ** 2) * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, (L, nz)))
    m[:, nz // 2] += 0.01
    return m


def material_at(geom: Geometry, xmap, l, z):
    """x/X0 of layer l at z (cm, in the layer's own frame): linear interpolation
    between the bin centres of xmap[l] over [-Z_L, Z_L], constant beyond the outer
    centres."""
    xmap = np.asarray(xmap, np.float64)
    nz = xmap.shape[1]
    if nz == 1:
        return np.full(np.shape(z), xmap[l, 0])
    u = (np.asarray(z, np.float64) + geom.zhalf[l]) / (2.0 * geom.zhalf[l]) * nz - 0.5
    u = np.clip(u, 0.0, nz - 1.0)
    k = np.minimum(np.floor(u).astype(np.int64), nz - 2)
    t = u - k
    return xmap[l, k] * (1.0 - t) + xmap[l, k + 1] * t


def material_workload(n: int = 100_000, event: int = 0, nz: int = 16, eloss: float = ELOSS_SI_GEV_PER_X0):
    """The 17-layer fit workload (pT log-uniform 0.5..50 GeV, |eta| < 1.5) through a
    material map with energy loss: returns (geom, ts, (xmap, eloss))."""
    geom = workload_geometry(2)
    xmap = material_map(geom, nz)
    ts = simulate(geom, rng_for(7, event), n, (0.5, 50.0), True, 1.5, material=(xmap, eloss))
    return geom, ts, (xmap, eloss)


# A solenoid-like field falling off away from the centre: 1.2% lower at r = 110 cm and
# 16% lower at |z| = 200 cm (coefficients of B_z(r, z) = B (1 + c_r r^2 + c_z z^2), cm^-2).
FIELD_SOLENOID = (-1.0e-6, -4.0e-6)


def field_workload(n: int = 100_000, event: int = 0, field=FIELD_SOLENOID, material=True):
    """The 17-layer fit workload in the field B_z(r, z) (and, with material=True, through
    the material map with silicon's energy loss): returns (geom, ts, field, material or None)."""
    geom = workload_geometry(2)
    mat = (material_map(geom, 16), ELOSS_SI_GEV_PER_X0) if material else None
    ts = simulate(geom, rng_for(9, event), n, (0.5, 50.0), True, 1.5, material=mat, field=field)
    return geom, ts, field, mat


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------

def workload_geometry(k: int) -> Geometry:
    """Geometry of workload k (1..5)."""
    if k == 1:
        return barrel(10, 4.0, 100.0, B=3.8, xX0=0.0, eta_max=1.0)
    return barrel(17, 4.0, 110.0, B=3.8, xX0=0.02, eta_max=1.5)


def fit_workload(k: int, n: int | None = None, keep_truth=False, align=None, event=0):
    """Tracks for the fit workloads.

    k = 1: 1 000 tracks, 10 layers 4..100 cm, no material, pT ~ U(0.5, 10), |eta| < 1.
    k = 2: 1e6 tracks, 17 layers 4..110 cm, x/X0 = 0.02, pT log-uniform 0.5..50, |eta| < 1.5.
    k = 4: as 2 with 1e5 tracks and a per-layer misalignment (see misalignment()).
    """
    geom = workload_geometry(k)
    rng = rng_for(k, event)
    if k == 1:
        n = 1000 if n is None else n
        ts = simulate(geom, rng, n, (0.5, 10.0), False, 1.0, keep_truth=keep_truth, align=align)
    else:
        n = (1_000_000 if k == 2 else 100_000) if n is None else n
        if k == 4 and align is None:
            align = misalignment(geom.n_layers)
        ts = simulate(geom, rng, n, (0.5, 50.0), True, 1.5, keep_truth=keep_truth, align=align)
    return geom, ts


def misalignment(n_layers: int, sigma_shift=0.005, sigma_rot=1e-4, workload=4):
    """True per-layer alignment (dx, dy, dz, dphi): N(0, 50 um) shifts, N(0, 0.1 mrad) rotation."""
    rng = np.random.Generator(np.random.Philox(key=[BASE_SEED + workload, 2 ** 31 - 1]))
    a = rng.standard_normal((n_layers, 4))
    a[:, :3] *= sigma_shift
    a[:, 3] *= sigma_rot
    return a


@dataclasses.dataclass
class EventBatch:
    """Hits of several events for the finder, grouped by event then by layer.

    hit_off[e][L] .. hit_off[e][L+1] is the slice of event e's hits on layer L in the
    global arrays (hit_off[e][n_layers] == hit_off[e+1][0]).
    """
    hits: np.ndarray        # [3][H] float32 nominal-frame positions
    hit_off: np.ndarray     # [E][L+1] int64
    hit_track: np.ndarray   # [H] int64 global track id, -1 for noise
    seed_hits: np.ndarray   # [3][S] int32 global hit indices on layers 0, 1, 2
    seed_event: np.ndarray  # [S] int32
    seed_track: np.ndarray  # [S] int64 global track id of the seed
    track_event: np.ndarray  # [T] int32
    track_hits: np.ndarray  # [L][T] int64 global hit index of each track's hit (-1 none)
    n_tracks: np.ndarray    # [E]


def make_events(geom: Geometry, n_tracks_per_event, workload=3, noise_frac=0.2,
                pt_range=(0.5, 50.0), pt_log=True, eta_max=1.5, scatter=True, smear=True,
                first_event=0, material=None, field=None):
    """Events for the finder: simulated tracks plus noise hits, shuffled per layer.

    Noise: round(noise_frac * true hits on L) hits uniform in phi in [-pi, pi) and in
    z in [-Z_L, Z_L], on the cylinder.  Seeds are the true triplets on layers 0-2.
    material / field: as for simulate().
    """
    L = geom.n_layers
    all_hits, offs, tr_ids, seeds, seed_ev, seed_tr = [], [], [], [], [], []
    track_ev, track_hits = [], []
    base = 0
    tid_base = 0
    for e, nt in enumerate(n_tracks_per_event):
        rng = rng_for(workload, first_event + e)
        ts = simulate(geom, rng, int(nt), pt_range, pt_log, eta_max, keep_truth=False,
                      smear=smear, scatter=scatter, material=material, field=field)
        off = np.zeros(L + 1, dtype=np.int64)
        ev_hits = []
        ev_trk = []
        pos_of = np.full((L, int(nt)), -1, dtype=np.int64)
        for l in range(L):
            have = (ts.hit_mask >> np.uint32(l)) & np.uint32(1)
            idx = np.nonzero(have)[0]
            h = ts.hits[l][:, idx].astype(np.float32)
            nn = int(round(noise_frac * idx.shape[0]))
            ph = rng.uniform(-math.pi, math.pi, nn)
            if geom.is_disk[l]:   # on the disk: uniform in phi and in its radii
                rr = rng.uniform(geom.disk_rmin[l], geom.disk_rmax[l], nn)
                hn = np.stack([rr * np.cos(ph), rr * np.sin(ph), np.full(nn, geom.disk_z[l])]).astype(np.float32)
            else:
                zz = rng.uniform(-geom.zhalf[l], geom.zhalf[l], nn)
                rr = geom.radius[l]
                hn = np.stack([rr * np.cos(ph), rr * np.sin(ph), zz]).astype(np.float32)
            hl = np.concatenate([h, hn], axis=1)
            tl = np.concatenate([idx.astype(np.int64) + tid_base, np.full(nn, -1, np.int64)])
            perm = rng.permutation(hl.shape[1])
            hl = hl[:, perm]
            tl = tl[perm]
            inv = np.empty_like(perm)
            inv[perm] = np.arange(perm.shape[0])
            pos_of[l, idx] = base + off[l] + inv[: idx.shape[0]]
            ev_hits.append(hl)
            ev_trk.append(tl)
            off[l + 1] = off[l] + hl.shape[1]
        all_hits.append(np.concatenate(ev_hits, axis=1))
        tr_ids.append(np.concatenate(ev_trk))
        offs.append(off + base)
        ok = (pos_of[0] >= 0) & (pos_of[1] >= 0) & (pos_of[2] >= 0)
        sidx = np.nonzero(ok)[0]
        if geom.has_disks:
            # seeds grouped by eta region (of the seed's third hit) within the event, the
            # order in which they are processed (Sec. 2)
            p2 = pos_of[2, sidx] - base
            zz = np.concatenate(ev_hits, axis=1)[2, p2].astype(np.float64)
            rr = np.hypot(*np.concatenate(ev_hits, axis=1)[:2, p2].astype(np.float64))
            sidx = sidx[np.argsort(eta_region(np.arcsinh(zz / rr)), kind="stable")]
        seeds.append(pos_of[:3, sidx].astype(np.int32))
        seed_ev.append(np.full(sidx.shape[0], e, np.int32))
        seed_tr.append(sidx.astype(np.int64) + tid_base)
        track_ev.append(np.full(int(nt), e, np.int32))
        track_hits.append(pos_of)
        base += int(off[L])
        tid_base += int(nt)
    return EventBatch(
        hits=np.ascontiguousarray(np.concatenate(all_hits, axis=1)),
        hit_off=np.stack(offs).astype(np.int64),
        hit_track=np.concatenate(tr_ids),
        seed_hits=np.ascontiguousarray(np.concatenate(seeds, axis=1)),
        seed_event=np.concatenate(seed_ev),
        seed_track=np.concatenate(seed_tr),
        track_event=np.concatenate(track_ev),
        track_hits=np.concatenate(track_hits, axis=1),
        n_tracks=np.asarray(n_tracks_per_event, dtype=np.int64),
    )


def endcap_find_workload(n_tracks: int = 5000, n_events: int = 1, eta_max: float = 2.5, workload: int = 12):
    """Events of n_tracks tracks each in the barrel-and-endcap geometry (x/X0 = 0.02 per
    layer), |eta| < eta_max, 20% noise per layer, seeds grouped by eta region."""
    geom = barrel_endcap(xX0=0.02)
    return geom, make_events(geom, [n_tracks] * n_events, workload=workload, eta_max=eta_max)


def find_workload(k: int = 3, n_tracks: int | None = None, n_events: int | None = None):
    """k = 3: one event of 5 000 tracks.  k = 5: 64 events with Poisson(mu_e) tracks,
    mu_e ~ U(5 000, 20 000).  Geometry and noise as in the 17-layer fit workload."""
    geom = workload_geometry(2)
    if k == 3:
        nt = [5000 if n_tracks is None else n_tracks] * (1 if n_events is None else n_events)
    else:
        ne = 64 if n_events is None else n_events
        rng = rng_for(k, 2 ** 31 - 2)
        mu = rng.uniform(5000, 20000, ne)
        nt = rng.poisson(mu)
        if n_tracks is not None:   # scaled-down copy of the same pileup mix
            nt = np.maximum(1, np.round(nt * (n_tracks / 12500.0))).astype(np.int64)
    return geom, make_events(geom, nt, workload=k)


# --------------------------------------------------------------------------------------
# injected duplicate seeds (tests of duplicate handling)
# --------------------------------------------------------------------------------------

def inject_duplicate_seeds(geom: Geometry, ev: EventBatch, frac: float = 0.1, workload: int = 6):
    """A copy of `ev` with duplicates of a fraction `frac` of its seeds appended after
    all the original seeds, as a detector with overlapping modules makes them: the same
    track measured twice on a layer.  A duplicate replaces, in turn, hit 0, hit 1, hit 2,
    hits 1 and 2, or all three hits of its original by a second measurement of the
    same crossing (the
    original hit moved along the cylinder by N(0, 2 sigma_rphi^2) in r*phi and
    N(0, 2 sigma_z^2) in z, so that the pair differs as two independent measurements
    do).  The new hits join their event's layer slices (after the existing hits there).

    Returns (batch, dup_of): dup_of [S'] is the original seed of each injected seed and
    -1 for the original seeds; seed_track of a duplicate is its original's track."""
    rng = rng_for(workload)
    S = ev.seed_hits.shape[1]
    L = geom.n_layers
    E = ev.hit_off.shape[0]
    pick = np.nonzero(rng.random(S) < frac)[0]
    variants = np.arange(pick.shape[0]) % 5          # 0, 1, 2: that hit; 3: hits 1, 2; 4: all
    new = {}                                          # (event, layer) -> list of (x, y, z, track)
    dup_hits = np.array(ev.seed_hits[:, pick], np.int64)
    new_ref = []                                      # (k, l, event, position in new list)
    for k, s in enumerate(pick):
        e = int(ev.seed_event[s])
        layers = [variants[k]] if variants[k] < 3 else ([1, 2] if variants[k] == 3 else [0, 1, 2])
        for l in layers:
            j = int(ev.seed_hits[l, s])
            x, y, z = (float(ev.hits[q, j]) for q in range(3))
            r = geom.radius[l]
            ang = math.atan2(y, x) + rng.normal() * math.sqrt(2.0) * geom.sigma_rphi / r
            zz = z + rng.normal() * math.sqrt(2.0) * geom.sigma_z
            lst = new.setdefault((e, l), [])
            new_ref.append((k, l, e, len(lst)))
            lst.append((r * math.cos(ang), r * math.sin(ang), zz, int(ev.hit_track[j])))
    # rebuild the hit arrays event by event, layer by layer, with the new hits at the
    # end of each slice
    old_to_new = np.empty(ev.hits.shape[1], np.int64)
    hits, tracks, offs = [], [], np.zeros_like(ev.hit_off)
    start_of_new = {}
    pos = 0
    for e in range(E):
        for l in range(L):
            a, b = int(ev.hit_off[e, l]), int(ev.hit_off[e, l + 1])
            offs[e, l] = pos
            old_to_new[a:b] = pos + np.arange(b - a)
            hits.append(ev.hits[:, a:b])
            tracks.append(ev.hit_track[a:b])
            pos += b - a
            extra = new.get((e, l), [])
            start_of_new[(e, l)] = pos
            if extra:
                arr = np.array(extra, np.float64)
                hits.append(arr[:, :3].T.astype(np.float32))
                tracks.append(arr[:, 3].astype(np.int64))
                pos += len(extra)
        offs[e, L] = pos
    seed_hits = old_to_new[ev.seed_hits].astype(np.int64)
    dup = old_to_new[dup_hits]
    for k, l, e, q in new_ref:
        dup[l, k] = start_of_new[(e, l)] + q
    track_hits = np.where(ev.track_hits >= 0, old_to_new[np.maximum(ev.track_hits, 0)], -1)
    out = EventBatch(
        hits=np.ascontiguousarray(np.concatenate(hits, axis=1)),
        hit_off=offs,
        hit_track=np.concatenate(tracks),
        seed_hits=np.ascontiguousarray(np.concatenate([seed_hits, dup], axis=1).astype(np.int32)),
        seed_event=np.concatenate([ev.seed_event, ev.seed_event[pick]]),
        seed_track=np.concatenate([ev.seed_track, ev.seed_track[pick]]),
        track_event=ev.track_event,
        track_hits=track_hits,
        n_tracks=ev.n_tracks,
    )
    dup_of = np.concatenate([np.full(S, -1, np.int64), pick.astype(np.int64)])
    return out, dup_of
