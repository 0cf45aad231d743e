"""Seeded synthetic Gamma Knife planning cases.

This module is the one input generator shared by the oracle, the tests and the
benchmark.  It draws geometry, isocentres and dose-rate kernels and returns the
raw material of a planning problem: the dose-influence matrix phi (dose points
x shot columns), the point-group table, and the slider weights of each plan.
It holds none of the planning method's arithmetic: no LP assembly, no scaling,
no step of the solver.  Everything is deterministic in the seed.

Geometry follows the description of the clinical inputs in the paper (Sec. 2.A
and Sec. 3.B): dose points are taken from the target surface and interior, a
ring just outside each target, a low-dose region further out, and OAR surfaces;
isocentres are placed inside the targets.  The clinical cases themselves are
not available, so the shapes and sizes below are synthetic stand-ins.

Column layout of phi: column j = (i * n_sectors + s) * n_collimators + c for
isocentre i, sector s and collimator c (collimator fastest), which matches the
Kronecker structure C = I (x) I_8 (x) 1_{1x3} of App. A.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

# Point-group types (App. A: TS, TI, R, LD, O).
TS, TI, RING, LD, OAR = 0, 1, 2, 3, 4
TYPE_NAMES = {TS: "TS", TI: "TI", RING: "R", LD: "LD", OAR: "O"}


@dataclasses.dataclass
class Group:
    """One block of dose points with its own threshold dose and weight share."""
    type: int            # TS / TI / RING / LD / OAR
    structure: int       # target index (TS/TI/RING), LD level, or OAR index
    threshold: float     # D_alpha in Gy (D_O for an OAR)
    share: float         # q_kA (TS), q_kV (TI), 1/n_targets (RING), 1 (LD, OAR)


@dataclasses.dataclass
class KernelModel:
    """Parameters of the Gaussian-sum dose-rate kernels of every shot column."""
    iso: np.ndarray          # (n_iso, 3) isocentre positions in mm
    sector_factor: np.ndarray  # (n_iso, n_sectors) per-sector output factor
    fwhm: np.ndarray         # (n_collimators,) mm
    output_factor: np.ndarray  # (n_collimators,) relative output
    sector_dir: np.ndarray   # (n_sectors, 3) unit vectors
    phi_cal: float           # calibration dose rate, Gy/min
    offset_frac: float       # centre offset along the sector direction, x FWHM

    @property
    def n_iso(self):
        return self.iso.shape[0]

    @property
    def n_sectors(self):
        return self.sector_dir.shape[0]

    @property
    def n_collimators(self):
        return self.fwhm.shape[0]

    def dose_rate(self, pos_mm: np.ndarray, dtype=np.float64, chunk: int = 65536):
        """Dose rate of every shot column at the given points (M x n_t)."""
        pos_mm = np.asarray(pos_mm, dtype=np.float64)
        m = pos_mm.shape[0]
        S, C = self.n_sectors, self.n_collimators
        n_t = self.n_iso * S * C
        out = np.empty((m, n_t), dtype=dtype)
        sig1 = self.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
        sig3 = 3.0 * sig1
        for r0 in range(0, m, chunk):
            p = pos_mm[r0:r0 + chunk]
            for i in range(self.n_iso):
                rel = p - self.iso[i]                            # (mc, 3)
                r2 = np.einsum("md,md->m", rel, rel)             # (mc,)
                blk = np.empty((p.shape[0], S, C), dtype=np.float64)
                for s in range(S):
                    proj = rel @ self.sector_dir[s]              # (mc,)
                    for c in range(C):
                        off = self.offset_frac * self.fwhm[c]
                        d2 = r2 - 2.0 * off * proj + off * off   # |x - iso - off*dir|^2
                        g = (0.9 * np.exp(-d2 / (2.0 * sig1[c] ** 2))
                             + 0.1 * np.exp(-d2 / (2.0 * sig3[c] ** 2)))
                        amp = (self.sector_factor[i, s] * (self.phi_cal / S)
                               * self.output_factor[c])
                        blk[:, s, c] = amp * g
                out[r0:r0 + chunk, i * S * C:(i + 1) * S * C] = blk.reshape(p.shape[0], S * C)
        return out


@dataclasses.dataclass
class Case:
    """A synthetic planning case: dose points, groups and the dose matrix phi."""
    name: str
    dose: np.ndarray          # (N, n_t) phi, entries >= 0, row-major
    group: np.ndarray         # (N,) int32 index into groups
    groups: list              # list[Group]
    coords: np.ndarray        # (N, 3) int32 voxel indices of the dose points
    kernel: KernelModel
    prescription_mean: float  # D_T (mean over targets)
    grid_shape: tuple         # voxel grid (mm spacing = 1)
    target_mask: np.ndarray   # bool grid, any target
    ld_candidates: np.ndarray  # (M, 3) int32 voxels eligible for low-dose points
    seed: int

    @property
    def n_points(self):
        return self.dose.shape[0]

    @property
    def n_iso(self):
        return self.kernel.n_iso

    @property
    def n_sectors(self):
        return self.kernel.n_sectors

    @property
    def n_collimators(self):
        return self.kernel.n_collimators

    @property
    def n_t(self):
        return self.dose.shape[1]

    @property
    def phi_cal(self):
        return self.kernel.phi_cal

    def group_counts(self):
        return np.bincount(self.group, minlength=len(self.groups))

    def point_types(self):
        return np.array([g.type for g in self.groups], dtype=np.int32)[self.group]

    def with_points(self, keep: np.ndarray, extra_ld=None, ld_group=None, name=None, extra=None):
        """A copy that keeps rows `keep` and appends low-dose points `extra_ld`.

        `extra_ld` are voxel coordinates; their dose rows are evaluated from the
        same kernel model, and they join group `ld_group`.  `extra` is a list of
        such (coordinates, group) pairs appended in order after `extra_ld`.
        Used to build the second-pass case once its low-dose point sets are
        known.
        """
        keep = np.asarray(keep)
        dose = self.dose[keep]
        group = self.group[keep]
        coords = self.coords[keep]
        parts = [] if extra_ld is None else [(extra_ld, ld_group)]
        parts += list(extra or [])
        for pts, g in parts:
            if pts is None or not len(pts):
                continue
            pts = np.asarray(pts, dtype=np.int32)
            dose = np.concatenate([dose, self.kernel.dose_rate(pts, dtype=self.dose.dtype)])
            group = np.concatenate([group, np.full(len(pts), g, np.int32)])
            coords = np.concatenate([coords, pts])
        return dataclasses.replace(self, dose=np.ascontiguousarray(dose), group=group,
                                   coords=coords, name=name or self.name + "+pass2")


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------

def _ellipsoid_mask(shape, center, radii):
    zz, yy, xx = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in shape), indexing="ij")
    q = (((zz - center[0]) / radii[0]) ** 2 + ((yy - center[1]) / radii[1]) ** 2
         + ((xx - center[2]) / radii[2]) ** 2)
    return q <= 1.0


def _surface(mask):
    """Voxels of `mask` with at least one 6-neighbour outside it."""
    inner = ndimage.binary_erosion(mask, structure=ndimage.generate_binary_structure(3, 1),
                                   border_value=0)
    return mask & ~inner


def _kmeans_iso(points, n, rng, iters=12):
    """Spread n isocentres over a target's voxels (k-means++ then Lloyd steps)."""
    pts = points.astype(np.float64)
    if n >= len(pts):
        return pts[:n].copy()
    centers = [pts[rng.integers(len(pts))]]
    d2 = np.sum((pts - centers[0]) ** 2, axis=1)
    for _ in range(1, n):
        prob = d2 / d2.sum()
        centers.append(pts[rng.choice(len(pts), p=prob)])
        d2 = np.minimum(d2, np.sum((pts - centers[-1]) ** 2, axis=1))
    centers = np.array(centers)
    for _ in range(iters):
        lab = np.argmin(((pts[:, None, :] - centers[None, :, :]) ** 2).sum(-1), axis=1)
        for c in range(n):
            sel = pts[lab == c]
            if len(sel):
                centers[c] = sel.mean(0)
    # snap to the nearest target voxel so every isocentre lies inside the target
    idx = np.argmin(((pts[:, None, :] - centers[None, :, :]) ** 2).sum(-1), axis=0)
    return pts[idx] + rng.uniform(-0.25, 0.25, size=(n, 3))


def _sector_dirs(n_sectors):
    """Unit vectors of the sectors, spread around the beam axis with a tilt."""
    ang = 2.0 * np.pi * (np.arange(n_sectors) + 0.5) / n_sectors
    tilt = 0.35
    d = np.stack([np.full(n_sectors, math.sin(tilt)), np.cos(ang) * math.cos(tilt),
                  np.sin(ang) * math.cos(tilt)], axis=1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# case construction
# ---------------------------------------------------------------------------

def build_case(spec: dict, seed: int, dtype=np.float64) -> Case:
    """Build a case from a geometric spec (see CONFIGS for examples).

    spec keys:
      grid        : (nz, ny, nx) voxel grid, 1 mm spacing
      targets     : list of (center_zyx, radii_zyx, prescription_Gy)
      n_ring      : number of ring points (all targets together)
      ring_mm     : initial ring thickness; grown until n_ring voxels exist
      n_ld        : number of first-pass low-dose points
      ld_region   : ("cube", edge_mm) around the grid centre, or ("shell", r_out_mm)
                    beyond the ring
      ld_fraction : D_LD / D_T,mean
      ld_levels   : optional list of D_LD / D_T,mean, one low-dose group per level
                    (App. A uses two thresholds); n_ld points are drawn for each
      n_iso       : isocentres (split over targets by volume^(2/3))
      oars        : list of (center_zyx, radii_zyx, max_dose_Gy, n_points)
      sectors, collimators, fwhm, output_factor, phi_cal, offset_frac
    """
    rng = np.random.default_rng(seed)
    shape = tuple(spec["grid"])
    targets = spec["targets"]
    n_tg = len(targets)
    tmasks = [_ellipsoid_mask(shape, c, r) for c, r, _ in targets]
    any_t = np.zeros(shape, bool)
    for m in tmasks:
        any_t |= m
    # a voxel shared by two targets belongs to the first
    owned = []
    taken = np.zeros(shape, bool)
    for m in tmasks:
        owned.append(m & ~taken)
        taken |= m
    surf = [_surface(m) & o for m, o in zip(tmasks, owned)]
    inter = [o & ~s for o, s in zip(owned, surf)]
    area = np.array([s.sum() for s in surf], np.float64)
    vol = np.array([o.sum() for o in owned], np.float64)

    # distance from each voxel to the nearest target voxel, and which target
    dist, inds = ndimage.distance_transform_edt(~any_t, return_indices=True)
    label = np.full(shape, -1, np.int32)
    for k, o in enumerate(owned):
        label[o] = k
    nearest = label[inds[0], inds[1], inds[2]]

    # ring: grow the thickness until enough voxels exist, then subsample
    n_ring = int(spec["n_ring"])
    ring_mm = float(spec.get("ring_mm", 3.0))
    oar_mask = np.zeros(shape, bool)
    for (c, r, _, _) in spec.get("oars", []):
        oar_mask |= _ellipsoid_mask(shape, c, r)
    while True:
        ring = (~any_t) & (dist <= ring_mm) & ~oar_mask
        if ring.sum() >= n_ring or ring_mm > min(shape) / 2:
            break
        ring_mm += 1.0
    ring_vox = np.argwhere(ring)
    if len(ring_vox) > n_ring:
        ring_vox = ring_vox[np.sort(rng.choice(len(ring_vox), n_ring, replace=False))]

    # first-pass low-dose candidates and points
    region = spec["ld_region"]
    outside = (~any_t) & (dist > ring_mm) & ~oar_mask
    if region[0] == "cube":
        half = region[1] / 2.0
        ctr = np.array(shape, np.float64) / 2.0
        zz, yy, xx = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
        box = ((np.abs(zz - ctr[0]) <= half) & (np.abs(yy - ctr[1]) <= half)
               & (np.abs(xx - ctr[2]) <= half))
        ld_cand = outside & box
    else:
        ld_cand = outside & (dist <= ring_mm + region[1])
    ld_cand_vox = np.argwhere(ld_cand).astype(np.int32)
    n_ld = int(spec["n_ld"])
    levels = list(spec.get("ld_levels", [spec.get("ld_fraction", 0.5)]))
    ld_sets = [ld_cand_vox[np.sort(rng.choice(len(ld_cand_vox), n_ld, replace=False))]
               for _ in levels]

    # groups and points, in the block order of App. A: TS_k, TI_k, R_k, LD, O_m
    groups, coords, gid = [], [], []
    presc = np.array([p for _, _, p in targets], np.float64)
    d_mean = float(presc.mean())
    for k in range(n_tg):
        groups.append(Group(TS, k, float(presc[k]), float(area[k] / area.sum())))
        coords.append(np.argwhere(surf[k])); gid.append(len(groups) - 1)
    for k in range(n_tg):
        groups.append(Group(TI, k, float(presc[k]), float(vol[k] / vol.sum())))
        coords.append(np.argwhere(inter[k])); gid.append(len(groups) - 1)
    ring_owner = nearest[ring_vox[:, 0], ring_vox[:, 1], ring_vox[:, 2]]
    for k in range(n_tg):
        groups.append(Group(RING, k, float(presc[k]), 1.0 / n_tg))
        coords.append(ring_vox[ring_owner == k]); gid.append(len(groups) - 1)
    for lvl, (frac, ld_vox) in enumerate(zip(levels, ld_sets)):
        groups.append(Group(LD, lvl, float(frac) * d_mean, 1.0))
        coords.append(ld_vox); gid.append(len(groups) - 1)
    for m, (c, r, dmax, npts) in enumerate(spec.get("oars", [])):
        om = _surface(_ellipsoid_mask(shape, c, r))
        ov = np.argwhere(om)
        if len(ov) > npts:
            ov = ov[np.sort(rng.choice(len(ov), npts, replace=False))]
        groups.append(Group(OAR, m, float(dmax), 1.0))
        coords.append(ov); gid.append(len(groups) - 1)

    pts = np.concatenate(coords).astype(np.int32)
    group = np.concatenate([np.full(len(c), g, np.int32) for c, g in zip(coords, gid)])

    # isocentres per target, proportional to volume^(2/3), at least one each
    n_iso = int(spec["n_iso"])
    share = vol ** (2.0 / 3.0)
    alloc = np.maximum(1, np.floor(n_iso * share / share.sum()).astype(int))
    while alloc.sum() < n_iso:
        alloc[np.argmax(n_iso * share / share.sum() - alloc)] += 1
    while alloc.sum() > n_iso:
        alloc[np.argmax(alloc)] -= 1
    isos = np.concatenate([_kmeans_iso(np.argwhere(owned[k]), int(alloc[k]), rng)
                           for k in range(n_tg)])

    S = int(spec.get("sectors", 8))
    C = int(spec.get("collimators", 3))
    fwhm = np.asarray(spec.get("fwhm", (4.0, 8.0, 16.0))[:C], np.float64)
    of = np.asarray(spec.get("output_factor", (0.81, 0.90, 1.0))[:C], np.float64)
    kern = KernelModel(iso=isos, sector_factor=rng.uniform(0.8, 1.2, size=(n_iso, S)),
                       fwhm=fwhm, output_factor=of, sector_dir=_sector_dirs(S),
                       phi_cal=float(spec.get("phi_cal", 3.0)),
                       offset_frac=float(spec.get("offset_frac", 0.05)))
    dose = kern.dose_rate(pts, dtype=dtype)
    return Case(name=spec.get("name", "case"), dose=dose, group=group, groups=groups,
                coords=pts, kernel=kern, prescription_mean=d_mean, grid_shape=shape,
                target_mask=any_t, ld_candidates=ld_cand_vox, seed=seed)


def _spread_targets(radii, grid, rng, gap=6.0):
    """Place ellipsoids without overlap inside the grid (seeded rejection)."""
    centers = []
    margin = 14.0
    for r in radii:
        for _ in range(10000):
            c = np.array([rng.uniform(margin + r[i], grid[i] - margin - r[i]) for i in range(3)])
            ok = all(np.linalg.norm(c - c2) > max(r) + max(r2) + gap
                     for c2, r2 in zip(centers, radii))
            if ok:
                centers.append(c)
                break
        else:
            raise RuntimeError("could not place targets")
    return centers


# ---------------------------------------------------------------------------
# the configurations of the workload (sizes of the paper's largest and
# smallest problems, Table 1, extended to the batch sizes of Sec. 3.E)
# ---------------------------------------------------------------------------

def config_spec(config: int) -> dict:
    """Geometric spec of the named configurations.

    0: one sphere r=6 mm, 3 mm ring subsampled to 1,000 points, 500 LD points
       in a 30 mm cube, 8 isocentres -> N ~ 2,400, n_t = 192.
    1: three targets r 5-12 mm (~10 cm^3), 5,000 LD points, 60 isocentres ->
       N = 40,000, n_t = 1,440.
    2: nine targets r 3-18 mm (~52 cm^3), 200 isocentres -> N = 200,000,
       n_t = 4,800.
    """
    if config == 0:
        return dict(name="c0-sphere6-2400x192", grid=(40, 40, 40),
                    targets=[((19.5, 19.5, 19.5), (6.0, 6.0, 6.0), 20.0)],
                    n_ring=1000, ring_mm=3.0, n_ld=500, ld_region=("cube", 30.0),
                    n_iso=8)
    if config == 1:
        rng = np.random.default_rng(101)
        radii = [(12.0, 10.0, 9.0), (8.0, 8.0, 8.0), (6.0, 5.0, 5.5)]
        grid = (96, 96, 96)
        centers = _spread_targets(radii, grid, rng)
        tg = [(tuple(c), r, 20.0) for c, r in zip(centers, radii)]
        n_target = sum(_ellipsoid_mask(grid, c, r).sum() for c, r, _ in tg)
        return dict(name="c1-3targets-40000x1440", grid=grid, targets=tg,
                    n_ring=40000 - 5000 - int(n_target), ring_mm=3.0, n_ld=5000,
                    ld_region=("shell", 12.0), n_iso=60)
    if config == 2:
        rng = np.random.default_rng(202)
        base = [18.0, 14.0, 11.5, 9.5, 8.0, 6.5, 5.0, 4.0, 3.0]
        radii = [(r, r * 0.95, r * 1.05) for r in base]
        grid = (160, 160, 160)
        centers = _spread_targets(radii, grid, rng, gap=4.0)
        tg = [(tuple(c), r, 20.0) for c, r in zip(centers, radii)]
        n_target = sum(_ellipsoid_mask(grid, c, r).sum() for c, r, _ in tg)
        return dict(name="c2-9targets-200000x4800", grid=grid, targets=tg,
                    n_ring=200000 - 20000 - int(n_target), ring_mm=3.0, n_ld=20000,
                    ld_region=("shell", 14.0), n_iso=200)
    raise ValueError(f"unknown config {config}")


def uneven_spec(seed: int) -> dict:
    """A case of the uneven multi-case workload: one u ~ U[0, 1] per seed sets
    the size between the small and the large configuration on a log scale,
    N = 2,400 (200,000 / 2,400)^u points and n_iso = round(8 * 25^u)
    isocentres (real N and n_iso grow together); 1 + round(8 u) targets share
    a target volume of 900 (52,000 / 900)^u voxels; a tenth of the points are
    low-dose points, the rest ring points."""
    rng = np.random.default_rng(seed)
    u = float(rng.uniform())
    n_total = int(round(2400 * (200000 / 2400) ** u))
    n_iso = max(1, int(round(8 * 25 ** u)))
    n_tg = 1 + int(round(8 * u))
    vol = 900.0 * (52000.0 / 900.0) ** u
    share = rng.uniform(0.5, 1.5, size=n_tg)
    share /= share.sum()
    radii = [tuple(float(x) for x in (3.0 * vol * s / (4.0 * np.pi)) ** (1.0 / 3.0)
                   * rng.uniform(0.9, 1.1, size=3)) for s in share]
    side = int(48 + 120 * u)
    for _ in range(20):
        try:
            centers = _spread_targets(radii, (side, side, side), rng, gap=4.0)
            break
        except RuntimeError:
            side += 16
    tg = [(tuple(c), r, 20.0) for c, r in zip(centers, radii)]
    n_target = sum(int(_ellipsoid_mask((side,) * 3, c, r).sum()) for c, r, _ in tg)
    n_ld = max(500, n_total // 10)
    return dict(name=f"uneven-{seed}-u{u:.3f}", grid=(side,) * 3, targets=tg,
                n_ring=max(200, n_total - n_target - n_ld), ring_mm=3.0, n_ld=n_ld,
                ld_region=("shell", 10.0 + 5.0 * u), n_iso=n_iso)


def uneven_case(seed: int, dtype=np.float64) -> Case:
    """The seeded case of the uneven multi-case and serving workloads."""
    return build_case(uneven_spec(seed), seed, dtype=dtype)


CONFIG_SEEDS = {0: 0, 1: 1, 2: 2}
CONFIG_PLANS = {0: 3, 1: 9, 2: 21}   # slider grid edge g; plans k = g * g


def make_case(config: int, seed=None, dtype=np.float64) -> Case:
    """The seeded synthetic case of a configuration."""
    return build_case(config_spec(config), CONFIG_SEEDS[config] if seed is None else seed,
                      dtype=dtype)


def mini_spec(n_iso=1, sectors=2, collimators=1, radius=2.0, n_ring=6, n_ld=4, oar=False):
    """Tiny cases whose LP is small enough for brute-force checks."""
    spec = dict(name=f"mini-{n_iso}x{sectors}x{collimators}", grid=(16, 16, 16),
                targets=[((7.5, 7.5, 7.5), (radius, radius, radius), 20.0)],
                n_ring=n_ring, ring_mm=1.5, n_ld=n_ld, ld_region=("shell", 4.0),
                n_iso=n_iso, sectors=sectors, collimators=collimators,
                fwhm=(4.0, 8.0, 16.0), output_factor=(0.81, 0.90, 1.0))
    if oar:
        spec["oars"] = [((7.5, 7.5, 13.0), (1.5, 1.5, 1.5), 8.0, 4)]
    return spec


# ---------------------------------------------------------------------------
# plan weights (slider grid)
# ---------------------------------------------------------------------------

W0_BOT = 1e-3     # weight of the BOT term at s_BOT = 0 (lowest allowed)
W1_BOT = 1.0      # weight of the BOT term at s_BOT = 1


def slider_grid(g: int):
    """All g x g combinations of the low-dose and BOT sliders in [0, 1]."""
    s = np.linspace(0.0, 1.0, g)
    s_ld, s_bot = np.meshgrid(s, s, indexing="ij")
    return s_ld.ravel(), s_bot.ravel()


def slider_weights(s_ld, s_bot, w0_bot=W0_BOT, w1_bot=W1_BOT):
    """Primal weights (w_T, w_R, w_LD, w_BOT) of each plan, one row per plan.

    The clinical slider-to-weight map is not published; this one keeps
    w_T = w_R = 1, takes w_LD = s_LD and spaces w_BOT logarithmically between
    w0_bot and w1_bot so that w_BOT > 0 always holds.
    """
    s_ld = np.atleast_1d(np.asarray(s_ld, np.float64))
    s_bot = np.atleast_1d(np.asarray(s_bot, np.float64))
    w = np.empty((s_ld.size, 4), np.float64)
    w[:, 0] = 1.0
    w[:, 1] = 1.0
    w[:, 2] = s_ld
    w[:, 3] = w0_bot * (w1_bot / w0_bot) ** s_bot
    return w


def config_weights(config: int):
    g = CONFIG_PLANS[config]
    return slider_weights(*slider_grid(g))


def random_weights(k: int, seed: int):
    """k weight vectors from uniformly drawn slider positions."""
    rng = np.random.default_rng(seed)
    return slider_weights(rng.uniform(0, 1, k), rng.uniform(0, 1, k))


# ---------------------------------------------------------------------------
# bitsets of voxel sets (input format of the low-dose point selection)
# ---------------------------------------------------------------------------

def random_volumes(k: int, n_vox: int, seed: int, kind="shells"):
    """k boolean volumes over n_vox voxels with overlapping, graded structure.

    'shells': voxels are ranked on a line and volume j is a window whose start
    and width drift with j, so neighbouring volumes overlap heavily, as the
    low-dose bands of nearby weightings do.  'random': independent Bernoulli.
    """
    rng = np.random.default_rng(seed)
    vols = np.zeros((k, n_vox), bool)
    if kind == "random":
        for j in range(k):
            vols[j] = rng.random(n_vox) < rng.uniform(0.05, 0.6)
        return vols
    order = rng.permutation(n_vox)
    for j in range(k):
        a = int(rng.uniform(0.0, 0.5) * n_vox)
        w = int(rng.uniform(0.1, 0.5) * n_vox)
        sel = order[a:a + w]
        vols[j, sel] = True
        # ragged edges
        flip = rng.random(n_vox) < 0.02
        vols[j] ^= flip
    return vols


def pack_bits(vols: np.ndarray) -> np.ndarray:
    """(k, n) bool -> (k, ceil(n/64)) uint64, bit b of word w = voxel 64*w + b."""
    k, n = vols.shape
    nw = (n + 63) // 64
    padded = np.zeros((k, nw * 64), bool)
    padded[:, :n] = vols
    by = np.packbits(padded.reshape(k, nw, 64)[:, :, ::-1], axis=2)  # big-endian bytes
    out = np.zeros((k, nw), np.uint64)
    for b in range(8):
        out |= by[:, :, b].astype(np.uint64) << np.uint64(8 * (7 - b))
    return out


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    words = np.asarray(words, np.uint64)
    k, nw = words.shape
    bits = ((words[:, :, None] >> np.arange(64, dtype=np.uint64)[None, None, :]) & np.uint64(1))
    return bits.reshape(k, nw * 64)[:, :n].astype(bool)
