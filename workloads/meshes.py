"""Seeded mesh and tissue generators.

Every generator returns a plain dict of NumPy arrays and scalars:

  dim            2 or 3
  xyz            (N, dim) float64 vertex coordinates [cm]
  elems          (E, dim+1) int32 simplices (P1 triangles or tetrahedra)
  region         (E,) int8 region code per element (REGION_*)
  region_sigma   (R,) float64 isotropic conductivity of each torso region
                 code [mS/cm]; the heart entry is unused
  fibre          (E, dim, dim) float64 local frame per element, columns are
                 the fibre, sheet (and normal) unit vectors
  sigma_i        (dim,) intracellular conductivities along the frame axes
  sigma_e        (dim,) extracellular conductivities along the frame axes
  chi, cm, dt    membrane surface-to-volume ratio [1/cm], capacitance
                 [uF/cm^2] and time step [ms]
  stim_mask      (N,) uint8, 1 at vertices that receive the stimulus
  stim_amp       stimulus current density [uA/cm^2]
  stim_t0/t1     stimulus window [ms]
  n_steps, tol   run length and relative-residual tolerance of the config

The tissue model follows Sec. 2 of the paper: heart conductivities are
diagonal in a moving fibre frame, the torso is isotropic and piecewise
constant per organ.  Geometry and values are synthetic stand-ins for the
paper's CT thorax slice (Sec. 6.1, 2D test case) and its orthotropic slab
(Sec. 6.1, 3D test case).
"""
import math

import numpy as np

REGION_TORSO = 0
REGION_HEART = 1
REGION_LUNG = 2

_SIG_I_2D = (3.0, 0.31)
_SIG_E_2D = (2.0, 1.35)
_SIG_T = 2.0
_SIG_LUNG = 0.5
_SIG_I_3D = (3.0, 1.0, 0.31)
_SIG_E_3D = (2.0, 1.65, 1.35)


def _frame2d(theta):
    c, s = np.cos(theta), np.sin(theta)
    f = np.empty(theta.shape + (2, 2))
    f[..., 0, 0] = c
    f[..., 1, 0] = s
    f[..., 0, 1] = -s
    f[..., 1, 1] = c
    return f


def _base(dim, xyz, elems, region, region_sigma, fibre, sig_i, sig_e,
          stim_mask, name, n_steps, tol, chi=200.0, cm=1.0, dt=0.1,
          stim_amp=50.0, stim_t0=0.0, stim_t1=2.0):
    return dict(
        name=name, dim=dim,
        xyz=np.ascontiguousarray(xyz, dtype=np.float64),
        elems=np.ascontiguousarray(elems, dtype=np.int32),
        region=np.ascontiguousarray(region, dtype=np.int8),
        region_sigma=np.asarray(region_sigma, dtype=np.float64),
        fibre=np.ascontiguousarray(fibre, dtype=np.float64),
        sigma_i=np.asarray(sig_i, dtype=np.float64),
        sigma_e=np.asarray(sig_e, dtype=np.float64),
        chi=float(chi), cm=float(cm), dt=float(dt),
        stim_mask=np.ascontiguousarray(stim_mask, dtype=np.uint8),
        stim_amp=float(stim_amp), stim_t0=float(stim_t0),
        stim_t1=float(stim_t1), n_steps=int(n_steps), tol=float(tol),
    )


# ---------------------------------------------------------------------------
# 2D square torso with an elliptic heart (small structured case)
# ---------------------------------------------------------------------------
def square2d(n=48, length=10.0, seed=0, semi=(3.0, 2.0), n_steps=20,
             tol=1e-10, stim_radius=0.25):
    """[0,L]^2 split into n x n squares, each cut along the '/' diagonal.

    Heart = elements whose centroid lies inside the ellipse of semi-axes
    `semi` centred in the square; fibres along x.  The stimulus disc centre
    is drawn by the seed inside the ellipse shrunk by 0.5 cm.
    """
    rng = np.random.default_rng(seed)
    h = length / n
    g = np.arange(n + 1) * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    xyz = np.stack([X.ravel(), Y.ravel()], axis=1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i, j = i.ravel(), j.ravel()
    v00 = j * (n + 1) + i
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    # '/' diagonal from (i, j) to (i+1, j+1)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    elems = np.concatenate([t1, t2], axis=0)
    cen = xyz[elems].mean(axis=1)
    c0 = length / 2.0
    a, b = semi
    inside = ((cen[:, 0] - c0) / a) ** 2 + ((cen[:, 1] - c0) / b) ** 2 < 1.0
    region = np.where(inside, REGION_HEART, REGION_TORSO).astype(np.int8)
    fibre = _frame2d(np.zeros(len(elems)))
    # stimulus centre: uniform in the shrunk ellipse (rejection sampling)
    while True:
        p = rng.uniform(-1.0, 1.0, size=2)
        if p[0] ** 2 + p[1] ** 2 < 1.0:
            break
    sc = np.array([c0 + p[0] * (a - 0.5), c0 + p[1] * (b - 0.5)])
    heart_nodes = np.zeros(len(xyz), dtype=bool)
    heart_nodes[elems[inside].ravel()] = True
    d = np.linalg.norm(xyz - sc, axis=1)
    stim = (d <= stim_radius) & heart_nodes
    if not stim.any():  # make sure at least the nearest heart node fires
        dd = np.where(heart_nodes, d, np.inf)
        stim[np.argmin(dd)] = True
    region_sigma = np.array([_SIG_T, 0.0, _SIG_LUNG])
    return _base(2, xyz, elems, region, region_sigma, fibre, _SIG_I_2D,
                 _SIG_E_2D, stim, f"square2d_n{n}", n_steps, tol)


# ---------------------------------------------------------------------------
# 2D thorax-like slice: ellipse torso, two-ventricle heart, two lungs
# ---------------------------------------------------------------------------
_LV_C = np.array([-3.0, 2.0])
_LV_R = (4.0, 5.0)
_RV_C = np.array([-1.5, 2.0])
_RV_R = (5.5, 6.5)


def _heart_geom(p):
    """Return (is_heart, wall_fraction, circumferential unit vector)."""
    dl = p - _LV_C
    rl = np.linalg.norm(dl, axis=1)
    dr = p - _RV_C
    rr = np.linalg.norm(dr, axis=1)
    lv = (rl >= _LV_R[0]) & (rl <= _LV_R[1])
    rv = (rr >= _RV_R[0]) & (rr <= _RV_R[1]) & (rl > _LV_R[1])
    frac = np.where(lv, (rl - _LV_R[0]) / (_LV_R[1] - _LV_R[0]),
                    (rr - _RV_R[0]) / (_RV_R[1] - _RV_R[0]))
    rad = np.where(lv[:, None], dl / np.maximum(rl, 1e-30)[:, None],
                   dr / np.maximum(rr, 1e-30)[:, None])
    circ = np.stack([-rad[:, 1], rad[:, 0]], axis=1)
    return lv | rv, np.clip(frac, 0.0, 1.0), circ


def _ellipse_boundary(a, b, h):
    t = np.linspace(0.0, 2.0 * np.pi, 20001)
    pts = np.stack([a * np.cos(t), b * np.sin(t)], axis=1)
    seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    m = max(8, int(math.ceil(s[-1] / h)))
    target = np.arange(m) * (s[-1] / m)
    tt = np.interp(target, s, t)
    return np.stack([a * np.cos(tt), b * np.sin(tt)], axis=1)


def _in_ellipse(p, c, ax, ang=0.0):
    d = p - c
    ca, sa = np.cos(ang), np.sin(ang)
    x = ca * d[:, 0] + sa * d[:, 1]
    y = -sa * d[:, 0] + ca * d[:, 1]
    return (x / ax[0]) ** 2 + (y / ax[1]) ** 2 < 1.0


def thorax2d(n_target=200_000, seed=1, sigma_scale=1.0, n_steps=500,
             tol=1e-10, semi=(15.0, 10.0), stim_radius=0.25, n_lv_sites=2,
             n_rv_sites=1):
    """Thorax-like slice meshed by Delaunay triangulation of a jittered
    hexagonal lattice (about `n_target` vertices) inside an ellipse.

    Heart: left-ventricle annulus (radii 4-5 cm) plus a right-ventricle
    crescent; fibre angle from the circumferential direction varies linearly
    from -60 to +60 degrees across the wall.  Two seeded lung ellipses with
    conductivity 0.5 mS/cm; the rest of the torso (cavities included) has
    2.0 mS/cm.  `sigma_scale` multiplies every conductivity.  Stimulus discs
    sit on seeded endocardial sites.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    a, b = semi
    h = math.sqrt(2.0 * math.pi * a * b / (math.sqrt(3.0) * n_target))
    dy = h * math.sqrt(3.0) / 2.0
    ny = int(math.ceil(2 * b / dy)) + 1
    nx = int(math.ceil(2 * a / h)) + 2
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = -a + ii * h + (jj % 2) * 0.5 * h
    y = -b + jj * dy
    p = np.stack([x.ravel(), y.ravel()], axis=1)
    p += rng.uniform(-0.3 * h, 0.3 * h, size=p.shape)
    keep = ((p[:, 0] / (a - 0.5 * h)) ** 2 + (p[:, 1] / (b - 0.5 * h)) ** 2) < 1.0
    p = p[keep]
    bnd = _ellipse_boundary(a, b, h)
    xyz = np.concatenate([p, bnd], axis=0)
    tri = Delaunay(xyz)
    elems = tri.simplices.astype(np.int64)
    # drop degenerate slivers that qhull may leave on the hull
    e = xyz[elems]
    area = 0.5 * np.abs((e[:, 1, 0] - e[:, 0, 0]) * (e[:, 2, 1] - e[:, 0, 1])
                        - (e[:, 2, 0] - e[:, 0, 0]) * (e[:, 1, 1] - e[:, 0, 1]))
    elems = elems[area > 1e-6 * h * h]
    used = np.zeros(len(xyz), dtype=bool)
    used[elems.ravel()] = True
    remap = -np.ones(len(xyz), dtype=np.int64)
    remap[used] = np.arange(used.sum())
    xyz = xyz[used]
    elems = remap[elems]

    cen = xyz[elems].mean(axis=1)
    is_heart, frac, circ = _heart_geom(cen)

    # two lungs, redrawn until inside the torso and clear of the heart
    lungs = []
    probe = np.stack(np.meshgrid(np.linspace(-a, a, 241),
                                 np.linspace(-b, b, 161)), -1).reshape(-1, 2)
    probe_heart, _, _ = _heart_geom(probe)
    probe_torso = (probe[:, 0] / (0.97 * a)) ** 2 + (probe[:, 1] / (0.97 * b)) ** 2 < 1
    for cx0, cy0, ax0, ay0 in ((-11.0, -1.5, 2.0, 3.5), (9.0, -1.0, 2.5, 4.0)):
        for _ in range(200):
            c = np.array([cx0 + rng.uniform(-0.5, 0.5), cy0 + rng.uniform(-0.5, 0.5)])
            ax = (ax0 + rng.uniform(0.0, 0.5), ay0 + rng.uniform(0.0, 0.5))
            ang = rng.uniform(-0.2, 0.2)
            inl = _in_ellipse(probe, c, (ax[0] + 0.3, ax[1] + 0.3), ang)
            inl_core = _in_ellipse(probe, c, ax, ang)
            if not (inl & probe_heart).any() and not (inl_core & ~probe_torso).any():
                lungs.append((c, ax, ang))
                break
        else:
            raise RuntimeError("could not place a lung")
    region = np.full(len(elems), REGION_TORSO, dtype=np.int8)
    for c, ax, ang in lungs:
        region[_in_ellipse(cen, c, ax, ang)] = REGION_LUNG
    region[is_heart] = REGION_HEART

    theta = np.deg2rad(-60.0 + 120.0 * frac)
    rad = np.stack([circ[:, 1], -circ[:, 0]], axis=1)
    f = np.cos(theta)[:, None] * circ + np.sin(theta)[:, None] * rad
    s = np.stack([-f[:, 1], f[:, 0]], axis=1)
    fibre = np.stack([f, s], axis=2)
    fibre[~is_heart] = np.eye(2)

    heart_nodes = np.zeros(len(xyz), dtype=bool)
    heart_nodes[elems[is_heart].ravel()] = True
    stim = np.zeros(len(xyz), dtype=bool)
    sites = []
    for _ in range(n_lv_sites):
        t = rng.uniform(0.0, 2.0 * np.pi)
        sites.append(_LV_C + (_LV_R[0] + 0.25) * np.array([np.cos(t), np.sin(t)]))
    for _ in range(n_rv_sites):
        t = rng.uniform(-np.pi / 3.0, np.pi / 3.0)
        sites.append(_RV_C + (_RV_R[0] + 0.25) * np.array([np.cos(t), np.sin(t)]))
    for sc in sites:
        d = np.linalg.norm(xyz - sc, axis=1)
        hit = (d <= stim_radius) & heart_nodes
        if not hit.any():
            hit[np.argmin(np.where(heart_nodes, d, np.inf))] = True
        stim |= hit
    region_sigma = np.array([_SIG_T, 0.0, _SIG_LUNG]) * sigma_scale
    out = _base(2, xyz, elems, region, region_sigma, fibre,
                np.array(_SIG_I_2D) * sigma_scale,
                np.array(_SIG_E_2D) * sigma_scale, stim,
                f"thorax2d_{len(xyz)}", n_steps, tol)
    out["mesh_h"] = h
    # six body-surface electrodes (the ECG leads of the 2D test case): the
    # mesh vertices nearest to the torso boundary at these angles, from the
    # top of the slice round the side the heart lies on
    used = xyz[np.unique(elems)]
    ang = np.deg2rad([80.0, 100.0, 120.0, 140.0, 160.0, 180.0])
    tgt = np.stack([a * np.cos(ang), b * np.sin(ang)], axis=1)
    out["electrodes"] = np.array([used[np.argmin(np.linalg.norm(used - t, axis=1))] for t in tgt])
    return out


# ---------------------------------------------------------------------------
# 3D orthotropic slab, isolated heart
# ---------------------------------------------------------------------------
def slab3d(n=64, length=1.0, n_steps=200, tol=1e-10, stim_radius=0.15,
           seed=2):
    """[0,L]^3 with n^3 hexahedra, each cut into 6 Kuhn tetrahedra along the
    (1,1,1) diagonal.  Isolated heart (every element is heart).  Fibres are
    horizontal and rotate from -60 to +60 degrees as z goes from 0 to L,
    sheet direction in-plane, normal along z.  Corner stimulus: vertices
    within `stim_radius` of the origin.
    """
    del seed  # the slab has no random parts; kept for a uniform signature
    h = length / n
    g = np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    m = n + 1
    step = np.array([1, m, m * m], dtype=np.int64)
    v0 = i + m * j + m * m * k
    v3 = v0 + step.sum()
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        tets.append(np.stack([v0, v1, v2, v3], axis=1))
    elems = np.concatenate(tets, axis=0)
    cen_z = xyz[elems][:, :, 2].mean(axis=1)
    theta = np.deg2rad(-60.0 + 120.0 * cen_z / length)
    c, s = np.cos(theta), np.sin(theta)
    fibre = np.zeros((len(elems), 3, 3))
    fibre[:, 0, 0] = c
    fibre[:, 1, 0] = s
    fibre[:, 0, 1] = -s
    fibre[:, 1, 1] = c
    fibre[:, 2, 2] = 1.0
    region = np.full(len(elems), REGION_HEART, dtype=np.int8)
    stim = np.linalg.norm(xyz, axis=1) <= stim_radius + 1e-12
    region_sigma = np.array([_SIG_T, 0.0, _SIG_LUNG])
    return _base(3, xyz, elems, region, region_sigma, fibre, _SIG_I_3D,
                 _SIG_E_3D, stim, f"slab3d_n{n}", n_steps, tol)


# ---------------------------------------------------------------------------
# named configurations
# ---------------------------------------------------------------------------
def _config4(seed=4, n_slices=64, lo=20_000, hi=300_000, n_steps=100):
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_slices))).astype(int)
    scales = rng.uniform(0.7, 1.3, n_slices)
    return [dict(n_target=int(sz), seed=1000 + s, sigma_scale=float(sc),
                 n_steps=n_steps) for s, (sz, sc) in enumerate(zip(sizes, scales))]


_CONFIGS = {
    "square48": lambda seed: square2d(n=48, seed=0 if seed is None else seed),
    "thorax200k": lambda seed: thorax2d(200_000, seed=1 if seed is None else seed),
    "slab64": lambda seed: slab3d(n=64, n_steps=200),
    "slab128": lambda seed: slab3d(n=128, n_steps=200),
}


def config_names():
    return ["square48", "thorax200k", "slab64", "slab128", "batch64"]


def make_config(name, seed=None):
    """Build a named workload.  `batch64` returns the list of per-slice
    generator arguments (call thorax2d(**kw) on each) rather than meshes."""
    if name == "batch64":
        return _config4(seed=4 if seed is None else seed)
    return _CONFIGS[name](seed)


def summary(cfg):
    heart = cfg["region"] == REGION_HEART
    hn = np.unique(cfg["elems"][heart].ravel())
    return dict(name=cfg["name"], dim=cfg["dim"], n_nodes=len(cfg["xyz"]),
                n_elems=len(cfg["elems"]), n_heart_elems=int(heart.sum()),
                n_heart_nodes=int(len(hn)), n_stim=int(cfg["stim_mask"].sum()))
