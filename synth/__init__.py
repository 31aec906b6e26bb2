"""Seeded synthetic orthogonal-raster OCT/OCTA scan pairs.

This module only makes inputs: it holds none of the registration method's
arithmetic and is shared by the tests, the benchmark and the smoke check.  The
clinical data of the paper are not available, so retina-shaped volumes of the
paper's workload shapes stand in for them (Sec. 3.3 describes 500 x 500 A-scan
raster scans, X-fast and Y-fast, with OCTA from amplitude decorrelation).

Recipe (all draws from numpy.random.SeedSequence([20100693100 + k, p]), k the
workload index, p the pair index, spawned into phantom / vessel / motion-X /
motion-Y streams; the large noise fields use torch generators seeded from the
phantom stream, so they depend on the device the pair is generated on):

  structure  six smooth layer boundaries z_b = d (c_b + P_b(u, v)) with
             quadratic P_b, seven layers of fixed mean reflectivity joined by
             logistic edges, multiplied by log-normal speckle
             exp(0.5 n - 0.125), n smoothed unit-variance Gaussian noise; the
             truth's 99th percentile is scaled to 1.
  vessels    a random branching tree of persistent random walks drawn in the
             en face plane, blurred (sigma 1 px), confined in depth to the slab
             between boundaries 1 and 3; Rayleigh noise (scale 0.1) per scan.
  motion     per scan a 3-D random walk over acquisition time (one step per
             A-scan period, including round(0.25 n) flyback periods per
             B-scan) plus saccade jumps at uniform random times.
  sampling   scan V's volume at output voxel q is the truth at q + m(t_V(q)),
             trilinear from a truth grid twice as fine as the scans (not the
             registration's cubic interpolator); the ground-truth pull field
             solves d = -m(p + d) (m interpolated between A-scans) and is
             centred so that the mean over both scans is zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch
import torch.nn.functional as F

SEED_BASE = 20100693100

# Workloads (shapes of the paper's scans and of the benchmark variants).
WORKLOADS = {
    # 64^2 A-scans x 128 samples, drift 0.05 px/A-scan, 2 saccades <= 3 px
    "tiny": dict(index=0, n=64, d=128, drift=0.05, saccades=(2, 2), amp=3.0, levels=3),
    # 300^2 x 640, drift 0.03, 5-10 saccades <= 8 px
    "clinical": dict(index=1, n=300, d=640, drift=0.03, saccades=(5, 10), amp=8.0, levels=4),
    # 500^2 x 800 dense / wide field, 15 saccades
    "dense": dict(index=2, n=500, d=800, drift=0.03, saccades=(15, 15), amp=8.0, levels=4),
    # batch of 200^2 x 512 pairs
    "batch": dict(index=3, n=200, d=512, drift=0.03, saccades=(5, 10), amp=8.0, levels=3),
    # serving requests (size drawn per request)
    "serving": dict(index=4, n=300, d=512, drift=0.03, saccades=(5, 10), amp=8.0, levels=4),
}

LAYER_C = (0.30, 0.36, 0.45, 0.55, 0.62, 0.70)
LAYER_R = (0.02, 0.9, 0.4, 0.7, 0.3, 1.0, 0.5)


@dataclass
class Pair:
    """One orthogonal scan pair.  Volumes are [h][w][d] (row j, column i,
    depth k) float32 in the common (x, y) frame; en face images [h][w];
    validity vx[h] (X-fast B-scans are rows) and vy[w] (Y-fast B-scans are
    columns); d_gt is [2][h][w][3] float64 (V, j, i, (dx, dy, dz))."""

    sx: torch.Tensor
    sy: torch.Tensor
    ax: torch.Tensor
    ay: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    d_gt: torch.Tensor
    ox: torch.Tensor | None = None
    oy: torch.Tensor | None = None
    saccade_ij: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        h, w, d = self.sx.shape
        return w, h, d


def _rng_streams(index: int, pair: int):
    ss = np.random.SeedSequence([SEED_BASE + index, pair])
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def acquisition_times(n: int, flyback: int):
    """t_X(i, j) = j (n + f) + i and t_Y(i, j) = i (n + f) + j, as [h][w] arrays."""
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return j * (n + flyback) + i, i * (n + flyback) + j


def _motion(rng, n, drift, nsac, amp, flyback):
    T = n * (n + flyback)
    steps = rng.normal(0.0, drift, size=(T, 3))
    steps[0] = 0
    walk = np.cumsum(steps, axis=0)
    k = int(rng.integers(nsac[0], nsac[1] + 1))
    times = np.sort(rng.integers(1, T, size=k))
    jumps = np.zeros((T, 3))
    for t in times:
        mag = rng.uniform(amp / 2, amp)
        th = rng.uniform(0, 2 * math.pi)
        jumps[t] += (mag * math.cos(th), mag * math.sin(th), rng.uniform(-amp / 2, amp / 2))
    return walk + np.cumsum(jumps, axis=0), times


def _vessel_map(rng, G, n2):
    """Binary branching vessel tree on a G x G fine grid (en face, two fine
    pixels per scan pixel, n2 = 2 n), blurred."""
    img = np.zeros((G, G), np.float32)
    scale = n2 / 128.0
    r0 = 2 * min(2.5 * math.sqrt(scale), 5.0)
    nroots = 3 + int(round(2 * scale))
    budget = int(60 * scale * scale) + 40
    stack = []
    for _ in range(nroots):
        side = rng.integers(4)
        pos = rng.uniform(0, G - 1)
        if side == 0:
            p, th = (pos, 0.0), math.pi / 2
        elif side == 1:
            p, th = (pos, G - 1.0), -math.pi / 2
        elif side == 2:
            p, th = (0.0, pos), 0.0
        else:
            p, th = (G - 1.0, pos), math.pi
        stack.append((p[0], p[1], th + rng.normal(0, 0.3), r0))
    pts, rads = [], []
    nseg = 0
    while stack and nseg < budget:
        x, y, th, r = stack.pop()
        nseg += 1
        length = int(rng.uniform(10, 40) * max(1.0, math.sqrt(scale)))  # scan px (2 fine px each)
        for _ in range(length):
            th += rng.normal(0, math.radians(15))
            x += 2 * math.cos(th)
            y += 2 * math.sin(th)
            if not (0 <= x < G and 0 <= y < G):
                break
            pts.append((x, y))
            rads.append(r)
        else:
            rn = max(r * 0.8, 1.2)
            if r * 0.8 >= 1.2:
                stack.append((x, y, th + rng.normal(0, 0.2), rn))
                if rng.uniform() < 0.3:
                    stack.append((x, y, th + rng.choice([-1, 1]) * rng.uniform(0.5, 1.2), rn))
    if pts:
        P = np.asarray(pts)
        R = np.asarray(rads)
        for rq in np.unique(np.round(R * 2) / 2):
            sel = P[np.abs(np.round(R * 2) / 2 - rq) < 1e-9]
            rr = int(math.ceil(rq))
            oy, ox = np.mgrid[-rr:rr + 1, -rr:rr + 1]
            disc = (ox * ox + oy * oy) <= rq * rq + 0.25
            oy, ox = oy[disc], ox[disc]
            xs = (np.round(sel[:, 0])[:, None] + ox[None, :]).astype(np.int64).ravel()
            ys = (np.round(sel[:, 1])[:, None] + oy[None, :]).astype(np.int64).ravel()
            ok = (xs >= 0) & (xs < G) & (ys >= 0) & (ys < G)
            img[ys[ok], xs[ok]] = 1.0
    # blur sigma = 1 scan px = 2 fine px (separable)
    k = np.exp(-0.5 * (np.arange(-6, 7) / 2.0) ** 2)
    k /= k.sum()
    img = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), 0, img)
    img = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), 1, img)
    return img.astype(np.float32)


def _bilinear(field, x, y):
    """Bilinear sample of an [h][w][3] field at (x, y), clamped to the grid."""
    h, w, _ = field.shape
    x = np.clip(x, 0, w - 1)
    y = np.clip(y, 0, h - 1)
    x0 = np.minimum(np.floor(x).astype(np.int64), w - 2 if w > 1 else 0)
    y0 = np.minimum(np.floor(y).astype(np.int64), h - 2 if h > 1 else 0)
    fx = (x - x0)[..., None]
    fy = (y - y0)[..., None]
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    return ((1 - fy) * ((1 - fx) * field[y0, x0] + fx * field[y0, x1])
            + fy * ((1 - fx) * field[y1, x0] + fx * field[y1, x1]))


def _inverse_field(pos, iters: int = 30):
    """Ground-truth pull field of one scan.  The scan's A-scan at grid point q
    sees the tissue at q + m(q) (m = motion at q's acquisition time), so the
    output A-scan p must sample the scan at q = p + d with p + d + m(p + d) = p,
    i.e. d = -m(p + d); m is interpolated bilinearly between grid points and
    the fixed point is found by iteration."""
    h, w, _ = pos.shape
    j, i = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    d = -pos.astype(np.float64)
    for _ in range(iters):
        d = 0.5 * d - 0.5 * _bilinear(pos, i + d[..., 0], j + d[..., 1])
    return d


def _gauss_smooth3(x: torch.Tensor, sigma: float):
    """Separable Gaussian smoothing with edge replication, as sums of shifted
    slices (no convolution library; works for any tensor size)."""
    r = int(math.ceil(3 * sigma))
    t = torch.arange(-r, r + 1, dtype=torch.float64)
    k = torch.exp(-0.5 * (t / sigma) ** 2)
    k = (k / k.sum()).tolist()
    for dim in range(3):
        n = x.shape[dim]
        idx = torch.clamp(torch.arange(-r, n + r, device=x.device), 0, n - 1)
        xp = torch.index_select(x, dim, idx)
        y = torch.zeros_like(x)
        for q, kq in enumerate(k):
            y.add_(xp.narrow(dim, q, n), alpha=kq)
        del xp
        x = y
    return x


def _quantile(x: torch.Tensor, q: float) -> float:
    flat = x.reshape(-1)
    step = max(1, flat.numel() // 4_000_000)
    return float(torch.quantile(flat[::step].float(), q))


@dataclass
class Scans:
    """n raster scans of one phantom: volumes [h][w][d] float32 in the common
    frame, en face images [h][w], validity per scan (h values for an X-fast
    scan, whose B-scans are rows; w for a Y-fast scan, whose B-scans are
    columns), orientation per scan (0: X-fast, 1: Y-fast) and the ground-truth
    pull fields d_gt [n][h][w][3] float64."""

    S: list
    A: list
    V: list
    orient: list
    d_gt: torch.Tensor
    O: list | None = None
    saccade_ij: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)


def make_pair(workload: str | dict = "tiny", pair: int = 0, *, n: int | None = None, d: int | None = None,
              device: str | torch.device = "cpu", octa_volumes: bool = True, white_lines: bool = False,
              drift: float | None = None, saccades=None, amp: float | None = None,
              decorrelation: bool = False) -> Pair:
    """Generate one scan pair of a workload (see WORKLOADS) on `device`.

    n, d, drift, saccades and amp override the workload's values (tests use
    this for ragged and tiny shapes).  With octa_volumes=False only the en
    face OCTA images are returned (they are still the depth mean of the
    sampled OCTA volume).  With white_lines=True the OCTA B-scans that contain
    a saccade are saturated and the validity vectors mark them and their two
    neighbours on each side invalid.  With decorrelation=True the OCTA
    volumes also carry the background of amplitude-decorrelation angiography:
    0.5 exp(-s / 0.1) for the structural reflectivity s, attenuated below the
    deepest layer boundary (e-folding depth 0.05 d), so that the vitreous and
    the deep choroid are bright and the retina between vessels is dark."""
    sc = make_scans(workload, pair, (0, 1), n=n, d=d, device=device, octa_volumes=octa_volumes,
                    white_lines=white_lines, drift=drift, saccades=saccades, amp=amp, decorrelation=decorrelation)
    return Pair(sx=sc.S[0], sy=sc.S[1], ax=sc.A[0], ay=sc.A[1], vx=sc.V[0], vy=sc.V[1], d_gt=sc.d_gt,
                ox=sc.O[0] if sc.O else None, oy=sc.O[1] if sc.O else None, saccade_ij=sc.saccade_ij,
                meta=sc.meta)


def make_scans(workload: str | dict = "tiny", pair: int = 0, orients=(0, 1, 0, 1), *, n: int | None = None,
               d: int | None = None, device: str | torch.device = "cpu", octa_volumes: bool = True,
               white_lines: bool = False, drift: float | None = None, saccades=None, amp: float | None = None,
               decorrelation: bool = False) -> Scans:
    """n = len(orients) scans of one phantom, each with its own motion (see
    make_pair for the options).  With orients (0, 1) this is make_pair's
    pair; every further scan draws its motion from a stream of its own."""
    cfg = dict(WORKLOADS[workload]) if isinstance(workload, str) else dict(workload)
    if n is not None:
        cfg["n"] = n
    if d is not None:
        cfg["d"] = d
    if drift is not None:
        cfg["drift"] = drift
    if saccades is not None:
        cfg["saccades"] = saccades
    if amp is not None:
        cfg["amp"] = amp
    n, d = cfg["n"], cfg["d"]
    device = torch.device(device)
    r_ph, r_ve, r_mx, r_my = _rng_streams(cfg["index"], pair)
    fly = int(round(0.25 * n))
    ns = len(orients)

    # motion of every scan
    mrng = [r_mx, r_my] + [np.random.default_rng(np.random.SeedSequence([SEED_BASE + cfg["index"], pair, 100 + s]))
                           for s in range(2, ns)]
    tXY = acquisition_times(n, fly)
    mot = [_motion(mrng[s], n, cfg["drift"], cfg["saccades"], cfg["amp"], fly) for s in range(ns)]
    pos = [mot[s][0][tXY[orients[s]]] for s in range(ns)]  # [h][w][3] motion at each output A-scan
    # The truth's coordinate frame is arbitrary: place it so that the motion
    # of all scans has zero mean, which is the gauge the mean-displacement
    # term selects (the registered volumes stay centred on the output grid).
    c = np.concatenate([q.reshape(-1, 3) for q in pos]).mean(axis=0)
    pos = [q - c for q in pos]
    margin = int(math.ceil(max(np.abs(q[..., :2]).max() for q in pos))) + 3
    mz = int(math.ceil(max(np.abs(q[..., 2]).max() for q in pos))) + 3
    # The truth lives on a grid twice as fine as the scans (fine index
    # u = 2 (x + margin)), so that trilinear acquisition sampling blurs only
    # at the fine scale.
    G = 2 * (n - 1 + 2 * margin) + 1
    Dz = 2 * (d - 1 + 2 * mz) + 1

    # layered structure on the truth grid (rows y, columns x, depth z)
    coef = r_ph.normal(0, 0.02, size=(6, 6))
    refl = np.asarray(LAYER_R) + r_ph.uniform(-0.05, 0.05, size=7)
    noise_seed = int(r_ph.integers(0, 2**62))
    g = torch.arange(G, dtype=torch.float32, device=device) / 2 - margin
    u = (g / max(n - 1, 1) - 0.5)
    vv, uu = torch.meshgrid(u, u, indexing="ij")
    basis = [torch.ones_like(uu), uu, vv, uu * uu, uu * vv, vv * vv]
    bnd = []
    for b in range(6):
        p = sum(float(coef[b, q]) * basis[q] for q in range(6))
        bnd.append(d * (LAYER_C[b] + p))
    bnd = torch.stack(bnd)
    bnd, _ = torch.sort(bnd, dim=0)
    for b in range(1, 6):
        bnd[b] = torch.maximum(bnd[b], bnd[b - 1] + 3.0)
    z = torch.arange(Dz, dtype=torch.float32, device=device) / 2 - mz
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    truth = torch.empty((G, G, Dz), dtype=torch.float32, device=device)
    slab = torch.empty((G, G, Dz), dtype=torch.float32, device=device)
    rows = max(1, int(2**25 // (G * Dz)))
    for r0 in range(0, G, rows):
        r1 = min(G, r0 + rows)
        zz = z.view(1, 1, -1)
        val = torch.full((r1 - r0, G, Dz), float(refl[0]), device=device)
        for b in range(6):
            edge = torch.sigmoid((zz - bnd[b, r0:r1, :, None]) / 0.5)
            val += float(refl[b + 1] - refl[b]) * edge
        truth[r0:r1] = val
        s1 = torch.sigmoid((zz - bnd[1, r0:r1, :, None]) / 0.5)
        s3 = torch.sigmoid((bnd[3, r0:r1, :, None] - zz) / 0.5)
        slab[r0:r1] = s1 * s3
    noise = torch.randn((G, G, Dz), generator=gen, device=device)
    noise = _gauss_smooth3(noise, 1.4)  # 0.7 scan voxels
    noise = noise / noise.std()
    truth *= torch.exp(0.5 * noise - 0.125)
    del noise
    truth /= _quantile(truth, 0.99)

    vmap = torch.from_numpy(_vessel_map(r_ve, G, 2 * n)).to(device)
    octa_truth = slab * vmap[:, :, None]
    del slab
    if decorrelation:
        for r0 in range(0, G, rows):
            r1 = min(G, r0 + rows)
            zz = z.view(1, 1, -1)
            att = torch.exp(-torch.clamp(zz - bnd[5, r0:r1, :, None], min=0.0) / (0.05 * d))
            octa_truth[r0:r1] += 0.5 * torch.exp(-truth[r0:r1] * att / 0.1)

    def sample(vol, pos):
        """Trilinear sample of the fine truth volume at output voxels
        (i + m_x, j + m_y, k + m_z), in row slabs; each slab reads only the
        truth rows it can reach."""
        out = torch.empty((n, n, d), dtype=torch.float32, device=device)
        post = torch.as_tensor(pos, dtype=torch.float32, device=device)
        kk = torch.arange(d, dtype=torch.float32, device=device)
        ii = torch.arange(n, dtype=torch.float32, device=device)
        rs = max(1, int(2**23 // (n * d)))
        for j0 in range(0, n, rs):
            j1 = min(n, j0 + rs)
            jj = torch.arange(j0, j1, dtype=torch.float32, device=device)
            P = post[j0:j1]
            yf = 2 * (jj[:, None] + P[..., 1] + margin)          # fine row coordinate
            r0 = max(0, int(math.floor(float(yf.min()))) - 1)
            r1 = min(G - 1, int(math.ceil(float(yf.max()))) + 1)
            inp = vol[r0:r1 + 1][None, None]  # (N, C, D=rows y, H=cols x, W=depth z)
            yy = (yf - r0)[..., None].expand(-1, -1, d)
            xx = (2 * (ii[None, :] + P[..., 0] + margin))[..., None].expand(-1, -1, d)
            zq = 2 * (kk[None, None, :] + P[..., 2:3] + mz)
            ny = max(r1 - r0, 1)
            grid = torch.stack([2 * zq / (Dz - 1) - 1, 2 * xx / (G - 1) - 1, 2 * yy / ny - 1], dim=-1)
            out[j0:j1] = F.grid_sample(inp, grid[None], mode="bilinear", padding_mode="border",
                                       align_corners=True)[0, 0]
        return out

    S = [sample(truth, q) for q in pos]
    del truth
    O = [sample(octa_truth, q) for q in pos]
    del octa_truth
    # Rayleigh noise of scale 0.1 per scan: sigma sqrt(-2 ln U)
    for o in O:
        uq = torch.rand(o.shape, generator=gen, device=device).clamp_min_(1e-12)
        o += 0.1 * torch.sqrt(-2.0 * torch.log(uq))
        del uq

    Vv = [torch.ones(n, dtype=torch.float32, device=device) for _ in range(ns)]
    sac = []
    if white_lines:
        for s in range(ns):
            o = orients[s]
            for t in mot[s][1]:
                b = int(t // (n + fly))
                if b >= n:
                    continue
                sac.append((s, b))
                Vv[s][max(0, b - 2):b + 3] = 0.0
                if o == 0:
                    O[s][b] = 1.0 + 0.05 * torch.rand(O[s][b].shape, generator=gen, device=device)
                else:
                    O[s][:, b] = 1.0 + 0.05 * torch.rand(O[s][:, b].shape, generator=gen, device=device)
    A = [o.mean(dim=2) for o in O]
    scale = _quantile(torch.cat([a.reshape(-1) for a in A]), 0.99)
    for a in A:
        a /= scale
    for o in O:
        o /= scale

    dgt = np.stack([_inverse_field(q) for q in pos])
    dgt -= dgt.reshape(-1, 3).mean(axis=0)
    meta = dict(workload=workload if isinstance(workload, str) else "custom", pair=pair, n=n, d=d,
                flyback=fly, margin=margin, saccade_times=tuple(m[1].tolist() for m in mot),
                levels=cfg.get("levels", 3), orients=tuple(orients))
    return Scans(S=S, A=A, V=Vv, orient=list(orients), d_gt=torch.from_numpy(dgt),
                 O=O if octa_volumes else None, saccade_ij=sac, meta=meta)


def perturbed_field(d_gt: torch.Tensor, sigma: float, seed: int) -> torch.Tensor:
    """Ground truth plus i.i.d. N(0, sigma^2) pixel noise (a test displacement)."""
    rng = np.random.default_rng(seed)
    return d_gt + torch.from_numpy(rng.normal(0, sigma, size=tuple(d_gt.shape)))


def smooth_random_field(w: int, h: int, amp: float, seed: int) -> torch.Tensor:
    """A smooth random displacement field [2][h][w][3] (sum of a few cosines)."""
    rng = np.random.default_rng(seed)
    j, i = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    out = np.zeros((2, h, w, 3))
    for V in range(2):
        for c in range(3):
            for _ in range(3):
                fx, fy = rng.uniform(0, 3, size=2)
                ph = rng.uniform(0, 2 * math.pi)
                out[V, :, :, c] += amp / 3 * np.cos(2 * math.pi * (fx * i / w + fy * j / h) + ph)
    return torch.from_numpy(out)


def random_field(w: int, h: int, amp: float, seed: int) -> torch.Tensor:
    """Uniform random displacements in [-amp, amp] (includes negative and
    out-of-range sample positions)."""
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.uniform(-amp, amp, size=(2, h, w, 3)))


def layered_axial_pair(h: int, w: int, d: int, mX, mY):
    """Analytic layered volumes [h][w][d] (four logistic layers over laterally
    curved boundaries) acquired with per-A-scan axial offsets mX, mY ([h][w]):
    scan V at (i, j, k) is the structure at depth k + m^V(i, j).  No lateral
    motion; the aligning pull fields satisfy d^X - d^Y = m^Y - m^X."""
    def vol(m):
        z = np.arange(d)[None, None, :] + np.asarray(m, dtype=np.float64)[:, :, None]
        x = np.arange(w)[None, :, None]
        y = np.arange(h)[:, None, None]
        out = np.zeros((h, w, d))
        for cl, a in ((0.30, 0.9), (0.42, -0.5), (0.55, 0.6), (0.70, 0.7)):
            b = d * cl + 1.5 * np.sin(x / 5.0) + 1.2 * np.cos(y / 6.0)
            out += a / (1 + np.exp(-(z - b) / 1.2))
        return out
    return vol(mX), vol(mY)


def planted_axial_motion(h: int, w: int, seed: int = 0, jump: float = 2.0, tilt_x: float = 0.04,
                         tilt_y: float = -0.03):
    """Per-B-scan axial offsets (random walks, a jump in the X-fast scan) and
    one tilt per scan along its fast axis: (mX, mY) [h][w]."""
    rng = np.random.default_rng(seed)
    sX = np.cumsum(rng.normal(0, 0.3, h))
    sX[h // 2:] += jump
    rY = np.cumsum(rng.normal(0, 0.3, w))
    mX = sX[:, None] + tilt_x * (np.arange(w)[None, :] - (w - 1) / 2)
    mY = rY[None, :] + tilt_y * (np.arange(h)[:, None] - (h - 1) / 2)
    return mX, mY
