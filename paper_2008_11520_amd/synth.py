"""Seeded synthetic inputs for the fine-level DNN-MG step.

This module only *makes inputs*: coarse meshes, coarse velocity/pressure
fields, network weights and serving arrivals.  It holds none of the method's
arithmetic (no prolongation, defect, network or restriction), so both the
GPU library and the FP64 oracle can be driven from it without sharing code.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written here from its
published definition: the state advances by the golden-ratio increment and
each output is the state passed through the two xor-shift-multiply rounds of
Stafford's "Mix13" finaliser.  Uniform doubles take the top 53 bits.

The paper's own flows (a Schaefer-Turek channel with an elliptic obstacle,
Sec. 5.1) and its trained weights are not available; the generators below
stand in for them with the channel's dimensions (2.2 x 0.41) and a parabolic
inflow, smooth divergence-free Fourier fields, and Xavier-uniform weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


class SplitMix64:
    """Counter-based SplitMix64 stream: output k is mix(seed + k*gamma)."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)

    def next_u64(self, n: int) -> np.ndarray:
        if n <= 16:
            # the same values from Python integers (a few draws cost less
            # this way than through numpy's small-array calls)
            mask = (1 << 64) - 1
            s0, g = int(self.state), int(_GAMMA)
            out = []
            for k in range(1, n + 1):
                z = (s0 + k * g) & mask
                z = ((z ^ (z >> 30)) * int(_M1)) & mask
                z = ((z ^ (z >> 27)) * int(_M2)) & mask
                out.append(z ^ (z >> 31))
            self.state = np.uint64((s0 + n * g) & mask)
            return np.array(out, dtype=np.uint64)
        with np.errstate(over="ignore"):
            k = np.arange(1, n + 1, dtype=np.uint64)
            z = self.state + k * _GAMMA
            self.state = self.state + np.uint64(n) * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def integers(self, n: int, lo: int, hi: int) -> np.ndarray:
        """Integers uniform in [lo, hi] (inclusive), by floor of a uniform draw."""
        u = self.uniform(n)
        return lo + np.minimum(np.floor(u * (hi - lo + 1)), hi - lo).astype(np.int64)


# --------------------------------------------------------------------------
# Meshes.  Coarse node (i, j) has index j*(nx+1)+i; arrays are (ny+1, nx+1, 2).
# --------------------------------------------------------------------------

def rect_mesh(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0,
              x0: float = 0.0, y0: float = 0.0) -> np.ndarray:
    xs = x0 + lx * np.arange(nx + 1, dtype=np.float64) / nx
    ys = y0 + ly * np.arange(ny + 1, dtype=np.float64) / ny
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X, Y], axis=-1)


def rect_mesh_torch(nx: int, ny: int, lx: float, ly: float, device):
    """rect_mesh formed on a torch device ((ny+1)(nx+1) x 2 float64), the
    same values: no host-to-device copy."""
    import torch
    xs = lx * torch.arange(nx + 1, dtype=torch.float64, device=device) / nx
    ys = ly * torch.arange(ny + 1, dtype=torch.float64, device=device) / ny
    Y, X = torch.meshgrid(ys, xs, indexing="ij")
    return torch.stack([X, Y], dim=-1).reshape(-1, 2)


def perturb_interior(cxy: np.ndarray, frac: float, seed: int) -> np.ndarray:
    """Move every interior coarse node by U[-frac*h, frac*h] in each direction
    (h = local spacing per direction); boundary nodes stay put."""
    ny1, nx1, _ = cxy.shape
    out = cxy.copy()
    hx = (cxy[0, -1, 0] - cxy[0, 0, 0]) / (nx1 - 1)
    hy = (cxy[-1, 0, 1] - cxy[0, 0, 1]) / (ny1 - 1)
    rng = SplitMix64(seed)
    n_int = max(nx1 - 2, 0) * max(ny1 - 2, 0)
    d = rng.uniform(2 * n_int, -frac, frac).reshape(max(ny1 - 2, 0), max(nx1 - 2, 0), 2)
    out[1:-1, 1:-1, 0] += d[..., 0] * hx
    out[1:-1, 1:-1, 1] += d[..., 1] * hy
    return out


# Dirichlet side flags (bit0 x=xmin, bit1 x=xmax, bit2 y=ymin, bit3 y=ymax).
DIR_XMIN, DIR_XMAX, DIR_YMIN, DIR_YMAX = 1, 2, 4, 8
DIR_ALL = 15
DIR_CHANNEL = DIR_XMIN | DIR_YMIN | DIR_YMAX   # inflow + walls; outflow is do-nothing


# --------------------------------------------------------------------------
# Fields.
# --------------------------------------------------------------------------

@dataclass
class FourierField:
    """Divergence-free velocity from a stream function of `nmodes` modes:
    psi = sum_m |k_m|^-1 sin(2 pi (kx x/Lx + ky y/Ly) + phi_m + w_m t),
    v = (d psi/dy, -d psi/dx), scaled so that max |v| over the coarse nodes
    at t = 0 equals `amplitude`.  A scalar field of `pmodes` modes and
    amplitude `p_amplitude` stands in for the coarse pressure."""
    lx: float
    ly: float
    seed: int
    nmodes: int = 8
    pmodes: int = 4
    amplitude: float = 1.0
    p_amplitude: float = 0.1
    k: np.ndarray = field(init=False)
    phi: np.ndarray = field(init=False)
    om: np.ndarray = field(init=False)
    pk: np.ndarray = field(init=False)
    pphi: np.ndarray = field(init=False)
    pom: np.ndarray = field(init=False)
    vscale: float = field(init=False, default=1.0)
    pscale: float = field(init=False, default=1.0)

    def __post_init__(self):
        rng = SplitMix64(self.seed)

        def draw_k(n):
            ks = []
            while len(ks) < n:
                kk = rng.integers(2, -4, 4)
                if kk[0] != 0 or kk[1] != 0:
                    ks.append(kk)
            return np.array(ks, dtype=np.float64)

        self.k = draw_k(self.nmodes)
        self.phi = rng.uniform(self.nmodes, 0.0, 2 * math.pi)
        self.om = 2 * math.pi * rng.uniform(self.nmodes, 0.5, 2.0)
        self.pk = draw_k(self.pmodes)
        self.pphi = rng.uniform(self.pmodes, 0.0, 2 * math.pi)
        self.pom = 2 * math.pi * rng.uniform(self.pmodes, 0.5, 2.0)

    def _raw_v(self, x, y, t):
        vx = np.zeros_like(x)
        vy = np.zeros_like(x)
        for m in range(self.nmodes):
            kx, ky = self.k[m]
            inv = 1.0 / math.hypot(kx, ky)
            th = 2 * math.pi * (kx * x / self.lx + ky * y / self.ly) + self.phi[m] + self.om[m] * t
            c = np.cos(th) * inv * 2 * math.pi
            vx += c * ky / self.ly
            vy -= c * kx / self.lx
        return vx, vy

    def _raw_p(self, x, y, t):
        p = np.zeros_like(x)
        for m in range(self.pmodes):
            kx, ky = self.pk[m]
            th = 2 * math.pi * (kx * x / self.lx + ky * y / self.ly) + self.pphi[m] + self.pom[m] * t
            p += np.sin(th)
        return p

    def calibrate(self, cxy: np.ndarray) -> "FourierField":
        x, y = cxy[..., 0], cxy[..., 1]
        vx, vy = self._raw_v(x, y, 0.0)
        m = float(np.sqrt(vx * vx + vy * vy).max())
        self.vscale = self.amplitude / m if m > 0 else 1.0
        pm = float(np.abs(self._raw_p(x, y, 0.0)).max())
        self.pscale = self.p_amplitude / pm if pm > 0 else 1.0
        return self

    def velocity(self, cxy, t):
        vx, vy = self._raw_v(cxy[..., 0], cxy[..., 1], t)
        return np.stack([vx, vy], axis=-1) * self.vscale

    def pressure(self, cxy, t):
        return self._raw_p(cxy[..., 0], cxy[..., 1], t) * self.pscale

    # The same fields evaluated with torch on a device tensor of node
    # coordinates (N x 2, float64), for inputs made on the GPU.
    def _raw_torch(self, xy, times):
        """Raw v and p at the nodes for every time, all modes at once (a few
        kernels whatever the number of modes): (T x N) each."""
        import torch
        dev, dt_ = xy.device, xy.dtype
        x, y = xy[:, 0][None, :, None], xy[:, 1][None, :, None]
        t = torch.as_tensor(times, dtype=dt_, device=dev).reshape(-1, 1, 1)

        # the field's constants in one array, copied once (from pinned memory
        # to a device: asynchronously, without waiting for the stream)
        M, Mp = self.nmodes, self.pmodes
        host = np.concatenate([self.k[:, 0], self.k[:, 1], self.phi, self.om,
                               2 * math.pi / np.hypot(self.k[:, 0], self.k[:, 1]),
                               self.pk[:, 0], self.pk[:, 1], self.pphi, self.pom])
        up = getattr(self, "_upload", None)
        if dev.type == "cpu":
            cst = torch.from_numpy(host).to(dt_)
        elif up is not None:
            # (the caller's asynchronous host-to-device path, e.g. the serving
            # arena's staging ring: no pinned allocation per field)
            cst = torch.empty(host.size, dtype=torch.float64, device=dev)
            up(cst, host)
            cst = cst.to(dt_)
        else:
            cst = torch.from_numpy(host).to(dt_).pin_memory().to(dev, non_blocking=True)
        kx, ky, phi, om, inv = (cst[i * M:(i + 1) * M] for i in range(5))
        pkx, pky, pphi, pom = (cst[5 * M + i * Mp:5 * M + (i + 1) * Mp] for i in range(4))
        th = 2 * math.pi * (kx * x / self.lx + ky * y / self.ly) + phi + om * t
        c = torch.cos(th) * inv
        vx = (c * (ky / self.ly)).sum(-1)
        vy = -(c * (kx / self.lx)).sum(-1)
        p = torch.sin(2 * math.pi * (pkx * x / self.lx + pky * y / self.ly) + pphi + pom * t).sum(-1)
        return vx, vy, p

    def calibrate_torch(self, xy) -> "FourierField":
        vx, vy, p = self._raw_torch(xy, [0.0])
        m = float(torch_hypot_max(vx, vy))
        self.vscale = self.amplitude / m if m > 0 else 1.0
        pm = float(p.abs().max())
        self.pscale = self.p_amplitude / pm if pm > 0 else 1.0
        return self

    def fields_torch(self, xy, times, inflow_max=0.0, height=0.41):
        """(v, p) at the given times: (T x N x 2, T x N) on xy's device."""
        import torch
        vx, vy, p = self._raw_torch(xy, times)
        vx, vy, p = vx * self.vscale, vy * self.vscale, p * self.pscale
        if inflow_max > 0.0:
            y = xy[:, 1][None, :]
            prof = 4.0 * y * (height - y) / (height * height)
            vx, vy = vx * prof + inflow_max * prof, vy * prof
        return torch.stack([vx, vy], dim=-1), p


def fields_torch_calibrated(ff: "FourierField", xy, times, inflow_max=0.0, height=0.41, upload=None):
    """ff.fields_torch with the calibration (max |v| and max |p| over the
    nodes at t = 0) done on the device as well: no value is read back to the
    host, so evaluating a flow's fields does not wait for the stream's other
    work.  Same scaling rule as calibrate()."""
    import torch
    # (times formed on the device: a host list would be copied with a
    # stream synchronisation)
    if not torch.is_tensor(times):
        times = torch.as_tensor(times, dtype=xy.dtype).to(xy.device, non_blocking=True)
    ff._upload = upload
    vx0, vy0, p0 = ff._raw_torch(xy, torch.zeros(1, dtype=xy.dtype, device=xy.device))
    m = torch_hypot_max(vx0, vy0)
    pm = p0.abs().max()
    one = torch.ones((), dtype=xy.dtype, device=xy.device)
    vscale = torch.where(m > 0, ff.amplitude / torch.where(m > 0, m, one), one)
    pscale = torch.where(pm > 0, ff.p_amplitude / torch.where(pm > 0, pm, one), one)
    vx, vy, p = ff._raw_torch(xy, times)
    vx, vy, p = vx * vscale, vy * vscale, p * pscale
    if inflow_max > 0.0:
        y = xy[:, 1][None, :]
        prof = 4.0 * y * (height - y) / (height * height)
        vx, vy = vx * prof + inflow_max * prof, vy * prof
    return torch.stack([vx, vy], dim=-1), p


def torch_hypot_max(vx, vy):
    return (vx * vx + vy * vy).sqrt().max()


def channel_rings_torch(ffs, meshes, times, lx, ly, inflow_max, height, device, upload=None):
    """fields_torch_calibrated for a group of flows on rect_mesh(nx, ny, lx,
    ly) meshes, evaluated together (a few tens of kernels for the group
    instead of per flow).  ffs: FourierField per flow (same nmodes, pmodes);
    meshes: (nx, ny) per flow.  Returns v (T x N x 2), p (T x N), FP64, the
    flows' nodes one after another, and the F + 1 node offsets (flow f holds
    nodes offs[f] .. offs[f+1]-1).  Every node value is formed by element-wise
    operations only, the modes summed one after another, and the calibration
    maxima are per flow, so a flow's values do not depend on which flows share
    its group."""
    import torch
    F = len(ffs)
    M, Mp = ffs[0].nmodes, ffs[0].pmodes
    if any(f.nmodes != M or f.pmodes != Mp for f in ffs):
        raise ValueError("all flows of a group need the same mode counts")
    counts = np.array([(nx + 1) * (ny + 1) for nx, ny in meshes], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)])
    N = int(offs[-1])
    times = np.asarray(times, dtype=np.float64).reshape(-1)
    T = times.size
    # one host array, one copy: per flow nx, ny, nx + 1, first node, the two
    # amplitudes and the field constants; then the times (t = 0 first, for
    # the calibration) and the node counts
    c0 = 6
    per = np.empty((F, c0 + 5 * M + 4 * Mp), dtype=np.float64)
    for f, (ff, (nx, ny)) in enumerate(zip(ffs, meshes)):
        per[f, :c0] = (nx, ny, nx + 1, offs[f], ff.amplitude, ff.p_amplitude)
        per[f, c0:] = np.concatenate([ff.k[:, 0], ff.k[:, 1], ff.phi, ff.om,
                                      2 * math.pi / np.hypot(ff.k[:, 0], ff.k[:, 1]),
                                      ff.pk[:, 0], ff.pk[:, 1], ff.pphi, ff.pom])
    host = np.concatenate([per.reshape(-1), [0.0], times, counts.astype(np.float64)])
    if torch.device(device).type == "cpu":
        buf = torch.from_numpy(host.copy())
    elif upload is not None:
        buf = torch.empty(host.size, dtype=torch.float64, device=device)
        upload(buf, host)
    else:
        buf = torch.from_numpy(host).pin_memory().to(device, non_blocking=True)
    dev = buf.device
    per_t = buf[:per.size].reshape(per.shape)
    t = buf[per.size:per.size + 1 + T].reshape(-1, 1)
    cnt = buf[per.size + 1 + T:].to(torch.int64)
    fid = torch.repeat_interleave(torch.arange(F, device=dev), cnt, output_size=N)
    g = per_t.t()[:, fid]                            # the node's flow constants, one row per constant
    local = torch.arange(N, device=dev) - g[3].to(torch.int64)
    nx1 = g[2].to(torch.int64)
    # rect_mesh_torch's arithmetic: (l * index) / n
    x = lx * (local % nx1).double() / g[0]
    y = ly * torch.div(local, nx1, rounding_mode="floor").double() / g[1]
    kx = lambda m: g[c0 + m]
    ky = lambda m: g[c0 + M + m]
    phi = lambda m: g[c0 + 2 * M + m]
    om = lambda m: g[c0 + 3 * M + m]
    inv = lambda m: g[c0 + 4 * M + m]
    pc = c0 + 5 * M
    vx = torch.zeros(T + 1, N, dtype=torch.float64, device=dev)
    vy = torch.zeros_like(vx)
    p = torch.zeros_like(vx)
    for m in range(M):
        th = 2 * math.pi * (kx(m) * x / lx + ky(m) * y / ly) + phi(m) + om(m) * t
        c = torch.cos(th) * inv(m)
        vx += c * (ky(m) / ly)
        vy -= c * (kx(m) / lx)
    for m in range(Mp):
        th = 2 * math.pi * (g[pc + m] * x / lx + g[pc + Mp + m] * y / ly) + g[pc + 2 * Mp + m] + g[pc + 3 * Mp + m] * t
        p += torch.sin(th)
    # calibration at t = 0: maxima over each flow's run of nodes (exact in
    # any order)
    mv = torch.segment_reduce((vx[0] * vx[0] + vy[0] * vy[0]).sqrt(), "max", lengths=cnt)
    mp = torch.segment_reduce(p[0].abs(), "max", lengths=cnt)
    one = torch.ones((), dtype=torch.float64, device=dev)
    vscale = torch.where(mv > 0, per_t[:, 4] / torch.where(mv > 0, mv, one), one)[fid]
    pscale = torch.where(mp > 0, per_t[:, 5] / torch.where(mp > 0, mp, one), one)[fid]
    vx, vy, p = vx[1:] * vscale, vy[1:] * vscale, p[1:] * pscale
    if inflow_max > 0.0:
        prof = 4.0 * y * (height - y) / (height * height)
        vx, vy = vx * prof + inflow_max * prof, vy * prof
    return torch.stack([vx, vy], dim=-1), p, offs


CHANNEL_LX, CHANNEL_LY = 2.2, 0.41


def channel_profile(y: np.ndarray, height: float = CHANNEL_LY) -> np.ndarray:
    return 4.0 * y * (height - y) / (height * height)


@dataclass
class Flow:
    """One synthetic flow: a coarse mesh plus the coarse fields per time step."""
    nx: int
    ny: int
    cxy: np.ndarray           # (ny+1, nx+1, 2) float64
    dirichlet: int
    dt: float
    fourier: FourierField
    inflow_max: float = 0.0   # > 0: channel form v = inflow*e_x + fourier*profile

    def fields(self, step: int):
        """Coarse (v, p) at t_n = n*dt, float32, node-major (Nc, 2) and (Nc,)."""
        t = step * self.dt
        v = self.fourier.velocity(self.cxy, t)
        if self.inflow_max > 0.0:
            prof = channel_profile(self.cxy[..., 1])
            v = v * prof[..., None]
            v[..., 0] += self.inflow_max * prof
        p = self.fourier.pressure(self.cxy, t)
        nc = (self.nx + 1) * (self.ny + 1)
        return (v.reshape(nc, 2).astype(np.float32),
                p.reshape(nc).astype(np.float32))


def unit_square_flow(nx=16, ny=16, field_seed=1, dt=0.01) -> Flow:
    cxy = rect_mesh(nx, ny)
    ff = FourierField(1.0, 1.0, field_seed).calibrate(cxy)
    return Flow(nx, ny, cxy, DIR_ALL, dt, ff)


def channel_flow(nx=256, ny=64, field_seed=1, dt=0.005, perturb_seed=None,
                 perturb_frac=0.1, inflow_max=1.5) -> Flow:
    cxy = rect_mesh(nx, ny, CHANNEL_LX, CHANNEL_LY)
    if perturb_seed is not None:
        cxy = perturb_interior(cxy, perturb_frac, perturb_seed)
    ff = FourierField(CHANNEL_LX, CHANNEL_LY, field_seed).calibrate(cxy)
    return Flow(nx, ny, cxy, DIR_CHANNEL, dt, ff, inflow_max=inflow_max)


def stretched_flow(nx=128, ny=128, stretch=1.0, field_seed=1, dt=0.01) -> Flow:
    cxy = rect_mesh(nx, ny, stretch, 1.0)
    ff = FourierField(stretch, 1.0, field_seed).calibrate(cxy)
    return Flow(nx, ny, cxy, DIR_ALL, dt, ff)


def stretch_factors(nflows: int, seed: int = 5, lo: float = 1.0, hi: float = 8.0):
    return SplitMix64(seed).uniform(nflows, lo, hi)


# --------------------------------------------------------------------------
# Network weights: W_z, W_r, W_h (H x Nin), U_z, U_r, U_h (H x H), then
# M1 (Hm x H) and M2 (Nout x Hm), or M (Nout x H); row-major (out x in),
# no biases.  Xavier-uniform bound sqrt(6 / (fan_in + fan_out)) per matrix.
# --------------------------------------------------------------------------

def net_shapes(K: int, H: int, Hm: int):
    n = 1 << K
    nf = (n + 1) * (n + 1)
    nout = 2 * nf
    nin = 2 * nf + 2 * nf + 4
    shapes = [(H, nin)] * 3 + [(H, H)] * 3
    shapes += [(Hm, H), (nout, Hm)] if Hm > 0 else [(nout, H)]
    return nin, nout, shapes


def xavier_weights(K: int, H: int, Hm: int, seed: int) -> np.ndarray:
    _, _, shapes = net_shapes(K, H, Hm)
    rng = SplitMix64(seed)
    parts = []
    for (o, i) in shapes:
        a = math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(o * i, -a, a))
    return np.concatenate(parts).astype(np.float32)


def paper_net_weights(K: int, H: int, seed: int) -> np.ndarray:
    """Seeded weights of the paper's network form (DNNMG_F_PAPER_NET): the
    GRU over 3 nf + 24 inputs and the dense layer Xavier-uniform, the two
    convolutional blocks' 36 weights each uniform in +-1/3, the last
    layer's nout weights uniform in [0.5, 1.5]."""
    n = 1 << K
    nf = (n + 1) * (n + 1)
    nin, nout = 3 * nf + 24, 2 * nf
    rng = SplitMix64(seed)
    parts = []
    for (o, i) in [(H, nin)] * 3 + [(H, H)] * 3 + [(nout, H)]:
        a = math.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(o * i, -a, a))
    parts.append(rng.uniform(72, -1.0 / 3.0, 1.0 / 3.0))
    parts.append(rng.uniform(nout, 0.5, 1.5))
    return np.concatenate(parts).astype(np.float32)


def split_weights(w: np.ndarray, K: int, H: int, Hm: int):
    """Views of the packed weight vector as the individual matrices."""
    _, _, shapes = net_shapes(K, H, Hm)
    out, off = [], 0
    for (o, i) in shapes:
        out.append(w[off:off + o * i].reshape(o, i))
        off += o * i
    assert off == w.size, (off, w.size)
    return out


# --------------------------------------------------------------------------
# Named workloads (sizes of the paper-derived configurations).
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    K: int
    H: int
    Hm: int
    nu: float
    steps: int
    flows: list
    weight_seed: int = 1234


def workload(name: str) -> Workload:
    if name == "unit16_k1":          # 16x16 unit square, K=1, H=32, linear 32->18
        return Workload(name, 1, 32, 0, 1e-3, 10, [unit_square_flow(16, 16, 1, 0.01)])
    if name == "channel256x64_k2":   # 256x64 channel, K=2, H=64, MLP 64->64->50
        return Workload(name, 2, 64, 64, 1e-3, 100, [channel_flow(256, 64, 1, 0.005)])
    if name == "channel1024x256_k2_perturbed":
        return Workload(name, 2, 64, 64, 1e-3, 200,
                        [channel_flow(1024, 256, 1, 0.005, perturb_seed=7)])
    if name == "stretched64x128x128_k3":
        s = stretch_factors(64, 5)
        return Workload(name, 3, 128, 128, 1e-3, 100,
                        [stretched_flow(128, 128, float(s[f]), 100 + f, 0.01) for f in range(64)])
    raise KeyError(name)


# --------------------------------------------------------------------------
# Serving arrivals: Poisson process, mesh sizes and step counts per request.
# --------------------------------------------------------------------------

SERVE_MESHES = [(32, 8), (64, 16), (128, 32), (256, 64), (512, 128)]


def serving_requests(n: int = 256, rate: float = 20.0, seed: int = 11,
                     steps_lo: int = 50, steps_hi: int = 500):
    rng = SplitMix64(seed)
    gaps = -np.log1p(-rng.uniform(n)) / rate
    arrivals = np.cumsum(gaps)
    mesh_idx = rng.integers(n, 0, len(SERVE_MESHES) - 1)
    steps = rng.integers(n, steps_lo, steps_hi)
    reqs = []
    for r in range(n):
        nx, ny = SERVE_MESHES[int(mesh_idx[r])]
        reqs.append(dict(id=r, arrival=float(arrivals[r]), nx=nx, ny=ny,
                         steps=int(steps[r]), field_seed=1000 + r))
    return reqs


# --------------------------------------------------------------------------
# Unstructured quadrilateral meshes (explicit connectivity, curved edges).
# --------------------------------------------------------------------------

@dataclass
class UMesh:
    """A coarse quadrilateral mesh: node coordinates (Nc x 2), elements
    (P x 4 node indices v0, v1, v2, v3 counter-clockwise), Dirichlet edges
    (node pairs), circles (cx, cy, r) and curved edges (node a, node b,
    circle index)."""
    xy: np.ndarray
    elems: np.ndarray
    dirichlet_edges: np.ndarray
    circles: np.ndarray
    curved: np.ndarray


@dataclass
class UFlow:
    """A synthetic flow on an unstructured mesh: the coarse fields per step."""
    mesh: UMesh
    dt: float
    fourier: FourierField
    inflow_max: float = 0.0
    height: float = CHANNEL_LY
    hole: tuple = None        # (cx, cy, r): velocity damped to zero on this circle

    def fields(self, step: int):
        xy = self.mesh.xy
        t = step * self.dt
        v = self.fourier.velocity(xy, t)
        if self.inflow_max > 0.0:
            prof = channel_profile(xy[:, 1], self.height)
            v = v * prof[:, None]
            v[:, 0] += self.inflow_max * prof
        if self.hole is not None:
            cx, cy, r = self.hole
            d = np.hypot(xy[:, 0] - cx, xy[:, 1] - cy)
            s = np.clip((d - r) / r, 0.0, 1.0)
            v = v * (s * s * (3.0 - 2.0 * s))[:, None]
        p = self.fourier.pressure(xy, t)
        return v.astype(np.float32), p.astype(np.float32)


def _signed_area(xy, e):
    p = xy[e]
    return 0.5 * float(np.sum(p[:, 0] * np.roll(p[:, 1], -1) - np.roll(p[:, 0], -1) * p[:, 1]))


class _NodeSet:
    """Nodes merged by their coordinates (rounded to 1e-12 of the domain)."""

    def __init__(self, scale):
        self.q = 1e-12 * scale
        self.idx, self.pts = {}, []

    def add(self, x, y):
        key = (round(x / self.q), round(y / self.q))
        i = self.idx.get(key)
        if i is None:
            i = len(self.pts)
            self.idx[key] = i
            self.pts.append((x, y))
        return i


def cylinder_channel_umesh(m=8, length=CHANNEL_LX, height=CHANNEL_LY, center=(0.2, 0.2), radius=0.05,
                           half_box=0.1):
    """The channel [0, length] x [0, height] around a circular obstacle: an
    O-grid ring of 4 m x mr elements between the circle and a square box
    (half side half_box), and eight structured blocks outside the box, the
    box side cut into m elements; about uniform element size 2 half_box / m.
    Vertices where the ring meets the blocks' corners have five elements.
    Curved edges: the ring's edges on the circle.  Dirichlet edges: the
    inflow side x = 0, the walls y = 0, y = height and the circle; the
    outflow x = length is do-nothing."""
    cx, cy = center
    hs = 2.0 * half_box / m
    x0, x1 = cx - half_box, cx + half_box
    y0, y1 = cy - half_box, cy + half_box
    nodes = _NodeSet(max(length, height))
    elems, curved, dirichlet = [], [], []

    def add_quad(a, b, c, d, xy_tmp):
        e = [a, b, c, d]
        if _signed_area(xy_tmp, e) < 0:
            e = [a, d, c, b]
        elems.append(e)

    # square box perimeter, counter-clockwise from (x0, y0)
    per = []
    for k in range(m):
        per.append((x0 + (x1 - x0) * k / m, y0))
    for k in range(m):
        per.append((x1, y0 + (y1 - y0) * k / m))
    for k in range(m):
        per.append((x1 - (x1 - x0) * k / m, y1))
    for k in range(m):
        per.append((x0, y1 - (y1 - y0) * k / m))
    mr = max(1, int(round((half_box - radius) / hs)))
    ring = np.empty((4 * m, mr + 1), dtype=np.int64)
    for i, (qx, qy) in enumerate(per):
        d = math.hypot(qx - cx, qy - cy)
        px, py = cx + radius * (qx - cx) / d, cy + radius * (qy - cy) / d
        for j in range(mr + 1):
            s = j / mr
            ring[i, j] = nodes.add(px + s * (qx - px), py + s * (qy - py)) if j < mr else nodes.add(qx, qy)
    # blocks outside the box
    xb = [(0.0, x0), (x0, x1), (x1, length)]
    yb = [(0.0, y0), (y0, y1), (y1, height)]
    blocks = []
    for bj, (ya, yb_) in enumerate(yb):
        for bi, (xa, xb_) in enumerate(xb):
            if bi == 1 and bj == 1:
                continue
            nxb = m if bi == 1 else max(1, int(round((xb_ - xa) / hs)))
            nyb = m if bj == 1 else max(1, int(round((yb_ - ya) / hs)))
            ids = np.empty((nyb + 1, nxb + 1), dtype=np.int64)
            for j in range(nyb + 1):
                for i in range(nxb + 1):
                    ids[j, i] = nodes.add(xa + (xb_ - xa) * i / nxb, ya + (yb_ - ya) * j / nyb)
            blocks.append(ids)
    xy = np.array(nodes.pts, dtype=np.float64)
    for i in range(4 * m):
        i2 = (i + 1) % (4 * m)
        for j in range(mr):
            add_quad(ring[i, j], ring[i2, j], ring[i2, j + 1], ring[i, j + 1], xy)
        curved.append((ring[i, 0], ring[i2, 0], 0))
        dirichlet.append((ring[i, 0], ring[i2, 0]))
    for ids in blocks:
        nyb, nxb = ids.shape[0] - 1, ids.shape[1] - 1
        for j in range(nyb):
            for i in range(nxb):
                add_quad(ids[j, i], ids[j, i + 1], ids[j + 1, i + 1], ids[j + 1, i], xy)
        for j in range(nyb):
            for i in (0, nxb):
                a, b = ids[j, i], ids[j + 1, i]
                if abs(xy[a, 0]) < 1e-12 and abs(xy[b, 0]) < 1e-12:
                    dirichlet.append((a, b))
        for i in range(nxb):
            for j in (0, nyb):
                a, b = ids[j, i], ids[j, i + 1]
                if (abs(xy[a, 1]) < 1e-12 and abs(xy[b, 1]) < 1e-12) or \
                   (abs(xy[a, 1] - height) < 1e-12 and abs(xy[b, 1] - height) < 1e-12):
                    dirichlet.append((a, b))
    return UMesh(xy, np.array(elems, dtype=np.int32), np.array(dirichlet, dtype=np.int32),
                 np.array([[cx, cy, radius]], dtype=np.float64), np.array(curved, dtype=np.int32))


def cylinder_channel_flow(m=8, field_seed=1, dt=0.005, inflow_max=1.5) -> UFlow:
    mesh = cylinder_channel_umesh(m)
    ff = FourierField(CHANNEL_LX, CHANNEL_LY, field_seed).calibrate(mesh.xy)
    c = mesh.circles[0]
    return UFlow(mesh, dt, ff, inflow_max=inflow_max, hole=(c[0], c[1], c[2]))


def structured_as_umesh(cxy, dirichlet, order_seed=None, rotate_seed=None, renumber_seed=None):
    """A structured mesh (ny+1, nx+1, 2) as an unstructured one.  Element e of
    the structured mesh (row-major) becomes element order[e] with its corners
    c00, c10, c11, c01 cyclically shifted by rot[e] places; coarse node c
    becomes node perm[c].  Returns (UMesh, order, rot, perm); None seeds leave
    that part unchanged (identity)."""
    ny, nx = cxy.shape[0] - 1, cxy.shape[1] - 1
    nc, P = (nx + 1) * (ny + 1), nx * ny
    perm = np.arange(nc) if renumber_seed is None else np.random.default_rng(renumber_seed).permutation(nc)
    order = np.arange(P) if order_seed is None else np.random.default_rng(order_seed).permutation(P)
    rot = np.zeros(P, dtype=np.int64) if rotate_seed is None else np.random.default_rng(rotate_seed).integers(0, 4, P)
    xy = np.empty((nc, 2))
    xy[perm] = cxy.reshape(-1, 2)
    elems = np.empty((P, 4), dtype=np.int32)
    for j in range(ny):
        for i in range(nx):
            e = j * nx + i
            c = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
            c = [perm[k] for k in c]
            r = rot[e]
            elems[order[e]] = c[r:] + c[:r]
    dirs = []
    for j in range(ny + 1):
        for i in range(nx + 1):
            a = j * (nx + 1) + i
            if i < nx and ((j == 0 and dirichlet & DIR_YMIN) or (j == ny and dirichlet & DIR_YMAX)):
                dirs.append((perm[a], perm[a + 1]))
            if j < ny and ((i == 0 and dirichlet & DIR_XMIN) or (i == nx and dirichlet & DIR_XMAX)):
                dirs.append((perm[a], perm[a + nx + 1]))
    mesh = UMesh(xy, elems, np.array(dirs, dtype=np.int32).reshape(-1, 2), np.zeros((0, 3)),
                 np.zeros((0, 3), dtype=np.int32))
    return mesh, order, rot, perm
