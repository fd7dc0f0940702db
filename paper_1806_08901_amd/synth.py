"""Seeded synthetic fields shaped like the paper's workloads.

The paper evaluates on NYX (3-D cosmology), ATM (2-D climate, 79 fields of
1800 x 3600) and Hurricane (3-D, 13 fields of 100 x 500 x 500) (Section 6.1,
Table 1 and Section 6.3.2).  Those datasets are not available here; these
generators produce fields of the same shapes, counts and dtypes with
controllable smoothness instead.  Values are synthetic, not dataset values.

This module holds NO arithmetic of the estimator: it only makes inputs.  Both
the HIP path and the CPU oracle consume the same bytes produced here.
Generation uses torch so that large fields can be made directly in HBM; pass
``device="cpu"`` for CPU-only use.
"""
from __future__ import annotations

import math

import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def gaussian_bumps(shape=(64, 64, 64), nbumps=8, sigma_range=(4.0, 16.0), noise=1e-3,
                   seed=0, device="cpu", dtype=torch.float32) -> torch.Tensor:
    """Sum of ``nbumps`` Gaussian bumps (centres uniform in the box, widths
    uniform in ``sigma_range`` cells, amplitudes U(-1, 1)) plus N(0, noise^2)."""
    g = _gen(seed, device)
    nd = len(shape)
    centres = torch.rand(nbumps, nd, generator=g, device=device, dtype=torch.float64)
    centres = centres * torch.tensor(shape, device=device, dtype=torch.float64)
    lo, hi = sigma_range
    sig = lo + (hi - lo) * torch.rand(nbumps, generator=g, device=device, dtype=torch.float64)
    amp = 2.0 * torch.rand(nbumps, generator=g, device=device, dtype=torch.float64) - 1.0
    axes = [torch.arange(n, device=device, dtype=torch.float64) for n in shape]
    out = torch.zeros(shape, device=device, dtype=torch.float64)
    for b in range(nbumps):
        r2 = torch.zeros(shape, device=device, dtype=torch.float64)
        for k in range(nd):
            view = [1] * nd
            view[k] = shape[k]
            r2 = r2 + ((axes[k] - centres[b, k]) ** 2).view(view)
        out += amp[b] * torch.exp(-r2 / (2.0 * sig[b] ** 2))
    out += noise * torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    return out.to(dtype).contiguous()


def spectral(shape, slope=-5.0 / 3.0, kmax=64.0, noise=0.01, seed=0, device="cpu",
             dtype=torch.float32) -> torch.Tensor:
    """Random-phase Fourier modes with amplitude |k|^slope for 1 <= |k| <= kmax
    (zero elsewhere), normalised to zero mean and unit standard deviation, plus
    white noise of standard deviation ``noise``."""
    g = _gen(seed, device)
    nd = len(shape)
    freqs = []
    for k, n in enumerate(shape):
        f = torch.fft.rfftfreq(n, device=device) if k == nd - 1 else torch.fft.fftfreq(n, device=device)
        freqs.append((f * n).to(torch.float32))
    spec_shape = list(shape[:-1]) + [shape[-1] // 2 + 1]
    kk = torch.zeros(spec_shape, device=device, dtype=torch.float32)
    for k in range(nd):
        view = [1] * nd
        view[k] = spec_shape[k]
        kk = kk + freqs[k].view(view) ** 2
    kk = kk.sqrt_()
    amp = torch.where((kk >= 1.0) & (kk <= kmax), kk.clamp_min(1.0).pow(slope), torch.zeros_like(kk))
    del kk
    phase = torch.rand(spec_shape, generator=g, device=device, dtype=torch.float32) * (2.0 * math.pi)
    spec = torch.polar(amp, phase)
    del amp, phase
    f = torch.fft.irfftn(spec, s=tuple(shape))
    del spec
    f = f - f.mean()
    sd = f.std()
    if float(sd) > 0:
        f = f / sd
    f = f + noise * torch.randn(tuple(shape), generator=g, device=device, dtype=f.dtype)
    return f.to(dtype).contiguous()


def spiky_constant(shape, frac=1e-3, seed=0, device="cpu", dtype=torch.float32) -> torch.Tensor:
    """A constant c ~ U(-1, 1) plus N(0, 1) spikes at a fraction ``frac`` of
    the points (the mostly-constant fields of the 2-D batch).

    Built on the CPU for every device: a spike position drawn twice is
    written twice, and only the CPU's in-order writes make the field the
    same on every run."""
    g = _gen(seed, "cpu")
    c = 2.0 * torch.rand((), generator=g, dtype=torch.float64) - 1.0
    n = 1
    for s in shape:
        n *= s
    f = torch.full((n,), float(c), dtype=torch.float64)
    k = max(1, int(round(frac * n)))
    idx = torch.randint(0, n, (k,), generator=g)
    f[idx] += torch.randn(k, generator=g, dtype=torch.float64)
    return f.view(*shape).to(dtype).contiguous().to(device)


# ---------------------------------------------------------------------------
# The five workloads.  Seeds: 1000 * workload + field index.
# ---------------------------------------------------------------------------

EB_SWEEP = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)


def workload_bumps64(device="cpu"):
    """One 64^3 FP32 field of 8 Gaussian bumps plus 1e-3 noise; eb_rel 1e-4;
    every block sampled."""
    return gaussian_bumps((64, 64, 64), seed=1000, device=device)


def workload_turb512(device="cpu", n=512):
    """One n^3 FP32 turbulent-like field (k^-5/3, |k| <= 64, 1% white noise)."""
    return spectral((n, n, n), slope=-5.0 / 3.0, kmax=64.0, noise=0.01, seed=2000, device=device)


def workload_atm_specs(nfields=79, shape=(1800, 3600)):
    """Field recipes of the 2-D batch: spectral slope U[-4, -1] per field,
    every tenth field mostly constant with sparse spikes, eb_rel drawn from
    {1e-2, 1e-4, 1e-6}.  Returns a list of dicts (no tensors)."""
    g = torch.Generator().manual_seed(3000)
    specs = []
    for i in range(nfields):
        slope = float(-1.0 - 3.0 * torch.rand((), generator=g))
        eb = (1e-2, 1e-4, 1e-6)[int(torch.randint(0, 3, (), generator=g))]
        kind = "spiky" if i % 10 == 9 else "spectral"
        specs.append({"kind": kind, "shape": shape, "slope": slope, "eb": eb, "seed": 3000 + i,
                      "dtype": torch.float32})
    return specs


def workload_mix3d_specs():
    """Field recipes of the uneven 3-D batch: 13 x 100x500x500 FP32,
    6 x 256x384x384 FP64, 4 x 512^3 FP32, 20 x 64^3 FP32; slopes U[-5, -2];
    eb_rel from {1e-2, ..., 1e-6}."""
    g = torch.Generator().manual_seed(4000)
    groups = [((100, 500, 500), torch.float32, 13), ((256, 384, 384), torch.float64, 6),
              ((512, 512, 512), torch.float32, 4), ((64, 64, 64), torch.float32, 20)]
    specs = []
    i = 0
    for shape, dt, cnt in groups:
        for _ in range(cnt):
            slope = float(-2.0 - 3.0 * torch.rand((), generator=g))
            eb = EB_SWEEP[int(torch.randint(0, 5, (), generator=g))]
            specs.append({"kind": "spectral", "shape": shape, "slope": slope, "eb": eb,
                          "seed": 4000 + i, "dtype": dt})
            i += 1
    return specs


def make_field(spec, device="cpu") -> torch.Tensor:
    """Materialise one recipe from the workload_*_specs lists."""
    if spec["kind"] == "spiky":
        return spiky_constant(spec["shape"], seed=spec["seed"], device=device, dtype=spec["dtype"])
    kmax = min(64.0, min(spec["shape"]) / 2.0)
    return spectral(spec["shape"], slope=spec["slope"], kmax=kmax, noise=0.01, seed=spec["seed"],
                    device=device, dtype=spec["dtype"])
