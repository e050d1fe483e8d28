"""Seeded synthetic snapshot workloads for the TOI imaging path.

This module only *produces inputs*: antenna layouts, per-snapshot baseline
coordinates, point-source skies, visibilities predicted with the measurement
equation, thermal noise, flags and antenna gains.  It contains none of the
imager's arithmetic (no basis estimation, gridding, Fourier inversion,
re-projection or tLISI) and it is shared, unchanged, by the FP64 oracle's
tests, the GPU parity tests and the benchmark.

The measurement set the paper images is not available, so every workload is
synthetic with the shapes of the paper's data (Measurement-Set layout of
§3.5: UVW in metres per row, DATA as complex64 ``[row][chan][corr]``, FLAG as
one byte per ``[row][chan][corr]``, optional WEIGHT_SPECTRUM, CHAN_FREQ).

Geometry.  Antennas are uniform in a disk (east, north) with Gaussian
heights.  Local ENU offsets are rotated to the equatorial XYZ frame for the
site latitude and then to (u, v, w) for hour angle H and declination
delta (the standard rotation, Thompson, Moran & Swenson, *Interferometry and
Synthesis in Radio Astronomy*, 3rd ed., eqs. 4.1 and 4.15).  Visibilities are
``V = sum_s S_s exp(-i 2 pi (u l_s + v m_s + w (n_s - 1)))`` with ``(u,v,w)``
in wavelengths, the visibility equation of the paper's introduction.

Randomness.  Every stream is drawn from numpy's PCG64 seeded by the tuple
``(seed, stream, index)`` so that any snapshot of any workload is
reproducible on its own, on the host, without generating its predecessors.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 299_792_458.0          # m/s
SIDEREAL_RATE = 7.292115855e-5   # rad/s (Earth rotation w.r.t. the stars)

# stream identifiers for the seeded generators
_S_ARRAY, _S_SKY, _S_NOISE, _S_FLAGS, _S_GAINS, _S_VAR = range(6)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and content recipe of one synthetic imaging workload."""
    name: str
    n_ant: int
    diameter_m: float
    sigma_h_m: float
    n_chan: int
    freq0_hz: float          # lower edge of the band
    dfreq_hz: float          # channel width (channel centres at freq0 + (c + 1/2) dfreq)
    n_corr: int              # 1 (Stokes I) or 4 (XX, XY, YX, YY)
    n_pix: int
    cell_arcsec: float
    n_steady: int
    flux_law: str            # "uniform" (U[lo, hi]) or "powerlaw" (dN/dS ~ S^-1.5 on [lo, hi])
    flux_lo: float
    flux_hi: float
    noise_sigma: float       # Jy per real/imag part per correlation
    n_snap: int
    forced_planes: tuple     # (n_slab, cheb_k); (0, 0) = automatic selection
    seed: int
    lat_deg: float = -30.7
    dec_deg: float = -30.0
    ha0_h: float = -3.0
    dump_s: float = 8.0
    transient_flux: float = 0.0          # C1: one transient present in snapshot 0
    pulsar_flux: float = 0.0             # on/off pulsar amplitude (Jy)
    pulsar_period: int = 12
    pulsar_ramp: float = 1.0             # amplitude multiplier reached at the last snapshot
    n_faint_transients: int = 0
    flag_frac_max: float = 0.0           # per snapshot flagged fraction ~ U[0, max]
    with_gains: bool = False

    @property
    def n_row(self) -> int:
        return self.n_ant * (self.n_ant - 1) // 2

    @property
    def n_vis(self) -> int:
        return self.n_row * self.n_chan

    @property
    def cell_rad(self) -> float:
        return self.cell_arcsec / 3600.0 * math.pi / 180.0

    @property
    def cell_deg(self) -> float:
        return self.cell_arcsec / 3600.0


def _ch_width(lo_hz, hi_hz, n):
    return (hi_hz - lo_hz) / n


# The workloads: a tiny plain imager, the MeerKAT-shaped single batch, the
# batched uneven-flag stream, the differentiable imager, an AA2-like
# many-slab array and the full FIP-TOI run.
WORKLOADS = {
    "tiny": Workload(
        name="tiny", n_ant=16, diameter_m=1000.0, sigma_h_m=2.0,
        n_chan=64, freq0_hz=856e6, dfreq_hz=1e6, n_corr=1,
        n_pix=256, cell_arcsec=10.0, n_steady=3, flux_law="uniform",
        flux_lo=0.1, flux_hi=1.0, noise_sigma=0.01, n_snap=1,
        forced_planes=(1, 4), seed=0, ha0_h=-1.0, transient_flux=0.05),
    "meerkat": Workload(
        name="meerkat", n_ant=64, diameter_m=8000.0, sigma_h_m=5.0,
        n_chan=4096, freq0_hz=856e6, dfreq_hz=_ch_width(856e6, 1712e6, 4096), n_corr=4,
        n_pix=2048, cell_arcsec=1.5, n_steady=200, flux_law="powerlaw",
        flux_lo=1e-3, flux_hi=1.0, noise_sigma=0.2, n_snap=50,
        forced_planes=(1, 16), seed=1, pulsar_flux=2e-3),
    "batched": Workload(
        name="batched", n_ant=64, diameter_m=8000.0, sigma_h_m=5.0,
        n_chan=4096, freq0_hz=856e6, dfreq_hz=_ch_width(856e6, 1712e6, 4096), n_corr=4,
        n_pix=2048, cell_arcsec=1.5, n_steady=200, flux_law="powerlaw",
        flux_lo=1e-3, flux_hi=1.0, noise_sigma=0.2, n_snap=1500,
        forced_planes=(1, 16), seed=2, pulsar_flux=2e-3, flag_frac_max=0.4),
    "adjoint": Workload(
        name="adjoint", n_ant=64, diameter_m=8000.0, sigma_h_m=5.0,
        n_chan=1024, freq0_hz=856e6, dfreq_hz=_ch_width(856e6, 1712e6, 1024), n_corr=4,
        n_pix=2048, cell_arcsec=1.5, n_steady=200, flux_law="powerlaw",
        flux_lo=1e-3, flux_hi=1.0, noise_sigma=0.2, n_snap=20,
        forced_planes=(1, 16), seed=3, with_gains=True),
    # SKA AA2 (MID)-like non-coplanar array (the many-slab regime of the
    # paper's Chebyshev table: Phi_max ~ 164 gives 17 slabs of K = 16, 272
    # planes): 65 antennas (2080 baselines) in a 4 km disk (every baseline
    # inside the uv extent of the 5.3" cells) with 31.1 m rms heights, which
    # set Phi_max; 128 channels of 1 MHz from 1.2 GHz, a 3 degree field on
    # 2048^2 pixels, phase centre at declination 0.
    "aa2": Workload(
        name="aa2", n_ant=65, diameter_m=4000.0, sigma_h_m=31.1,
        n_chan=128, freq0_hz=1.2e9, dfreq_hz=1e6, n_corr=4,
        n_pix=2048, cell_arcsec=3.0 * 3600.0 / 2048, n_steady=16, flux_law="uniform",
        flux_lo=0.1, flux_hi=1.0, noise_sigma=0.2, n_snap=8,
        forced_planes=(17, 16), seed=5, dec_deg=0.0),
    "full": Workload(
        name="full", n_ant=64, diameter_m=8000.0, sigma_h_m=5.0,
        n_chan=4096, freq0_hz=856e6, dfreq_hz=_ch_width(856e6, 1712e6, 4096), n_corr=4,
        n_pix=4096, cell_arcsec=1.5, n_steady=500, flux_law="powerlaw",
        flux_lo=1e-3, flux_hi=1.0, noise_sigma=0.2, n_snap=1500,
        forced_planes=(1, 16), seed=4, n_faint_transients=5, pulsar_period=12,
        pulsar_ramp=3.0),
}


def scaled(wl: Workload, **changes) -> Workload:
    """A copy of ``wl`` with some fields replaced (smaller test variants)."""
    return dataclasses.replace(wl, **changes)


def rng_for(wl: Workload, stream: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([wl.seed, stream, index])


# ----------------------------------------------------------------------------
# geometry

def antenna_enu(wl: Workload) -> np.ndarray:
    """(n_ant, 3) east/north/up offsets in metres: uniform in a disk, N(0, sigma_h) heights."""
    g = rng_for(wl, _S_ARRAY)
    r = 0.5 * wl.diameter_m * np.sqrt(g.random(wl.n_ant))
    th = 2.0 * math.pi * g.random(wl.n_ant)
    h = g.normal(0.0, wl.sigma_h_m, wl.n_ant) if wl.sigma_h_m > 0 else np.zeros(wl.n_ant)
    return np.stack([r * np.cos(th), r * np.sin(th), h], axis=1)


def baseline_pairs(n_ant: int):
    """Antenna indices (ant1 < ant2) of every baseline, row order (0,1), (0,2), ..."""
    a1, a2 = np.triu_indices(n_ant, k=1)
    return a1.astype(np.int32), a2.astype(np.int32)


def enu_to_xyz(enu: np.ndarray, lat_rad: float) -> np.ndarray:
    e, n, u = enu[..., 0], enu[..., 1], enu[..., 2]
    sl, cl = math.sin(lat_rad), math.cos(lat_rad)
    return np.stack([-sl * n + cl * u, e, cl * n + sl * u], axis=-1)


def xyz_to_uvw(xyz: np.ndarray, ha_rad: float, dec_rad: float) -> np.ndarray:
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    sh, ch = math.sin(ha_rad), math.cos(ha_rad)
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    u = sh * x + ch * y
    v = -sd * ch * x + sd * sh * y + cd * z
    w = cd * ch * x - cd * sh * y + sd * z
    return np.stack([u, v, w], axis=-1)


def hour_angle(wl: Workload, snap: int) -> float:
    return wl.ha0_h * math.pi / 12.0 + snap * wl.dump_s * SIDEREAL_RATE


def snapshot_uvw(wl: Workload, snap: int, enu: Optional[np.ndarray] = None) -> np.ndarray:
    """(n_row, 3) baseline coordinates in metres (ant2 - ant1) at snapshot ``snap``."""
    if enu is None:
        enu = antenna_enu(wl)
    xyz = enu_to_xyz(enu, math.radians(wl.lat_deg))
    a1, a2 = baseline_pairs(wl.n_ant)
    return xyz_to_uvw(xyz[a2] - xyz[a1], hour_angle(wl, snap), math.radians(wl.dec_deg))


def channel_freqs(wl: Workload) -> np.ndarray:
    return wl.freq0_hz + (np.arange(wl.n_chan) + 0.5) * wl.dfreq_hz


# ----------------------------------------------------------------------------
# sky

@dataclasses.dataclass
class Sky:
    l: np.ndarray
    m: np.ndarray
    flux: np.ndarray      # steady flux (Jy)
    var_l: np.ndarray     # variable sources (pulsar / transients)
    var_m: np.ndarray
    var_flux: np.ndarray  # (n_var, n_snap) flux per snapshot


def _positions(g, n, half_width):
    return g.uniform(-half_width, half_width, n), g.uniform(-half_width, half_width, n)


def make_sky(wl: Workload) -> Sky:
    """Steady point sources in the central 80% of the field plus time-variable ones."""
    g = rng_for(wl, _S_SKY)
    half = 0.4 * wl.n_pix * wl.cell_rad
    l, m = _positions(g, wl.n_steady, half)
    if wl.flux_law == "uniform":
        s = g.uniform(wl.flux_lo, wl.flux_hi, wl.n_steady)
    else:  # dN/dS ~ S^-1.5 by inverse CDF on [lo, hi]
        u = g.random(wl.n_steady)
        a, b = wl.flux_lo ** -0.5, wl.flux_hi ** -0.5
        s = (a + u * (b - a)) ** -2.0
    var_l, var_m, var_f = [], [], []
    t = np.arange(wl.n_snap)
    # expected image noise (unit primary-plane Jacobian) for the faint-source recipes
    n_par = 2 if wl.n_corr == 4 else 1
    sigma_img = wl.noise_sigma / math.sqrt(n_par) / math.sqrt(max(wl.n_vis, 1))
    gv = rng_for(wl, _S_VAR)
    if wl.transient_flux > 0:
        vl, vm = _positions(gv, 1, half)
        var_l.append(vl[0]); var_m.append(vm[0])
        var_f.append(np.where(t == 0, wl.transient_flux, 0.0))
    if wl.pulsar_flux > 0 or wl.pulsar_ramp != 1.0:
        vl, vm = _positions(gv, 1, half)
        amp = wl.pulsar_flux if wl.pulsar_flux > 0 else 10.0 * sigma_img
        ramp = 1.0 + (wl.pulsar_ramp - 1.0) * t / max(wl.n_snap - 1, 1)
        on = (t % wl.pulsar_period) < (wl.pulsar_period // 2)
        var_l.append(vl[0]); var_m.append(vm[0])
        var_f.append(np.where(on, amp * ramp, 0.0))
    for _ in range(wl.n_faint_transients):
        vl, vm = _positions(gv, 1, half)
        snr = gv.uniform(5.0, 8.0)
        dur = int(gv.integers(4, 65))
        start = int(gv.integers(0, max(wl.n_snap - dur, 1)))
        var_l.append(vl[0]); var_m.append(vm[0])
        var_f.append(np.where((t >= start) & (t < start + dur), snr * sigma_img, 0.0))
    return Sky(l=l, m=m, flux=s, var_l=np.array(var_l), var_m=np.array(var_m),
               var_flux=np.array(var_f).reshape(len(var_f), wl.n_snap))


def sources_at(sky: Sky, snap: int):
    """(l, m, flux) of every source visible in snapshot ``snap``."""
    if sky.var_flux.size:
        f = sky.var_flux[:, snap]
        on = f != 0
        return (np.concatenate([sky.l, sky.var_l[on]]), np.concatenate([sky.m, sky.var_m[on]]),
                np.concatenate([sky.flux, f[on]]))
    return sky.l, sky.m, sky.flux


# ----------------------------------------------------------------------------
# visibilities

def predict(uvw_m, freq_hz, l, m, flux, n_corr: int, device="cpu", chunk_rows: int = 256):
    """Unpolarised point-source visibilities, complex64 ``[row][chan][corr]``.

    ``XX = YY = I`` and ``XY = YX = 0`` for four correlations; one Stokes-I
    correlation otherwise.  Evaluated in float64 with torch (host or device).
    """
    import torch
    uvw = torch.as_tensor(np.asarray(uvw_m, dtype=np.float64), device=device)
    nu = torch.as_tensor(np.asarray(freq_hz, dtype=np.float64), device=device) / C_LIGHT
    l_t = torch.as_tensor(np.asarray(l, dtype=np.float64), device=device)
    m_t = torch.as_tensor(np.asarray(m, dtype=np.float64), device=device)
    s_t = torch.as_tensor(np.asarray(flux, dtype=np.float64), device=device)
    nm1 = -(l_t * l_t + m_t * m_t) / (1.0 + torch.sqrt(1.0 - l_t * l_t - m_t * m_t))
    n_row, n_chan = uvw.shape[0], nu.shape[0]
    out = torch.zeros((n_row, n_chan, n_corr), dtype=torch.complex64, device=device)
    if l_t.numel() == 0:
        return out
    for r0 in range(0, n_row, chunk_rows):
        r1 = min(n_row, r0 + chunk_rows)
        d = (uvw[r0:r1, 0:1] * l_t[None] + uvw[r0:r1, 1:2] * m_t[None]
             + uvw[r0:r1, 2:3] * nm1[None])                        # (rows, src) metres
        ph = (-2.0 * math.pi) * nu[None, :, None] * d[:, None, :]   # (rows, chan, src)
        v = torch.polar(s_t[None, None, :].expand_as(ph).contiguous(), ph).sum(-1)
        v = v.to(torch.complex64)
        if n_corr == 1:
            out[r0:r1, :, 0] = v
        else:
            out[r0:r1, :, 0] = v
            out[r0:r1, :, n_corr - 1] = v
    return out


def noise(wl: Workload, snap: int, shape) -> np.ndarray:
    g = rng_for(wl, _S_NOISE, snap)
    z = g.standard_normal(tuple(shape) + (2,), dtype=np.float32)
    z *= np.float32(wl.noise_sigma)
    return z.view(np.complex64)[..., 0]


def flags(wl: Workload, snap: int) -> Optional[np.ndarray]:
    """Per-snapshot uniform flagging of a U[0, max] fraction of (baseline, channel) pairs."""
    if wl.flag_frac_max <= 0:
        return None
    g = rng_for(wl, _S_FLAGS, snap)
    frac = g.uniform(0.0, wl.flag_frac_max)
    f2 = (g.random((wl.n_row, wl.n_chan)) < frac).astype(np.uint8)
    return np.repeat(f2[:, :, None], wl.n_corr, axis=2)


def gains(wl: Workload) -> Optional[np.ndarray]:
    """Per-antenna complex gains ``(1 + N(0, 0.05)) exp(i N(0, 0.1))``."""
    if not wl.with_gains:
        return None
    g = rng_for(wl, _S_GAINS)
    amp = 1.0 + g.normal(0.0, 0.05, wl.n_ant)
    ph = g.normal(0.0, 0.1, wl.n_ant)
    return (amp * np.exp(1j * ph)).astype(np.complex64)


def make_snapshot(wl: Workload, snap: int = 0, *, with_noise: bool = True,
                  device="cpu", sky: Optional[Sky] = None, enu=None,
                  apply_gains: bool = True) -> dict:
    """Everything a snapshot imager receives, as host numpy arrays.

    Keys: ``uvw`` f64[n_row][3] m, ``vis`` c64[n_row][n_chan][n_corr],
    ``flag`` u8 same shape or None, ``weight`` None (unit weights),
    ``freq`` f64[n_chan] Hz, ``ant1``/``ant2`` i32[n_row], ``gains`` c64[n_ant]
    or None (per-antenna complex factors the imager applies to each row as
    ``g_ant1 conj(g_ant2)``).
    """
    enu = antenna_enu(wl) if enu is None else enu
    sky = make_sky(wl) if sky is None else sky
    uvw = snapshot_uvw(wl, snap, enu)
    freq = channel_freqs(wl)
    l, m, s = sources_at(sky, snap)
    vis = predict(uvw, freq, l, m, s, wl.n_corr, device=device).cpu().numpy()
    if with_noise and wl.noise_sigma > 0:
        vis += noise(wl, snap, vis.shape)
    a1, a2 = baseline_pairs(wl.n_ant)
    g = gains(wl) if apply_gains else None
    return dict(uvw=uvw, vis=vis, flag=flags(wl, snap), weight=None, freq=freq,
                ant1=a1, ant2=a2, gains=g, snap=snap)
