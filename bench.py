#!/usr/bin/env python3
"""Benchmark of the TOI snapshot-imaging hot path on one MI355X.

One step = one snapshot through the whole path: sample statistics, basis and
plan, gridding of the moment planes, inverse FFT with grid correction and
Chebyshev/slab combination, re-projection, and the tLISI map of the three
youngest images.  Inputs are resident in HBM before the timed region starts
(a pool of distinct synthetic snapshots generated on the device by the seeded
generator and cycled through).  The per-stage breakdown is timed with HIP
events on steps run before the timed region; inside it only the dominant
stage's launches carry events (its average launch duration gives the
roofline figure).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload meerkat] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/snapshot imaged (2016 bl×4096 ch→2048²), batched vs plain; adjoint ms"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pool(wl, n_pool, device):
    """n_pool distinct snapshots of the workload: visibilities predicted on the device,
    thermal noise and flags from the seeded host generator of synth_inputs (the same
    per-snapshot streams as ``synth_inputs.make_snapshot``), so that the oracle can
    regenerate any snapshot the benchmark images from its index alone."""
    import torch

    import synth_inputs as S
    enu, sky = S.antenna_enu(wl), S.make_sky(wl)
    freq_h = S.channel_freqs(wl)
    freq = torch.from_numpy(freq_h).to(device)
    a1, a2 = S.baseline_pairs(wl.n_ant)
    ant1, ant2 = torch.from_numpy(a1).to(device), torch.from_numpy(a2).to(device)
    g = S.gains(wl)
    gains = None if g is None else torch.from_numpy(g).to(device)
    pool = []
    for t in range(n_pool):
        uvw = S.snapshot_uvw(wl, t, enu)
        l, m, s = S.sources_at(sky, t)
        vis = S.predict(uvw, freq_h, l, m, s, wl.n_corr, device=device, chunk_rows=32)
        if wl.noise_sigma > 0:
            vis += torch.from_numpy(S.noise(wl, t, tuple(vis.shape))).to(device)
        f = S.flags(wl, t)
        flag = None if f is None else torch.from_numpy(f).to(device)
        pool.append(dict(uvw=torch.from_numpy(uvw).to(device), vis=vis.contiguous(), flag=flag, weight=None,
                         freq=freq, ant1=ant1, ant2=ant2, gains=gains))
    torch.cuda.synchronize()
    return pool


FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (dense)
FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X FP32 matrix cores (dense)
F16_MFMA_PEAK_TFLOPS = 2500.0     # MI355X fp16 / bf16 matrix cores (dense)


def grid_flops(wl, P):
    """Useful gridding arithmetic per snapshot: each sample adds a complex value times a
    real kernel weight (4 flops) to 8 x 8 cells of each of the P planes."""
    return wl.n_vis * 64 * P * 4


def planes_per_group(K, gp=16):
    """Planes gridded and transformed together (one plane group): a slab's orders,
    split into ceil(K / gp) groups when K > gp."""
    parts = -(-K // gp)
    return -(-K // parts)


def stage_bytes(wl, K, with_flags, occ):
    """HBM bytes per launch of each stage, counting each array a stage must touch once and,
    for the grid planes and the row-pass output, only what holds samples: ``occ`` is
    ``Imager.bin_info()`` of the snapshot (occupied (plane group, tile) pairs, each 8 x 8
    cells of every plane of its group; occupied tile rows, each 8 grid rows of N kept bins
    per plane of its group)."""
    N = wl.n_pix
    ppg = planes_per_group(K)
    vis = wl.n_row * wl.n_chan * wl.n_corr * 8
    flags = wl.n_row * wl.n_chan * wl.n_corr if with_flags else 0
    recs = wl.n_row * wl.n_chan * 32            # one 32-byte gridding record per sample
    tiles = occ["tiles"] * 64 * 8 * ppg
    rows = occ["tile_rows"] * 8 * N * 8 * ppg
    img = N * N * 4
    return {
        "prep": flags + wl.n_chan * 8 + wl.n_row * 24,
        "bin": vis + flags + recs,
        "grid": recs + tiles,
        "fft_rows": tiles + rows,
        "fft_cols": rows + img,
        "reproject": 2 * img,
        "tlisi": 3 * img,
    }


def method_bytes(wl, P, with_flags, adjoint=False):
    """Algorithmic HBM bytes of one snapshot under the method's own decomposition, with
    gridding fused into the row pass and the combination into the column pass: the input
    (visibilities, flags) or, for the adjoint, the gradient written, once; each plane's
    M x N row-pass intermediate written and read once; about six N x N images (t-plane
    written, re-projection read and written, the three tLISI reads) or four for the
    adjoint (image gradient read, t-plane gradient written and read, ...)."""
    N, M = wl.n_pix, 2 * wl.n_pix
    data = wl.n_row * wl.n_chan * wl.n_corr * 8 + (wl.n_row * wl.n_chan * wl.n_corr if with_flags else 0)
    return data + P * 2 * M * N * 8 + (4 if adjoint else 6) * N * N * 4


def hbm_frac(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)


GRIDDER_SOURCES = ("toi_grid.hip", "toi_grid.h", "toi_device.h")


def sources_digest(names=GRIDDER_SOURCES):
    """First 16 hex digits of the SHA-256 of the named kernel sources, concatenated."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(ROOT, "paper_2512_06254_amd", "csrc", n), "rb").read())
    return h.hexdigest()[:16]


ALL_SOURCES = tuple(sorted(n for n in os.listdir(os.path.join(ROOT, "paper_2512_06254_amd", "csrc"))
                           if n.endswith((".hip", ".h", ".cpp"))))


def recorded_traffic(key, sources=GRIDDER_SOURCES, workload="meerkat"):
    """HBM bytes measured by rocprofv3 FETCH_SIZE/WRITE_SIZE (profiles/): the line
    ``traffic_bytes <key>``, or None when the sources it depends on have changed since the
    counters were taken (the digest line ``source_sha256 <names>`` no longer matches)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith(("traffic_bytes ", "source_sha256 ")):
            k, val = line.split(":", 1)
            rec[k.strip()] = val.strip()
    names = "all" if sources == ALL_SOURCES else "+".join(sources)
    if rec.get("source_sha256 " + names) != sources_digest(sources) or f"traffic_bytes {key}" not in rec:
        return None
    return int(rec[f"traffic_bytes {key}"])


def cpu_info():
    """CPU model and the threads the oracle's steps use (numpy element-wise steps and
    FFTs run on one thread; matrix products on the BLAS pool)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl
        pools = [p for p in threadpoolctl.threadpool_info() if p.get("user_api") == "blas"]
        blas = max((p["num_threads"] for p in pools), default=None)
    except Exception:
        pass
    return model, os.cpu_count(), blas


def cpu_baseline(wl, snap_dev, n_slab, K, n_side=16, grid_rows=8, fft_planes=2, comb_rows=256):
    """The FP64 oracle timed on bounded samples of one snapshot of the workload, scaled to a
    whole snapshot (labelled extrapolated):
      * gridded mode (oracle/gridded.py, the path the GPU computes): ES gridding of the
        samples of ``grid_rows`` rows, scaled by rows; inverse FFT and grid correction of
        ``fft_planes`` full planes, scaled by planes; the Chebyshev/slab combination on
        ``comb_rows`` image rows, scaled by rows; re-projection and tLISI on full images;
      * the direct sum (eq. 10 via the moments) on an n_side x n_side pixel sub-grid,
        scaled by pixels.
    Sample selection, basis and plan run on all samples."""
    import numpy as np

    from oracle import fitrig as F
    from oracle import gridded as G
    from oracle import toi as O
    host = {k: (None if v is None else v.cpu().numpy()) for k, v in snap_dev.items()}
    N, M, P = wl.n_pix, 2 * wl.n_pix, n_slab * K
    wall0 = time.perf_counter()
    t0 = time.perf_counter()
    smp = O.select_samples(host)
    bas = O.snapshot_basis(smp.b)
    r = O.rotate(bas.V, smp.b)
    plan = O.make_plan(r[:, 2], bas.V, N, wl.cell_deg, n_slab=n_slab, K=K)
    t_fixed = time.perf_counter() - t0
    # gridded mode
    p, sq = O.slab_of(r[:, 2], plan)
    T_ = O.cheb_T(plan.K, sq)
    X, Y = G.grid_coords(r[:, 0], r[:, 1], M, wl.cell_deg)
    sel = smp.row < grid_rows
    t0 = time.perf_counter()
    grid = G.grid_values((T_[sel] * smp.x[sel, None]).T, X[sel], Y[sel], M)
    t_grid = (time.perf_counter() - t0) * wl.n_row / grid_rows
    t0 = time.perf_counter()
    G.grid_to_image(grid[:fft_planes], N)
    t_fft = (time.perf_counter() - t0) * P / fft_planes
    del grid
    rows = np.linspace(0, N - 1, comb_rows).astype(np.int64)
    mom = np.zeros((plan.n_slab, plan.K, rows.size, N), dtype=np.complex128)
    t0 = time.perf_counter()
    tp_rows = O.image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, N, wl.cell_deg, M=mom, j2=rows)
    t_comb = (time.perf_counter() - t0) * N / comb_rows
    tp = np.zeros((N, N))
    tp[rows] = tp_rows
    t0 = time.perf_counter()
    img, _ = O.reproject(tp, bas.V, N, wl.cell_deg)
    F.tlisi(img, img + 1.0, img, tile=32)
    t_post = time.perf_counter() - t0
    gridded_s = t_fixed + t_grid + t_fft + t_comb + t_post
    # direct sum
    rng = np.random.default_rng(0)
    j1 = np.sort(rng.choice(N, n_side, replace=False))
    j2 = np.sort(rng.choice(N, n_side, replace=False))
    t0 = time.perf_counter()
    O.image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, N, wl.cell_deg, j1=j1, j2=j2)
    t_pix = (time.perf_counter() - t0) / (n_side * n_side)
    direct_s = t_fixed + t_pix * N * N + t_post
    model, ncpu, blas = cpu_info()
    return {
        "value": round(gridded_s * 1e3, 1), "unit": "ms/snapshot", "cores": blas or 1, "kind": "oracle",
        "extrapolated": True, "cpu_model": model, "host_cpus": ncpu,
        "threads": f"BLAS products on {blas} threads; numpy element-wise steps, np.add.at and FFTs on 1",
        "direct_sum_ms_per_snapshot": round(direct_s * 1e3, 1),
        "sample": (f"FP64 oracle on one {wl.name} snapshot ({smp.n} samples): selection, SVD basis and plan on "
                   f"all samples {t_fixed:.1f} s; gridded mode (oracle/gridded.py): ES gridding of the "
                   f"{int(sel.sum())} samples of {grid_rows} rows scaled to {wl.n_row} rows {t_grid:.1f} s, inverse "
                   f"FFT + correction of {fft_planes} of {P} {M}^2 planes scaled to {P} {t_fft:.1f} s, "
                   f"Chebyshev/slab combination on {comb_rows} of {N} rows scaled {t_comb:.1f} s, re-projection "
                   f"and tLISI on full images {t_post:.1f} s -> value; direct sum of eq. 10 at "
                   f"{n_side}x{n_side} pixels ({t_pix:.3f} s/pixel) scaled to {N}^2 pixels -> "
                   f"direct_sum_ms_per_snapshot; wall time of the samples {time.perf_counter() - wall0:.1f} s"),
    }


def time_events(fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def batched_leg(n_batch, reps, device):
    """Uneven flagged snapshots: plain per-snapshot calls vs one captured-graph batch launch."""
    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["batched"]
    n_slab, K = wl.forced_planes
    pool = make_pool(wl, min(8, n_batch), device)
    snaps = [pool[i % len(pool)] for i in range(n_batch)]
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K, tile=32)
    variant, _ = im.tune(pool[0])
    imgs = torch.zeros((n_batch, N, N), dtype=torch.float32, device=device)
    tls = torch.zeros((max(n_batch - 2, 1), TT, TT), dtype=torch.float32, device=device)

    def plain():
        for i, sn in enumerate(snaps):
            im.grid(sn)
            im.image(out=imgs[i])
            if i >= 2:
                im.tlisi(imgs[i - 2], imgs[i - 1], imgs[i], out=tls[i - 2])

    def batched():
        im.image_batch(snaps, imgs, tls)

    plain()
    t0 = time.perf_counter()
    batched()                                   # capture + instantiate + first replay
    torch.cuda.synchronize()
    capture_s = time.perf_counter() - t0
    ms_plain = time_events(plain, reps) / n_batch
    ms_batch = time_events(batched, reps) / n_batch
    kept = [float(1.0 - p["flag"][:, :, 0].float().mean()) for p in pool]
    im.close()
    alg = method_bytes(wl, n_slab * K, True)
    return {"workload": wl.name, "snapshots_per_launch": n_batch, "launches_timed": reps,
            "ms_per_snapshot_batched": round(ms_batch, 4), "ms_per_snapshot_plain": round(ms_plain, 4),
            "hbm_roofline_frac_batched": hbm_frac(alg, ms_batch), "hbm_roofline_frac_plain": hbm_frac(alg, ms_plain),
            "algorithmic_bytes_per_snapshot": alg,
            "first_launch_with_capture_s": round(capture_s, 3), "tuned_variant": variant,
            "kept_sample_fraction": [round(k, 3) for k in kept]}


def ingest_leg(n_snap, reps, device):
    """Host-resident MeerKAT-shaped snapshots (page-locked) imaged with toi_ingest: the
    H2D copy of each snapshot overlaps the imaging of the previous one.  Reports the
    end-to-end ms/snapshot including H2D, the copy alone and the device-resident path."""
    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["meerkat"]
    n_slab, K = wl.forced_planes
    dev = make_pool(wl, 2, device)
    host = []
    for d in dev:
        host.append({k: (None if v is None else v.to("cpu").pin_memory()) for k, v in d.items()})
    snaps = [host[i % 2] for i in range(n_snap)]
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K, tile=32)
    imgs = torch.zeros((n_snap, N, N), dtype=torch.float32, device=device)
    tls = torch.zeros((n_snap - 2, TT, TT), dtype=torch.float32, device=device)
    im.ingest(snaps[:2], imgs[:2])              # staging allocation and warm-up
    torch.cuda.synchronize()
    ms_ingest = time_events(lambda: im.ingest(snaps, imgs, tls), reps) / n_snap
    h2d_bytes = sum(v.numel() * v.element_size() for v in host[0].values() if v is not None)
    dst = {k: torch.empty_like(v, device=device) for k, v in host[0].items() if v is not None}
    ms_copy = time_events(lambda: [dst[k].copy_(v, non_blocking=True) for k, v in host[0].items() if v is not None],
                          reps)

    def resident():
        for i in range(n_snap):
            im.grid(dev[i % 2])
            im.image(out=imgs[i])
            if i >= 2:
                im.tlisi(imgs[i - 2], imgs[i - 1], imgs[i], out=tls[i - 2])

    resident()
    ms_res = time_events(resident, reps) / n_snap
    im.close()
    return {"workload": "meerkat, host-resident page-locked snapshots", "snapshots_per_call": n_snap,
            "ms_per_snapshot_end_to_end": round(ms_ingest, 4), "ms_h2d_copy_per_snapshot": round(ms_copy, 4),
            "h2d_bytes_per_snapshot": h2d_bytes, "h2d_GBps": round(h2d_bytes / (ms_copy * 1e-3) / 1e9, 1),
            "ms_per_snapshot_device_resident": round(ms_res, 4),
            "ms_if_serial": round(ms_copy + ms_res, 4)}


def many_slab_leg(n_snap, reps, device):
    """The AA2-like many-slab regime (17 slabs x K = 16 = 272 planes, 2048^2 images):
    ms/snapshot of the plain path and its stages."""
    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["aa2"]
    n_slab, K = wl.forced_planes
    pool = make_pool(wl, 2, device)
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K, tile=32,
                  max_planes=n_slab * K)
    variant, _ = im.tune(pool[0])
    imgs = torch.zeros((n_snap, N, N), dtype=torch.float32, device=device)

    def run():
        for i in range(n_snap):
            im.grid(pool[i % 2])
            im.image(out=imgs[i])
            if i >= 2:
                im.tlisi(imgs[i - 2], imgs[i - 1], imgs[i])

    run()
    ms = time_events(run, reps) / n_snap
    im.profile(True)
    run()
    prof = im.profile_read()
    im.profile(False)
    info = im.plan_info()
    im.close()
    alg = method_bytes(wl, n_slab * K, False)
    return {"workload": "aa2", "baselines": wl.n_row, "channels": wl.n_chan, "correlations": wl.n_corr,
            "image": f"{N}x{N}", "planes": f"{info['n_slab']} slabs x K={info['K']}", "tuned_variant": variant,
            "ms_per_snapshot": round(ms, 4),
            "hbm_roofline_frac": hbm_frac(alg, ms), "algorithmic_bytes": alg,
            "stages_ms": {k: round(v[0] / v[1], 4) for k, v in prof.items() if v[1]}}


def full_leg(n_snap, reps, device):
    """The full run's snapshot shape: 2016 baselines x 4096 channels x 4 correlations imaged
    at 4096^2 (8192^2 grid, 16 planes) with the tLISI map of 128 x 128 tiles; ms/snapshot of
    the plain path, its stages and its fraction of the HBM roofline."""
    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["full"]
    n_slab, K = wl.forced_planes
    pool = make_pool(wl, 2, device)
    N = wl.n_pix
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K, tile=32)
    variant, _ = im.tune(pool[0])
    ring = [torch.zeros((N, N), dtype=torch.float32, device=device) for _ in range(3)]
    tl = torch.zeros((N // 32, N // 32), dtype=torch.float32, device=device)
    state = {"i": 0}

    def run():
        for _ in range(n_snap):
            i = state["i"]
            im.grid(pool[i % 2])
            im.image(out=ring[i % 3])
            if i >= 2:
                im.tlisi(ring[(i - 2) % 3], ring[(i - 1) % 3], ring[i % 3], out=tl)
            state["i"] = i + 1

    run()
    ms = time_events(run, reps) / n_snap
    im.profile(True)
    run()
    prof = im.profile_read()
    im.profile(False)
    info = im.plan_info()
    im.close()
    alg = method_bytes(wl, n_slab * K, False)
    return {"workload": wl.name, "baselines": wl.n_row, "channels": wl.n_chan, "correlations": wl.n_corr,
            "image": f"{N}x{N}", "grid": f"{2 * N}x{2 * N}", "planes": f"{info['n_slab']} slab x K={info['K']}",
            "tuned_variant": variant,
            "status": info["status"], "ms_per_snapshot": round(ms, 4), "hbm_roofline_frac": hbm_frac(alg, ms),
            "algorithmic_bytes": alg, "stages_ms": {k: round(v[0] / v[1], 4) for k, v in prof.items() if v[1]}}


def detect_cube_leg(n_maps, T, reps, device):
    """Whole-run detection (fitrig_detect_cube) over a synthetic tLISI cube of n_maps maps of
    T x T tiles (the full run's 4096^2 images with 32-pixel tiles: T = 128), with planted
    on/off tiles of period 12; ms per cube and the boxes found."""
    import torch

    from paper_2512_06254_amd import toi as T_
    gen = torch.Generator(device=device).manual_seed(11)
    cube = 1.0 - (torch.randn((n_maps, T, T), generator=gen, device=device) * 0.02).abs()
    tau = torch.arange(n_maps, device=device)
    onoff = torch.where((tau % 12) < 6, 0.55, 0.95)
    for (y, x) in [(10, 20), (11, 21), (70, 90)]:
        cube[:, y, x] = onoff
    im = T_.Imager(T * 32, 0.001, 1, 1, 1, mode=2, tile=32)
    boxes, n = im.detect_cube(cube, n_maps - 1)
    torch.cuda.synchronize()
    ms = time_events(lambda: im.detect_cube(cube, n_maps - 1), reps)
    found = int(n.item())
    # then the pair and the full-resolution position of each candidate, in a
    # synthetic 4096^2 difference with a source in each box
    bx = boxes[:found]
    k = im.strongest_map(cube, bx)
    N = T * 32
    a = torch.randn((N, N), generator=gen, device=device) * 0.01
    b = a + torch.randn((N, N), generator=gen, device=device) * 0.01
    yy, xx = torch.meshgrid(torch.arange(N, device=device), torch.arange(N, device=device), indexing="ij")
    for row in bx.cpu().tolist():
        cx, cy = (row[1] + row[3]) / 2 + 0.3, (row[2] + row[4]) / 2 - 0.2
        b += 0.5 * torch.exp(-0.5 * ((xx - cx) ** 2 + (yy - cy) ** 2) / 1.5 ** 2)
    pos = im.localise(a, b, bx, 135.0, -40.0)
    ms_loc = time_events(lambda: im.localise(a, b, bx, 135.0, -40.0), reps)
    out = {"maps": n_maps, "tiles": f"{T}x{T}", "ms_per_cube": round(ms, 3), "boxes_found": found,
           "boxes": [list(map(int, r)) for r in bx[:8].cpu().tolist()],
           "strongest_map": k[:8].cpu().tolist(),
           "localise_ms": round(ms_loc, 3), "positions_j1_j2": [[round(p[1], 3), round(p[2], 3)]
                                                                for p in pos[:8].cpu().tolist()]}
    im.close()
    return out


def adjoint_leg(reps, device):
    """Forward image and the hand-written adjoint (vis + gain gradients) on the 1024-channel workload."""
    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["adjoint"]
    n_slab, K = wl.forced_planes
    pool = make_pool(wl, 2, device)
    N = wl.n_pix
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K, n_ant=wl.n_ant)
    out = torch.zeros((N, N), dtype=torch.float32, device=device)
    grad = torch.randn((N, N), dtype=torch.float32, device=device)
    gv = torch.empty_like(pool[0]["vis"])
    gg = torch.empty_like(pool[0]["gains"])
    state = {"i": 0}

    def fwd():
        sn = pool[state["i"] % 2]
        im.grid(sn)
        im.image(out=out)

    def bwd():
        import ctypes
        sn = pool[state["i"] % 2]
        desc = T.snapshot_struct(sn)
        im._sync_stream()
        T._check(T.lib().toi_degrid(im.ctx, T._ptr(grad), ctypes.byref(desc), T._ptr(gv), T._ptr(gg)), im.ctx)

    fwd(); bwd()
    torch.cuda.synchronize()
    ms_f = time_events(fwd, reps)
    fwd()
    ms_b = time_events(bwd, reps)
    im.close()
    P = n_slab * K
    alg_f, alg_b = method_bytes(wl, P, False), method_bytes(wl, P, False, adjoint=True)
    return {"workload": wl.name, "baselines": wl.n_row, "channels": wl.n_chan, "image": f"{N}x{N}",
            "ms_forward": round(ms_f, 4), "ms_adjoint": round(ms_b, 4),
            "hbm_roofline_frac_forward": hbm_frac(alg_f, ms_f), "hbm_roofline_frac_adjoint": hbm_frac(alg_b, ms_b),
            "gradients": "vis (complex64, all correlations) and 64 antenna gains"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="meerkat")
    ap.add_argument("--pool", type=int, default=4, help="distinct resident snapshots cycled through")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", type=int, default=None,
                    help="gridder variant of the plain leg instead of the autotuner's choice (the tuner still runs)")
    ap.add_argument("--batch", type=int, default=32, help="snapshots per batched graph launch (0 = skip)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--ingest", type=int, default=8, help="host-resident snapshots per toi_ingest call (0 = skip)")
    ap.add_argument("--many-slab", type=int, default=4, help="AA2-like 272-plane snapshots timed (0 = skip)")
    ap.add_argument("--full", type=int, default=4, help="4096^2 full-run-shape snapshots per timing (0 = skip)")
    ap.add_argument("--detect-cube", type=int, default=1500, help="maps of the whole-run detection cube (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this path has no multi-GPU mode (asked for --gpus {args.gpus}). "
              "Snapshots are independent, so N GPUs would each take a contiguous time block.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth_inputs as S
    from paper_2512_06254_amd import toi as T

    wl = S.WORKLOADS[args.workload]
    device = torch.device("cuda", 0)
    torch.cuda.set_device(device)
    n_slab, K = wl.forced_planes
    P = n_slab * K
    log(f"[bench] generating {args.pool} snapshots of '{wl.name}' on the GPU")
    pool = make_pool(wl, args.pool, device)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, mode=3, n_slab=n_slab, cheb_k=K,
                  n_ant=wl.n_ant, tile=32)
    variant, tune_ms = im.tune(pool[0])
    log(f"[bench] autotuned gridder variant {variant}: " + ", ".join(f"{m:.2f}" for m in tune_ms) + " ms")
    if args.tuning is not None:   # a fixed variant (profiling runs: the same kernels whatever the timing)
        variant = args.tuning
        im.set_tuning(variant)
        log(f"[bench] gridder variant {variant} (--tuning)")
    N = wl.n_pix
    ring = [torch.zeros((N, N), dtype=torch.float32, device=device) for _ in range(3)]
    tl = torch.zeros((N // 32, N // 32), dtype=torch.float32, device=device)

    def step(i):
        im.grid(pool[i % len(pool)])
        im.image(out=ring[i % 3])
        if i >= 2:
            im.tlisi(ring[(i - 2) % 3], ring[(i - 1) % 3], ring[i % 3], out=tl)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    # stage breakdown: every stage's launches timed with HIP events, on steps
    # run before the timed region (each timed launch adds two event records to
    # the stream, which the timed region should not pay for)
    n_stage = max(1, min(args.steps, 10))
    im.profile(True)
    for i in range(args.warmup, args.warmup + n_stage):
        step(i)
    prof_all = im.profile_read()
    im.profile(False)
    occ = im.bin_info()
    sb = stage_bytes(wl, K, wl.flag_frac_max > 0, occ)
    stages = {}
    for name, (tot, n) in prof_all.items():
        if n:
            avg = tot / n
            stages[name] = {"avg_ms": round(avg, 4), "launches": n, "bytes": sb.get(name),
                            "GBps": round(sb[name] / (avg * 1e-3) / 1e9, 1) if name in sb else None}
            measured = recorded_traffic(f"stage {name}", ALL_SOURCES) if wl.name == "meerkat" else None
            stages[name]["measured_bytes"] = measured
            stages[name]["measured_GBps"] = None if measured is None else round(measured / (avg * 1e-3) / 1e9, 1)
    for name, st in stages.items():   # every byte count is one the stage really moves: never above peak
        for key in ("GBps", "measured_GBps"):
            if st.get(key) is not None and st[key] > HBM_PEAK_GBPS:
                log(f"[bench] WARNING stage {name} {key} {st[key]} above the HBM peak")
    if "grid" in stages:
        stages["grid"]["TFLOPs"] = round(grid_flops(wl, P) / (stages["grid"]["avg_ms"] * 1e-3) / 1e12, 2)
    dom = max((s for s in stages if s in sb), key=lambda s: stages[s]["avg_ms"] * stages[s]["launches"])
    log(f"[bench] warmup done ({args.warmup} + {n_stage} stage-timed steps; dominant stage {dom}); "
        f"timing {args.steps} steps")
    # timed region: only the dominant stage's launches carry events, giving
    # its average launch duration over exactly these steps
    t0 = args.warmup + n_stage
    im.profile(True, stages=[dom])
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(t0, t0 + args.steps):
        step(i)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    tot, n = im.profile_read()[dom]
    im.profile(False)
    dom_ms = tot / n
    info = im.plan_info()
    log(f"[bench] {ms:.3f} ms/snapshot; {dom} {dom_ms:.3f} ms per launch; plan n_slab={info['n_slab']} "
        f"K={info['K']} status={info['status']}")

    split16 = not (variant & 4)      # 16 planes per pass: fp16 matrix cores with split operands
    if dom == "grid":
        # 16 planes per pass: products on the fp16 matrix cores beside the vector
        # ALU, the kernel bound by vector-ALU issue (staging, operand splits):
        # "alu" against the FP32 vector peak.  8 planes per pass: FP32 matrix
        # instructions, which share the vector ALU on gfx950.
        ach = grid_flops(wl, P) / (dom_ms * 1e-3) / 1e12
        kname = "k_grid_bins16" if variant & 8 else "k_grid_tiles_mfma"
        bound = "alu" if split16 else "mfma"
        peak = FP32_VECTOR_PEAK_TFLOPS if split16 else FP32_MFMA_PEAK_TFLOPS
        roofline = {"bound": bound, "achieved": round(ach, 2), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                    "traffic": recorded_traffic(kname) if wl.name == "meerkat" else None,
                    "kernel": kname, "algorithmic_flops": grid_flops(wl, P),
                    "avg_launch_ms": round(dom_ms, 4), "launches_timed": n,
                    "frac_of_f16_matrix_peak": round(ach / F16_MFMA_PEAK_TFLOPS, 4) if split16 else None,
                    "note": (("products on the fp16 matrix cores (operands split as hi + lo in fp16, 3 terms, "
                              "FP32 accumulation) beside the vector ALU; bound by vector-ALU issue"
                              + (" and latency (16 x 16 bins: 2 waves per SIMD)" if variant & 8 else ""))
                             if split16 else None)}
    else:
        ach = sb[dom] / (dom_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": dom,
                    "algorithmic_bytes": sb[dom], "avg_launch_ms": round(dom_ms, 4), "launches_timed": n}
    alg = method_bytes(wl, P, wl.flag_frac_max > 0)
    impl = recorded_traffic("step", ALL_SOURCES) if wl.name == "meerkat" else None
    roofline_step = {"bound": "hbm", "algorithmic_bytes": alg, "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": hbm_frac(alg, ms),
                     "implementation_bytes": impl,
                     "implementation_GBps": None if impl is None else round(impl / (ms * 1e-3) / 1e9, 1),
                     "note": "algorithmic bytes of the method's fused decomposition (input once, each plane's "
                             "M x N row-pass intermediate written and read once, ~6 images) over the whole "
                             "step; implementation bytes: rocprofv3 FETCH_SIZE + WRITE_SIZE of every kernel "
                             "of one step, null when any kernel source changed since they were taken"}
    fp32 = [tune_ms[v] for v in range(len(tune_ms)) if v & 4]
    b16 = [tune_ms[v] for v in range(len(tune_ms)) if not v & 4]
    bins8 = [tune_ms[v] for v in range(len(tune_ms)) if not v & 12]
    bins16 = [tune_ms[v] for v in range(len(tune_ms)) if v & 8]
    out = {
        "metric": METRIC, "value": round(ms, 4), "unit": "ms/snapshot", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "baselines": wl.n_row, "channels": wl.n_chan, "correlations": wl.n_corr,
                   "image": f"{N}x{N}", "cell_arcsec": wl.cell_arcsec, "planes": f"{n_slab} slab x K={K}",
                   "grid": f"{2 * N}x{2 * N} ES support 8", "tlisi_tile": 32, "path": "plain per-snapshot",
                   "pool": args.pool,
                   "arithmetic": ("FP32 values and sums; gridder products from FP32 operands split as hi + lo "
                                  "in fp16 (about 22 significant bits), 3 terms, FP32 accumulation"
                                  if split16 else "FP32 values, products and sums")},
        "roofline": roofline,
        "roofline_step": roofline_step,
        "stages": stages,
        "stages_note": (f"every stage timed on {n_stage} steps before the timed region; bytes: what the stage "
                        f"must move, grid planes and row-pass output counted only where they hold samples "
                        f"({occ['tiles']} occupied (plane group, tile) pairs, {occ['tile_rows']} tile rows, "
                        f"{occ['entries']} bin entries, {occ['units']} split units); measured: rocprofv3 "
                        f"FETCH_SIZE + WRITE_SIZE (profiles/), null when stale"),
        "tuning": {"variant": variant, "grid_plus_image_ms_per_variant": [round(m, 3) for m in tune_ms],
                   "variants": "bits 0-1 work-unit size 32 << bits items; bit 2 8 planes per pass on the FP32 "
                               "matrix cores instead of 16 on the fp16 matrix cores (split operands); bit 3 "
                               "bins of 16 x 16 cells instead of 8 x 8 (16 planes per pass)",
                   "best_ms_f16x3_16_planes": round(min(b16), 3),
                   "best_ms_f16x3_8x8_bins": round(min(bins8), 3),
                   "best_ms_f16x3_16x16_bins": round(min(bins16), 3) if bins16 else None,
                   "best_ms_fp32_8_planes": round(min(fp32), 3)},
    }
    im.close()
    if args.batch > 0:
        log(f"[bench] batched leg: {args.batch} uneven snapshots per graph launch")
        out["batched"] = batched_leg(args.batch, 2, device)
    if args.ingest > 0:
        log(f"[bench] ingest leg: {args.ingest} host-resident snapshots per call")
        out["ingest"] = ingest_leg(args.ingest, 2, device)
    if args.many_slab > 0:
        log(f"[bench] many-slab leg (AA2-like, 272 planes): {args.many_slab} snapshots")
        out["many_slab"] = many_slab_leg(args.many_slab, 2, device)
    if args.full > 0:
        log(f"[bench] full-run shape leg (4096^2 images): {args.full} snapshots per timing")
        out["full"] = full_leg(args.full, 2, device)
    if args.detect_cube > 0:
        log(f"[bench] whole-run detection leg: {args.detect_cube} tLISI maps of 128 x 128 tiles")
        out["detect_cube"] = detect_cube_leg(args.detect_cube, 128, 3, device)
    if not args.no_adjoint:
        log("[bench] adjoint leg")
        out["adjoint"] = adjoint_leg(max(3, args.steps // 4), device)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(wl, pool[0], n_slab, K)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
