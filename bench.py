"""Benchmark of the 3DGUT rasterizer hot path on one MI355X.

Step = one forward pass of the whole path (project -> bin -> render) over the
1M-Gaussian clustered scene (SH degree 3) seen by two 1920x1080 cameras, a
60-degree pinhole and a 180-degree OpenCV fisheye, issued as one two-camera
batch.  value = rendered megapixels per second (2 x 1920 x 1080 per step),
with the scene and all buffers resident in HBM; the step includes gut_bin's
one host read-back of the pair count.

Also reported on the same line:
  roofline      the compositing kernel (the dominant one; one launch renders
                both views): algorithmic FP32 FLOPs (E_eval x 55, E_eval =
                list entries evaluated per pixel up to its stop, counted by
                the kernel itself) per launch over its average duration from
                HIP events on its stream, against
                the chip's FP32 vector peak; plus its HBM bytes per launch
                from rocprofv3 FETCH_SIZE / WRITE_SIZE counters calibrated on
                kernels of known traffic (profiles/render_traffic.json, made
                by --pmc-summary; null when the kernel's sources have changed
                since the counters were taken)
  stages_ms     per-stage averages (events), Table-2 style
  fwd_bwd_ms_per_view   forward + L1 loss + backward on the fisheye view
                against a target rendered from parameters perturbed by
                N(0, 0.01) (the differentiation workload): median over the
                steps of each step's wall time between synchronisations; the
                mean, max and HIP-event median are in fwd_bwd_detail
  rolling_shutter_3m   stage times of the same forward step on the 3M-particle
                rolling-shutter fisheye 1600x1200 view (context, not the metric)
  generalized_degrees  the same forward step with the generalized Gaussian
                responses of degree 3, 4 and 8 (Supp. A), beside degree 2
  depth_clip    the same forward step with a per-pixel clip distance
                (hybrid rendering, Sec. 6.2)
  kbuffer_sorted  the same forward step rendered with the per-ray k = 16
                buffer ("Ours (sorted)", Sec. 4.3)
  cpu_baseline  the FP64 oracle on this host's cores, timed on whole steps of
                the same two-view batch (projection, binning, every tile)
                until its time budget is spent
"""
from __future__ import annotations

import argparse
import collections
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

F_EVAL = 55            # FP32 FLOPs per (pixel, particle) evaluation (mul and add counted apart)
F_EVAL_GEN = F_EVAL + 4   # degree-n response: (omega^2)^(n/2) as exp2(h log2 w), 2 transcendentals + fma + mul
F_EVAL_CLIP = F_EVAL + 5  # depth clip: o_g.d_g (2 fma), two products and the compare
PEAK_FP32_TFLOPS = 157.3
# the FP32 ceiling without packed-math instructions (256 CUs x 64 lanes x 2 FLOPs x 2.4 GHz),
# which libgut is compiled not to emit
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "render_traffic.json")
RENDER_SOURCES = ("render.hip", "tile_eval.h", "common.h")
CALIB_BYTES = 1 << 30  # the fill writes, and the add reads, exactly this many bytes


def render_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_12507_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def render_launches(cams):
    """Render launches gut_render makes for these cameras: consecutive cameras
    of one shutter type and one tile count share a launch, up to 4 (the
    benchmark's two 1920x1080 global-shutter views take one)."""
    launches, prev, run = 0, None, 0
    for c in cams:
        key = (c.get("shutter", "global"), -(-int(c["width"]) // 16) * -(-int(c["height"]) // 16))
        if key == prev and run < 4:
            run += 1
        else:
            launches, prev, run = launches + 1, key, 1
    return launches


def pmc_summary(fetch_dir, write_dir, out_path, command):
    """Per-launch HBM bytes of the timed render kernel (render_multi_kernel<false,
    false, false, false>: global shutter, no n_eval, Gaussian response, no
    clip, both views in one launch) from two
    rocprofv3 --pmc runs of `bench.py --calib-copy` (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch).
    Each counter is scaled by what it reads for a kernel of known traffic in
    the same run: the 1 GiB add (reads 1 GiB) for FETCH_SIZE and the 1 GiB
    fill (writes 1 GiB) for WRITE_SIZE."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        rows.sort()
        return rows

    def pick(rows, *keys):
        return [v for _, k, v in rows if any(key in k for key in keys)]

    fr, wr = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    f_add = pick(fr, "CUDAFunctor_add", "CUDAFunctorOnSelf_add")
    w_fill = pick(wr, "FillFunctor")
    f_r = pick(fr, "gut::render_multi_kernel<false, false, false, false>")
    w_r = pick(wr, "gut::render_multi_kernel<false, false, false, false>")
    if not (f_add and w_fill and f_r and w_r):
        raise SystemExit("pmc summary: calibration or render dispatches missing")
    ff = CALIB_BYTES / (f_add[0] * 1024.0)
    wf = CALIB_BYTES / (w_fill[0] * 1024.0)
    fetch = float(np.mean(f_r)) * 1024.0 * ff
    write = float(np.mean(w_r)) * 1024.0 * wf
    out = dict(render_kernel_bytes_per_launch=fetch + write, fetch_bytes=fetch, write_bytes=write,
               fetch_factor=ff, write_factor=wf, raw_fetch_kib=float(np.mean(f_r)),
               raw_write_kib=float(np.mean(w_r)), dispatches=len(f_r),
               source_sha256=render_source_hash(), command=command)
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


# Algorithmic bytes of the HBM-bound stages, per step.
# project: each particle's 236 B (SH degree 3) read once per launch of up to
# four cameras; per (camera, particle) 28 B written (rectangle, tiles, depth,
# colour) plus 24 B for tile culling (mean, extent ellipse); the 64 B render
# record per particle.
# bin: per entry its 4 B tile count read by the count and the scatter
# kernels; per visible entry 32 B (rectangle, mean, ellipse) read by each and
# 4 B depth by the scatter; per pair 8 B of key written and read back, 4 B of
# id written; per tile 24 B of counts, starts, ranges and order.
PROJ_CAMS_PER_LAUNCH = 4
# init, count, column scan, list scan, scatter, 4 sorts (three list lengths and the radix fallback); the
# sort of lists of 4096 entries or more is launched only when there are such lists, and the two-view
# benchmark batch has none
BIN_KERNELS = 9


def project_bytes(n, n_cams):
    launches = -(-n_cams // PROJ_CAMS_PER_LAUNCH)
    return launches * 236 * n + n_cams * (28 + 24) * n + 64 * n


def binning_bytes(E, nvis, P, T):
    return 8 * E + (2 * 32 + 4) * nvis + (8 + 8 + 4) * P + 24 * T


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_forward(gs, cams, steps, warmup, R, torch, params=None, clip=None, flush=None):
    """Forward steps back to back (warm).  With `flush` (a tensor larger than
    the 256 MB Infinity Cache) each timed step is preceded by a write of the
    whole tensor, outside the stage events, so every stage starts cold; the
    step time is then the sum of the stage events."""
    proj = R.alloc_projection(gs.n, len(cams), gs.means.device)
    R.project(gs, cams, params, out=proj)
    bins = R.bin_tiles(proj, cams, params)
    img = R.alloc_image(cams, gs.means.device)
    n_ev = 4
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(steps)]

    def step(e=None):
        if e: e[0].record()
        R.project(gs, cams, params, out=proj)
        if e: e[1].record()
        R.bin_tiles(proj, cams, params, bins=bins)
        if e: e[2].record()
        R.render(proj, bins, cams, params, out=img, clip=clip)
        if e: e[3].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # no Python garbage collection inside the timed region (a full collection
    # stalls the host, and with it the launches, for tens of milliseconds)
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for k in range(steps):
        if flush is not None:
            flush.fill_(float(k))
        step(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    st = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(n_ev - 1)] for k in range(steps)])
    ms_step = (t1 - t0) * 1e3 / steps if flush is None else float(st.sum(1).mean())
    # one extra, untimed render that counts evaluations per pixel
    img_eval = R.render(proj, bins, cams, params, with_eval=True, clip=clip)
    torch.cuda.synchronize()
    e_eval = int(img_eval.n_eval.to(torch.int64).sum().item())
    return dict(ms_per_step=ms_step, stage_ms=st.mean(0), stage_p10=np.percentile(st, 10, 0),
                stage_p90=np.percentile(st, 90, 0), e_eval=e_eval, n_pairs=bins.n_pairs,
                n_visible=int((proj.tiles > 0).sum().item()), img=img)


def bench_fwd_bwd(scene, cam, steps, warmup, R, G, torch, params=None):
    """Forward + L1 loss + backward on one view, the differentiation workload."""
    gs = R.GaussianScene.from_host(scene)
    tgt_scene = R.GaussianScene.from_host(G.perturb_raw(scene, seed=3004))
    _, _, timg = R.forward(tgt_scene, [cam], params)
    target = timg.rgb.clone()
    del tgt_scene, timg
    proj = R.alloc_projection(gs.n, 1, gs.means.device)
    R.project(gs, [cam], params, out=proj)
    bins = R.bin_tiles(proj, [cam], params)
    img = R.alloc_image([cam], gs.means.device)
    grads = dict(means=torch.empty_like(gs.means), scales=torch.empty_like(gs.scales),
                 quats=torch.empty_like(gs.quats), opacities=torch.empty_like(gs.opacities),
                 sh=torch.empty_like(gs.sh))
    ws = None
    npx = target.shape[0] * 3

    def step():
        nonlocal ws
        R.project(gs, [cam], params, out=proj)
        R.bin_tiles(proj, [cam], params, bins=bins)
        R.render(proj, bins, [cam], params, out=img)
        d_rgb = torch.sign(img.rgb - target) / npx          # dL/dC of mean |C - C_target|
        if ws is None:
            from paper_2412_12507_amd import _lib as L
            need = L.load().gut_render_bwd_workspace_bytes(gs.n, 1)
            ws = torch.empty(need, dtype=torch.uint8, device=gs.means.device)
        R.render_backward(gs, proj, bins, [cam], img, d_rgb, None, params, grads=grads, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    walls = []
    gc.collect()
    gc.disable()
    for k in range(steps):  # each step bracketed by synchronisations
        t0 = time.perf_counter()
        ev[k][0].record()
        step()
        ev[k][1].record()
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
    gc.enable()
    per = sorted(a.elapsed_time(b) for a, b in ev)
    return dict(ms_per_view=float(np.median(walls)), ms_mean=float(np.mean(walls)),
                ms_max=float(np.max(walls)), gpu_ms_median=per[len(per) // 2])


def _replay_sequential(gs, reqs, arr, render_sequential):
    """Serve the trace one request at a time, at its arrival times: a request
    starts when it has arrived and the previous one has finished, its cameras
    are rendered one after another, synchronously.  Returns per-request
    latencies (s) and the time the last one finished."""
    lat = np.empty(len(reqs))
    t0 = time.perf_counter()
    for i, (a, cams) in enumerate(zip(arr, reqs)):
        d = t0 + a - time.perf_counter()
        if d > 0:
            time.sleep(d)
        render_sequential(gs, cams)
        lat[i] = time.perf_counter() - t0 - a
    return lat, time.perf_counter() - t0


def bench_serving(n_requests, rates, R, G, torch, n_particles=3_000_000, warm=8, check_every=0,
                  check_load=0.9, check_tiles=4, save_checks=None):
    """Serving workload: the 3M-Gaussian scene resident in HBM, Poisson
    arrivals of requests with 1-8 cameras (half pinhole 640x480..3840x2160,
    half 1600x1200 rolling-shutter fisheye).  Capacity is the inverse of the
    sequential baseline's mean service time over the whole trace.  At each
    load the trace is served twice at the same arrival times: by the
    continuous-batching server, and by the sequential baseline replayed on
    the GPU (one request at a time, cameras one after another).  With
    check_every > 0, every check_every-th camera served at check_load keeps
    check_tiles random tiles of its image (with the camera) for an offline
    comparison with the oracle (tests/serve_oracle_check.py)."""
    from paper_2412_12507_amd.serve import Server, render_sequential
    scene = G.config3_scene(n_particles)
    gs = R.GaussianScene.from_host(scene)
    reqs = G.config5_requests(n_requests + warm, seed=3005)
    warm_reqs, reqs = reqs[:warm], reqs[warm:]
    for cams in warm_reqs:
        render_sequential(gs, cams)
    service = []
    for cams in reqs:
        t = time.perf_counter()
        render_sequential(gs, cams)
        service.append(time.perf_counter() - t)
    service = np.array(service)
    cap = 1.0 / service.mean()
    n_cams = np.array([len(c) for c in reqs])
    log(f"[bench] serving: {len(reqs)} requests, sequential capacity {cap:.1f} req/s")
    out = dict(capacity_req_per_s=cap, mean_cameras_per_request=float(n_cams.mean()),
               requests_per_rate=len(reqs), warmup_requests=warm, rates=[])
    checks = []
    rng = np.random.default_rng(3006)
    srv = Server(gs, mem_budget_bytes=48 << 30, max_slots=4, max_batch_cams=8)
    try:
        for cams in warm_reqs:
            rid, _ = srv.submit(cams)
            srv.wait(rid)
        for f in rates:
            lam = f * cap
            arr = G.poisson_arrivals(len(reqs), lam, seed=3005 + int(100 * f))
            keep = check_every > 0 and abs(f - check_load) < 1e-9
            srv.reset_stats()
            pending, picks, lat_s = collections.deque(), {}, []

            def finish(block):
                # collect finished requests in order (their images are freed)
                while pending and (block or srv.poll(pending[0])):
                    rid = pending.popleft()
                    outs = srv.wait(rid)
                    for j, cam in picks.pop(rid, []):
                        tx, ty = -(-int(cam["width"]) // 16), -(-int(cam["height"]) // 16)
                        tiles = np.sort(rng.choice(tx * ty, check_tiles, replace=False))
                        px = [outs[j][(int(t) // tx) * 16:(int(t) // tx) * 16 + 16,
                                      (int(t) % tx) * 16:(int(t) % tx) * 16 + 16].cpu().numpy() for t in tiles]
                        checks.append(dict(cam=cam, tiles=tiles, pixels=px))
                    lat_s.append(srv.latency_ms(rid))

            t0 = time.perf_counter()
            cam_no = 0
            for a, cams in zip(arr, reqs):
                while True:
                    finish(False)
                    d = t0 + a - time.perf_counter()
                    if d <= 0:
                        break
                    time.sleep(min(d, 1e-3))
                rid, _ = srv.submit(cams)
                pending.append(rid)
                if keep:
                    sel = [(j, cam) for j, cam in enumerate(cams) if (cam_no + j) % check_every == 0]
                    if sel:
                        picks[rid] = sel
                cam_no += len(cams)
            finish(True)
            st = srv.stats()
            lat_s = np.array(lat_s)
            log(f"[bench] serving load {f}: server p50 {np.percentile(lat_s, 50):.1f} "
                f"p99 {np.percentile(lat_s, 99):.1f} ms, {st['frames_per_s']:.0f} fps")
            lat_q, span = _replay_sequential(gs, reqs, arr, render_sequential)
            lat_q *= 1e3
            seq = dict(p50_ms=float(np.percentile(lat_q, 50)), p99_ms=float(np.percentile(lat_q, 99)),
                       frames_per_s=float(n_cams.sum() / span))
            log(f"[bench] serving load {f}: sequential replay p50 {seq['p50_ms']:.1f} "
                f"p99 {seq['p99_ms']:.1f} ms")
            out["rates"].append(dict(load=f, arrival_req_per_s=lam,
                                     server=dict(p50_ms=float(np.percentile(lat_s, 50)),
                                                 p99_ms=float(np.percentile(lat_s, 99)),
                                                 frames_per_s=st["frames_per_s"], batches=st["batches"]),
                                     sequential=seq))
    finally:
        srv.close()
    if save_checks and checks:
        import pickle
        with open(save_checks, "wb") as fh:
            pickle.dump(dict(n_particles=n_particles, load=check_load, every=check_every, checks=checks), fh)
        out["oracle_check"] = dict(cameras=len(checks), tiles_per_camera=check_tiles, file=save_checks)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cams, budget_s, O):
    """The FP64 oracle on this host, built here with -O3 -march=native and
    timed on the same step as the GPU (both views: projection, binning and
    every tile rendered) on all the threads it gets, repeated until the time
    budget is spent (whole steps only); then single-threaded on the pinhole
    view: projection, binning and one tile in 16 rendered, extrapolated to
    the whole step."""
    flags = O.use_native()
    threads = O.set_threads(0)
    p = O.default_params()
    osc = O.OScene.from_scene(scene)
    steps, t_proj, t_bin, t_render = 0, 0.0, 0.0, 0.0
    while steps == 0 or t_proj + t_bin + t_render < budget_s:
        for cam in cams:
            t0 = time.perf_counter()
            pr = O.project(osc, cam, p)
            t1 = time.perf_counter()
            ob = O.bin_tiles(pr, cam, p)
            t2 = time.perf_counter()
            O.render(osc, pr, cam, ob, p, alternatives=False)
            t3 = time.perf_counter()
            t_proj += t1 - t0
            t_bin += t2 - t1
            t_render += t3 - t2
        steps += 1
    total = t_proj + t_bin + t_render
    npx = steps * sum(c["width"] * c["height"] for c in cams)
    # one thread, one view, a sample of its tiles
    O.set_threads(1)
    cam = cams[0]
    t0 = time.perf_counter()
    pr = O.project(osc, cam, p)
    t1 = time.perf_counter()
    ob = O.bin_tiles(pr, cam, p)
    t2 = time.perf_counter()
    tx, ty = O.tiles_xy(cam, p)
    sample = np.arange(0, tx * ty, 16, dtype=np.int32)
    O.render(osc, pr, cam, ob, p, alternatives=False, tiles=sample)
    t3 = time.perf_counter()
    O.set_threads(threads)
    t_one = (t1 - t0) + (t2 - t1) + (t3 - t2) * (tx * ty) / len(sample)
    single = cam["width"] * cam["height"] / t_one / 1e6
    return dict(value=npx / total / 1e6, unit="Mpix/s", cores=threads, kind="oracle",
                sample=f"{steps} whole step(s) of the 1M-Gaussian pinhole + fisheye 1920x1080 "
                       f"batch: FP64 projection {t_proj:.1f} s, binning {t_bin:.1f} s, "
                       f"rendering every tile {t_render:.1f} s",
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
                build=flags, single_thread_mpix_per_s=single,
                single_thread_sample=f"pinhole 1920x1080 view on one thread: projection {t1 - t0:.2f} s, "
                                     f"binning {t2 - t1:.2f} s, {len(sample)} of {tx * ty} tiles "
                                     f"rendered in {t3 - t2:.2f} s (scaled to all tiles)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle rendering")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--traffic-json", default=TRAFFIC_JSON,
                    help="JSON with per-launch HBM bytes of the render kernel (from --pmc-summary)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write --traffic-json from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--pmc-command", default="", help="the profiling command, recorded in the JSON")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run two elementwise kernels of known traffic for counter "
                         "calibration: a 1 GiB fill (writes 1 GiB) and a 1 GiB add "
                         "(reads 1 GiB, writes 1 GiB)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--degrees", default="3,4,8",
                    help="generalized-Gaussian degrees (Supp. A) timed on the same forward step")
    ap.add_argument("--no-degrees", action="store_true")
    ap.add_argument("--no-kbuffer", action="store_true",
                    help="skip the k-buffer (\"Ours (sorted)\", Sec. 4.3) timing")
    ap.add_argument("--no-clip", action="store_true",
                    help="skip the hybrid-rendering depth-clip timing (Sec. 6.2)")
    ap.add_argument("--warm-only", action="store_true",
                    help="skip the cold-cache and tile-culling-off repeats of the forward step "
                         "(for counter runs, whose per-dispatch means should see warm steps only)")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 3M-particle rolling-shutter fisheye stage timings")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9,1.1",
                    help="arrival rates as fractions of the sequential baseline's capacity")
    ap.add_argument("--serve-protocol", metavar="OUT_JSON", default=None,
                    help="run only the serving protocol (2000 requests per load after 100 warm-up, "
                         "1 in 50 cameras at load 0.9 kept for the oracle check), write its "
                         "results to OUT_JSON and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.traffic_json, args.pmc_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: libgut renders on a single MI355X "
              "(how the path would shard over GPUs is described, not implemented); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import gut_synth as G
    from paper_2412_12507_amd import raster as R, _lib
    _lib.load()
    torch.cuda.set_device(0)
    if args.serve_protocol:
        res = bench_serving(2000, [float(x) for x in args.serve_loads.split(",")], R, G, torch, warm=100,
                            check_every=50, save_checks=os.path.splitext(args.serve_protocol)[0] + "_checks.pkl")
        with open(args.serve_protocol, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res), flush=True)
        return
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    log("[bench] generating the 1M-Gaussian scene")
    scene = G.config2_scene(args.n)
    cams = G.config2_cameras()
    gs = R.GaussianScene.from_host(scene)
    torch.cuda.synchronize()
    log("[bench] forward steps")
    fw = bench_forward(gs, cams, args.steps, args.warmup, R, torch)
    npx = sum(c["width"] * c["height"] for c in cams)
    value = npx / (fw["ms_per_step"] * 1e-3) / 1e6
    launches = render_launches(cams)
    render_ms_per_launch = fw["stage_ms"][2] / launches
    flops_per_launch = fw["e_eval"] * F_EVAL / launches
    achieved = flops_per_launch / (render_ms_per_launch * 1e-3) / 1e12
    traffic = None
    if args.traffic_json and os.path.exists(args.traffic_json):
        tj = json.load(open(args.traffic_json))
        if tj.get("source_sha256") == render_source_hash():  # else the kernel changed since
            traffic = tj.get("render_kernel_bytes_per_launch")
    roofline = dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=achieved / PEAK_FP32_TFLOPS, traffic=traffic,
                    peak_nonpacked=PEAK_FP32_NONPACKED_TFLOPS,
                    frac_nonpacked=achieved / PEAK_FP32_NONPACKED_TFLOPS,
                    kernel="render_multi_kernel (gut_render, both views in one launch)"
                    if launches == 1 and len(cams) > 1 else "render_kernel (gut_render)",
                    launches_per_step=launches,
                    e_eval_per_launch=fw["e_eval"] / launches, flops_per_eval=F_EVAL,
                    ms_per_launch=render_ms_per_launch)
    del fw["img"]
    n, nc, nvis, P = args.n, len(cams), fw["n_visible"], fw["n_pairs"]
    T = sum(-(-int(c["width"]) // 16) * -(-int(c["height"]) // 16) for c in cams)
    proj_bytes, bin_bytes = project_bytes(n, nc), binning_bytes(n * nc, nvis, P, T)
    stage_roofline = {
        k: dict(bound="hbm", bytes=b, achieved_gbs=b / (ms * 1e-3) / 1e9, peak_gbs=PEAK_HBM_GBS,
                frac=b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS)
        for k, b, ms in (("project", proj_bytes, fw["stage_ms"][0]), ("bin", bin_bytes, fw["stage_ms"][1]))}
    stage_roofline["bin"]["kernels"] = BIN_KERNELS

    cold = rect_only = None
    if not args.warm_only:
        # the same step with every stage cold: a 512 MB write before each step
        # evicts the scene and the buffers from the 256 MB Infinity Cache
        log("[bench] forward steps, cold (Infinity Cache flushed before each step)")
        flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
        fcold = bench_forward(gs, cams, max(3, args.steps // 2), 2, R, torch, flush=flush)
        del flush
        cold = dict(ms_per_step=fcold["ms_per_step"],
                    stages_ms={"project": fcold["stage_ms"][0], "bin": fcold["stage_ms"][1],
                               "render": fcold["stage_ms"][2]},
                    project_frac=proj_bytes / (fcold["stage_ms"][0] * 1e-3) / 1e9 / PEAK_HBM_GBS,
                    bin_frac=bin_bytes / (fcold["stage_ms"][1] * 1e-3) / 1e9 / PEAK_HBM_GBS)
        del fcold

        # the rectangle-only tile lists (tile culling off), for comparison
        log("[bench] forward steps without tile culling")
        frect = bench_forward(gs, cams, max(3, args.steps // 2), 2, R, torch, dict(tile_cull=0))
        rect_only = dict(mpix_per_s=npx / (frect["ms_per_step"] * 1e-3) / 1e6, n_pairs=frect["n_pairs"],
                         e_eval=frect["e_eval"],
                         stages_ms={"project": frect["stage_ms"][0], "bin": frect["stage_ms"][1],
                                    "render": frect["stage_ms"][2]})
        del frect

    # the generalized Gaussian responses of Supp. A on the same forward step
    # (its table trades quality for speed across degrees 2..8)
    degrees = None
    if args.degrees and not args.no_degrees:
        degrees = {"2": dict(mpix_per_s=value, stages_ms={"project": fw["stage_ms"][0],
                                                          "bin": fw["stage_ms"][1],
                                                          "render": fw["stage_ms"][2]},
                             n_pairs=fw["n_pairs"])}
        for d in [int(x) for x in args.degrees.split(",")]:
            log(f"[bench] forward steps, response of degree {d}")
            fd = bench_forward(gs, cams, max(3, args.steps // 2), 2, R, torch, dict(kernel_degree=d))
            ach = fd["e_eval"] * F_EVAL_GEN / launches / (fd["stage_ms"][2] / launches * 1e-3) / 1e12
            degrees[str(d)] = dict(mpix_per_s=npx / (fd["ms_per_step"] * 1e-3) / 1e6,
                                   stages_ms={"project": fd["stage_ms"][0], "bin": fd["stage_ms"][1],
                                              "render": fd["stage_ms"][2]},
                                   n_pairs=fd["n_pairs"], e_eval=fd["e_eval"],
                                   roofline=dict(bound="alu", achieved=ach, peak=PEAK_FP32_TFLOPS,
                                                 unit="TFLOP/s", frac=ach / PEAK_FP32_TFLOPS,
                                                 flops_per_eval=F_EVAL_GEN))
            del fd
        degrees["2"]["e_eval"] = fw["e_eval"]

    # hybrid rendering (Sec. 6.2): the same step with a per-pixel clip
    # distance, U[6, 10] (the clusters span distances 3..13 from the cameras)
    depth_clip = None
    if not args.no_clip:
        log("[bench] forward steps with a per-pixel depth clip")
        g = torch.Generator(device="cuda").manual_seed(4003)
        clip = 6.0 + 4.0 * torch.rand(npx, device="cuda", generator=g)
        fc = bench_forward(gs, cams, max(3, args.steps // 2), 2, R, torch, None, clip)
        ach = fc["e_eval"] * F_EVAL_CLIP / (fc["stage_ms"][2] * 1e-3) / 1e12
        depth_clip = dict(mpix_per_s=npx / (fc["ms_per_step"] * 1e-3) / 1e6,
                          stages_ms={"project": fc["stage_ms"][0], "bin": fc["stage_ms"][1],
                                     "render": fc["stage_ms"][2]},
                          e_eval=fc["e_eval"], clip="U[6, 10] per pixel",
                          roofline=dict(bound="alu", achieved=ach, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                                        frac=ach / PEAK_FP32_TFLOPS, flops_per_eval=F_EVAL_CLIP))
        del fc, clip

    # "Ours (sorted)" (Sec. 4.3): the same step with the per-ray k-buffer, k = 16
    kbuffer = None
    if not args.no_kbuffer:
        log("[bench] forward steps with the k = 16 per-ray buffer")
        fk = bench_forward(gs, cams, max(3, args.steps // 2), 2, R, torch, dict(kbuffer=16))
        kbuffer = dict(k=16, mpix_per_s=npx / (fk["ms_per_step"] * 1e-3) / 1e6,
                       stages_ms={"project": fk["stage_ms"][0], "bin": fk["stage_ms"][1],
                                  "render": fk["stage_ms"][2]},
                       e_eval=fk["e_eval"])
        del fk
        # Supp. A's table times the generalized kernels with the sorted variant
        if args.degrees and not args.no_degrees:
            kbuffer["degrees"] = {}
            for d in [int(x) for x in args.degrees.split(",")]:
                log(f"[bench] forward steps, k = 16 per-ray buffer, response of degree {d}")
                fk = bench_forward(gs, cams, max(3, args.steps // 4), 1, R, torch, dict(kbuffer=16, kernel_degree=d))
                kbuffer["degrees"][str(d)] = dict(mpix_per_s=npx / (fk["ms_per_step"] * 1e-3) / 1e6,
                                                  render_ms=fk["stage_ms"][2])
                del fk

    fwd_bwd = None
    if not args.no_fwd_bwd:
        log("[bench] fwd+bwd on the fisheye view")
        fwd_bwd = bench_fwd_bwd(scene, cams[1], max(3, args.steps // 2), 2, R, G, torch)
        if kbuffer is not None:
            log("[bench] fwd+bwd on the fisheye view, k = 16 per-ray buffer")
            kb = bench_fwd_bwd(scene, cams[1], max(3, args.steps // 4), 1, R, G, torch, dict(kbuffer=16))
            kbuffer["fwd_bwd_ms_per_view"] = kb["ms_per_view"]

    c3 = None
    if not args.no_c3:
        log("[bench] 3M-particle rolling-shutter fisheye view")
        del gs
        torch.cuda.empty_cache()
        gs3 = R.GaussianScene.from_host(G.config3_scene())
        cam3 = [G.config3_camera()]
        f3 = bench_forward(gs3, cam3, max(3, args.steps // 2), 2, R, torch)
        c3 = dict(workload="3M clustered Gaussians, rolling-shutter OpenCV fisheye 1600x1200",
                  mpix_per_s=1600 * 1200 / (f3["ms_per_step"] * 1e-3) / 1e6,
                  stages_ms={"project": f3["stage_ms"][0], "bin": f3["stage_ms"][1],
                             "render": f3["stage_ms"][2]},
                  n_pairs=f3["n_pairs"], n_visible=f3["n_visible"])
        del gs3, f3
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serve:
        log("[bench] serving")
        gs = None
        torch.cuda.empty_cache()
        serving = bench_serving(args.serve_requests, [float(x) for x in args.serve_loads.split(",")],
                                R, G, torch)
        top = max(serving["rates"], key=lambda r: r["load"])
        serving["p50_ms"] = top["server"]["p50_ms"]
        serving["p99_ms"] = top["server"]["p99_ms"]

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline")
        import oracle as O
        cpu = cpu_baseline(scene, cams, args.cpu_budget, O)

    out = {
        "metric": "Mpix/s fwd, fwd+bwd ms/view @1M Gaussians; serving p50/p99 ms",
        "value": value,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fw["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M clustered Gaussians (SH degree 3), pinhole + 180-deg fisheye "
                               "1920x1080, one two-camera batch per step",
                   "n_gaussians": args.n, "views": 2, "width": 1920, "height": 1080},
        "roofline": roofline,
        "stages_ms": {"project": fw["stage_ms"][0], "bin": fw["stage_ms"][1],
                      "render": fw["stage_ms"][2]},
        "stage_roofline": stage_roofline,
        "stages_cold": cold,
        "tile_cull_off": rect_only,
        "n_pairs": fw["n_pairs"],
        "n_visible": fw["n_visible"],
        "fwd_bwd_ms_per_view": fwd_bwd["ms_per_view"] if fwd_bwd else None,
        "fwd_bwd_detail": fwd_bwd,
        "rolling_shutter_3m": c3,
        "generalized_degrees": degrees,
        "depth_clip": depth_clip,
        "kbuffer_sorted": kbuffer,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
