#!/usr/bin/env python3
"""Benchmark of the 14-addition approximate-DCT block codec on one MI355X.

A step is one pass of the whole hot path over the batch of 64 uint8 images of
4096 x 4096 (per-image Q_ij = 1 + s (i + j)): one persistent launch of the
fused forward + quantise kernel over all 64 images, then one persistent launch
of the fused dequantise + inverse kernel (int16 coefficients in between).
`value` is pixels per second of that step (Gpixel/s, encode + decode), with
inputs resident in HBM before the timed region starts.

The JSON line also carries:
  roofline      the dominant kernel's algorithmic HBM bytes (3 B/px: 1 in,
                2 out for the encoder; 2 in, 1 out for the decoder) per launch
                over its average launch time, measured with HIP events on the
                launch stream, against the 8 TB/s HBM peak;
  cpu_baseline  the CPU oracle (dense 8x8 integer products) encoding and
                decoding a bounded sample of the same images on the host cores
                (and on one core);
and, unless --no-extras:
  fused_roundtrip  encode + decode fused with no coefficients in HBM;
  per_image     the same 64-image batch with one plain launch per image;
  forward       the int32 forward transform alone over the same batch (5 B/px);
  plain         the plain encode and decode calls on one image of 4096^2,
                8192^2 and 16384^2;
  latency_512   one 512 x 512 image: per-call latency of each plain entry
                point, and the PSNR of a zonal keep-10 reconstruction;
  ceiling       stream probes: the part's practical copy/read/write rates for
                the codec's access mixes (1:1, 1:2, 2:1, 1:3);
  video         256 4:2:0 frames to int8 zigzag, one graph vs one launch per plane;
  batched       10,000 ragged images as one persistent launch replayed from a
                hipGraph vs one plain launch per image;
  serving       Poisson request streams (60 s per rate) served by the resident
                kernel and with a plain launch per request, and (shorter) with
                continuous batching into launched kernels, with a plain launch
                per request over that same shorter trace, and with host payloads
                over PCIe: p50/p99/p99.9 latency, the tail's make-up, Gpixel/s,
                and the capacity of each form under a burst;
  quality       the zonal-coding sweep against the exact DCT (--no-quality
                skips it).
config.leg_seconds gives the wall time of each part of the run.
cpu_baseline also holds the oracle beside the 512 x 512 latency leg, the
ragged batch and the video frames, and its check of the served outputs (a
seeded 1 % of each trace plus every request of 32 Mpx or more).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The workloads by number (the 64 x 4096^2 step always runs): the extra legs
# each one adds.
CONFIG_LEGS = {1: "latency_512", 2: "", 3: "batched", 4: "video", 5: "serving"}
MAX_BATCH_PX = 64 << 20  # serving: a launch stops growing at 64 Mpx (~35 us of HBM time)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("tdct_kernels.hip", "tdct_tiles.hpp", "tdct_device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1702_00817_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(name: str):
    """HBM traffic per launch from a committed rocprofv3 counter summary,
    or None when absent or taken from a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source") != kernel_source_hash():
        return None
    return d


def make_large_batch(tdct, torch, n, side):
    import synth
    sizes, seeds, qs = synth.large_batch_spec(n=n, side=side)
    t0 = time.time()
    buf, off, strides = synth.batch(sizes, seeds)
    log("generated %d x %d^2 images in %.1fs" % (n, side, time.time() - t0))
    src = torch.from_numpy(buf).cuda()
    nblk = (side // 8) ** 2
    coef = torch.empty((n, nblk, 64), dtype=torch.int16, device="cuda")
    dst = torch.empty((n, side, side), dtype=torch.uint8, device="cuda")
    base = src.data_ptr()
    enc = [tdct.image_desc(tdct.OP_ENCODE, side, side, qtab=i, keep=64, src=base + int(off[i]),
                           src_stride=side, coef=coef[i]) for i in range(n)]
    dec = [tdct.image_desc(tdct.OP_DECODE, side, side, qtab=i, coef=coef[i], dst=dst[i],
                           dst_stride=side) for i in range(n)]
    return dict(buf=buf, off=off, strides=strides, sizes=sizes, qs=qs, src=src, coef=coef, dst=dst,
                enc=enc, dec=dec, pixels=n * side * side)


def parse_tune(text):
    """'WPG,GPC,TW[,XCD[,PIXEL_CACHE]]' as a launch-shape dict."""
    v = [int(x) for x in text.split(",")]
    if len(v) not in (3, 4, 5):
        raise SystemExit("a launch shape is WPG,GPC,TW[,XCD_REMAP[,PIXEL_CACHE]]: %r" % text)
    return dict(waves_per_group=v[0], groups_per_cu=v[1], tile_waves=v[2],
                xcd_remap=v[3] if len(v) >= 4 else 0, pixel_cache=v[4] if len(v) == 5 else 0)


# The launch shapes that measured fastest for the 64 x 4096^2 encode + decode
# step across boxes (encoder: 4 waves a group, one group a CU, two tiles a
# step, tiles in one range per XCD; decoder: 2 waves a group, full grid).
REFERENCE_TUNE = "4,1,2,1,0:2,4096,1,0,0"


def step_choice(tdct, torch, W, cands, stream, rounds=3, steps=10):
    """Times each (encode shape, decode shape) pair of `cands` in whole
    encode + decode steps of the batch, round-robin over `rounds` runs of
    `steps` steps (after 2 warm-up steps each): the autotuner times each plan
    alone, encode after encode, and shapes that tie there can differ when the
    encoder follows the decoder. Returns the index of the pair with the lowest
    median device time per step, and the medians (ms)."""
    plans = []
    try:
        for e, d in cands:
            plans.append((tdct.tdct_batch_plan(W["enc"], W["qs"], tune=e),
                          tdct.tdct_batch_plan(W["dec"], W["qs"], tune=d)))
        ms = [[] for _ in cands]
        for _ in range(rounds):
            for i, (pe, pd) in enumerate(plans):
                _, enc_ms, dec_ms = time_steps(tdct, torch, pe, pd, steps, 2, stream)
                ms[i].append(sum(enc_ms) / steps + sum(dec_ms) / steps)
    finally:
        for pe, pd in plans:
            tdct.tdct_plan_free(pe)
            tdct.tdct_plan_free(pd)
    med = [sorted(m)[len(m) // 2] for m in ms]
    return min(range(len(cands)), key=lambda i: med[i]), med


def time_steps(tdct, torch, pe, pd, steps, warmup, stream):
    for _ in range(warmup):
        tdct.tdct_batch_run(pe, stream)
        tdct.tdct_batch_run(pd, stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        tdct.tdct_batch_run(pe, stream)
        ev[k][1].record(stream)
        tdct.tdct_batch_run(pd, stream)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    dec_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    return wall, enc_ms, dec_ms


def cpu_baseline(W, min_s=10.0, max_passes=16):
    """The oracle, as it stands, on the host cores: encode + decode of whole
    4096 x 4096 images of the same batch, cycling through the batch until at
    least `min_s` seconds have passed (at most `max_passes` passes)."""
    import oracle as O
    import synth
    threads = max(1, min(os.cpu_count() or 1, 64))
    px = 0
    done = 0
    n = len(W["sizes"])
    t0 = time.perf_counter()
    while done < max_passes * n:
        i = done % n
        img = synth.batch_view(W["buf"], W["off"], W["strides"], W["sizes"], i)
        w, h = W["sizes"][i]
        q = O.quantise(img, W["qs"][i], 64, threads=threads)
        O.inverse(q, W["qs"][i], w, h, threads=threads)
        px += w * h
        done += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one core, over a smaller sample
    px1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < min_s / 4:
        img = synth.batch_view(W["buf"], W["off"], W["strides"], W["sizes"], 0)
        w, h = W["sizes"][0]
        q = O.quantise(img, W["qs"][0], 64, threads=1)
        O.inverse(q, W["qs"][0], w, h, threads=1)
        px1 += w * h
    dt1 = time.perf_counter() - t1
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(px / dt / 1e9, 4), "unit": "Gpixel/s", "cores": threads, "kind": "oracle",
            "sample": "encode+decode of %d images of 4096x4096 from the 64-image batch (%.1f s wall), "
                      "dense 8x8 integer products, %d threads, %s" % (done, dt, threads, cpu_model),
            "single_core": {"value": round(px1 / dt1 / 1e9, 4), "unit": "Gpixel/s",
                            "sample": "encode+decode of image 0, %d passes in %.1f s, 1 thread"
                                      % (px1 // (W["sizes"][0][0] * W["sizes"][0][1]), dt1)}}


def per_image_leg(tdct, torch, W, stream, reps=5):
    """The 64-image batch coded with one plain launch per image (all encodes,
    then all decodes): the comparison for the one-launch batch form."""
    tdct.tdct_run_per_image(W["enc"], W["qs"], stream)
    tdct.tdct_run_per_image(W["dec"], W["qs"], stream)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tdct.tdct_run_per_image(W["enc"], W["qs"], stream)
        tdct.tdct_run_per_image(W["dec"], W["qs"], stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = sorted(ms)[len(ms) // 2]
    return {"launches": 2 * len(W["enc"]), "ms": round(med, 4),
            "gpx_s": round(W["pixels"] / (med / 1e3) / 1e9, 2)}


def latency_leg(tdct, torch, stream, side=512, reps=100):
    """One 512 x 512 image (seed 1), Q = 1: the int32 forward transform, the
    quantiser with zonal keep 10, the decoder, and the fused round trip, each
    as the median of `reps` event-timed calls; the input (256 KiB) is cache
    resident, so these are latencies, not roofline figures. The calls are
    queued behind a spin kernel of about 20 ms, so each event pair brackets
    device time only (with an idle queue it would also take in the host's
    time to marshal and launch the call). The same measurement of a
    near-empty kernel (the spin kernel for one cycle) gives the floor of the
    method: event overhead plus one dispatch. Also the host clock from call
    to completion of one round trip, and the PSNR of the keep-10
    reconstruction."""
    import numpy as np

    import synth
    img = synth.plane(side, side, 1)
    one = np.ones(64, np.uint16)
    src = torch.from_numpy(img).cuda()
    nblk = (side // 8) ** 2
    Y = torch.empty((nblk, 64), dtype=torch.int32, device="cuda")
    q = torch.empty((nblk, 64), dtype=torch.int16, device="cuda")
    rec = torch.empty_like(src)
    rt = torch.empty_like(src)
    sse = torch.zeros(1, dtype=torch.int64, device="cuda")
    def empty():
        with torch.cuda.stream(stream):
            torch.cuda._sleep(1)

    ops = {
        "empty_kernel": empty,
        "forward_int32": lambda: tdct.tdct_forward(src, side, side, side, Y, stream),
        "quantise_keep10": lambda: tdct.tdct_quantise(src, side, side, side, one, 10, q, stream),
        "inverse": lambda: tdct.tdct_inverse(q, one, side, side, rec, side, stream),
        "roundtrip_keep10": lambda: tdct.tdct_roundtrip(src, side, side, side, one, 10, None, rt, side,
                                                        stream),
    }
    hold = spin_cycles(torch, stream, 20.0)
    out = {"side": side, "reps": reps}
    for name, f in ops.items():
        f()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        with torch.cuda.stream(stream):
            torch.cuda._sleep(hold)
        for k in range(reps):
            ev[2 * k].record(stream)
            f()
            ev[2 * k + 1].record(stream)
        torch.cuda.synchronize()
        t = sorted(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(reps))
        out[name + "_us"] = round(1e3 * t[reps // 2], 2)
    wall = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ops["roundtrip_keep10"]()
        stream.synchronize()
        wall.append(time.perf_counter() - t0)
    out["roundtrip_keep10_call_to_done_us"] = round(1e6 * sorted(wall)[reps // 2], 2)
    tdct.tdct_sse(src, side, rec, side, side, side, sse.data_ptr(), stream)
    torch.cuda.synchronize()
    mse = float(sse.item()) / (side * side)
    out["psnr_keep10_db"] = round(10 * np.log10(255.0 ** 2 / mse), 3) if mse > 0 else None
    return out


def graph_replay_ms(tdct, torch, plan, stream, warm=5, n=11):
    """Median device time (ms) of one replay of the plan's graph: the graph
    is captured and replayed `warm` times first, so that the clocks settle
    after the idle gap of the capture (the first launches after such a gap
    run up to 25 % slower), then each of `n` replays is timed with events on
    the launch stream."""
    for _ in range(1 + warm):
        tdct.tdct_batch_graph(plan, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    ev[0].record(stream)
    for k in range(n):
        tdct.tdct_batch_graph(plan, stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(n))[n // 2]


def batched_leg(tdct, torch, stream, n=10000, reps=5, per_image=True):
    """10,000 ragged images, encode + decode round trip with coefficients:
    persistent launch (graph replay median) vs one plain launch per image, and vs
    the same per-image launches captured in one hipGraph (no launch
    overhead: what remains is the cost of 10,000 small grids). per_image=False
    leaves the per-image comparisons out (for runs under a profiler)."""
    import numpy as np

    import synth
    sizes, seeds, qs = synth.ragged_batch_spec(n=n)
    t0 = time.time()
    buf, off, strides = synth.batch(sizes, seeds)
    log("generated %d ragged images (%.2f Gpx) in %.1fs" % (n, buf.size / 1e9, time.time() - t0))
    src = torch.from_numpy(buf).cuda()
    nblk = np.array([(w // 8) * (h // 8) for w, h in sizes], np.int64)
    boff = np.concatenate([[0], np.cumsum(nblk)])
    coef = torch.empty((int(boff[-1]), 64), dtype=torch.int16, device="cuda")
    dst = torch.empty(buf.size, dtype=torch.uint8, device="cuda")
    base, cb, db = src.data_ptr(), coef.data_ptr(), dst.data_ptr()
    descs = [tdct.image_desc(tdct.OP_ROUNDTRIP, w, h, qtab=i, keep=64, src=base + int(off[i]),
                             src_stride=w, coef=cb + 128 * int(boff[i]), dst=db + int(off[i]),
                             dst_stride=w) for i, (w, h) in enumerate(sizes)]
    px = int(sum(w * h for w, h in sizes))
    plan = tdct.tdct_batch_plan(descs, qs)
    try:
        tune = tdct.tdct_autotune(plan, stream, reps=2)
        graph_s = graph_replay_ms(tdct, torch, plan, stream) / 1e3
        info = tdct.tdct_plan_info_get(plan)
        per_s = per_graph_s = graph_same = None
        if per_image:
            tdct.tdct_run_per_image(descs, qs, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                tdct.tdct_run_per_image(descs, qs, stream)
            torch.cuda.synchronize()
            per_s = (time.perf_counter() - t0) / reps
            # the per-image launches captured once and replayed
            want = dst.clone()
            dst.zero_()
            torch.cuda.synchronize()
            cap = torch.cuda.Stream()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                tdct.tdct_run_per_image(descs, qs, cap)
            g.replay()
            torch.cuda.synchronize()
            graph_same = bool(torch.equal(dst, want))
            del want
            t0 = time.perf_counter()
            for _ in range(reps):
                g.replay()
            torch.cuda.synchronize()
            per_graph_s = (time.perf_counter() - t0) / reps
            del g
    finally:
        tdct.tdct_plan_free(plan)
    del src, coef, dst
    gbs = 4 * px / graph_s / 1e9
    traffic = load_traffic("roundtrip_ragged_10000")
    out = {"images": n, "pixels": px, "tiles": info["tiles"], "tune": tune,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(gbs / 8000.0, 4),
                        "traffic": traffic["hbm_bytes_per_launch"] if traffic else None},
           "graph_gpx_s": round(px / graph_s / 1e9, 2), "graph_ms": round(graph_s * 1e3, 3),
           "bytes_per_px": 4}
    if per_image:
        out.update({"per_image_gpx_s": round(px / per_s / 1e9, 2), "per_image_ms": round(per_s * 1e3, 3),
                    "per_image_graph_gpx_s": round(px / per_graph_s / 1e9, 2),
                    "per_image_graph_ms": round(per_graph_s * 1e3, 3), "per_image_graph_same": graph_same,
                    "speedup": round(per_s / graph_s, 2)})
    return (buf, off, strides, sizes, qs), out


PROBES = (("copy", 32), ("read", 16), ("write", 16), ("read1_write2", 48), ("read2_write1", 48),
          ("read1_write3", 64))


def ceiling_leg(tdct, torch, stream, mib=1024, reps=5, names=None):
    """HBM ceilings on this part: the codec's access mixes without arithmetic."""
    units = (mib << 20) // 16
    a = torch.ones(2 * units * 16, dtype=torch.uint8, device="cuda")
    b = torch.empty(3 * units * 16, dtype=torch.uint8, device="cuda")
    out = {}
    kinds = {"copy": tdct.PROBE_COPY, "read": tdct.PROBE_READ, "write": tdct.PROBE_WRITE,
             "read1_write2": tdct.PROBE_R1W2, "read2_write1": tdct.PROBE_R2W1,
             "read1_write3": tdct.PROBE_R1W3}
    for name, per_unit in PROBES:
        if names and name not in names:
            continue
        kind = kinds[name]
        tdct.tdct_stream_probe(kind, a, b, units, stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        for k in range(reps):
            ev[k].record(stream)
            tdct.tdct_stream_probe(kind, a, b, units, stream)
        ev[reps].record(stream)
        torch.cuda.synchronize()
        ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))[reps // 2]
        out[name] = round(per_unit * units / (ms / 1e3) / 1e9, 1)
    del a, b
    return {"unit": "GB/s", "mib_per_unit_side": mib, **out}


# VALU issue peak of the part: 256 CUs x 4 SIMDs x 16 lanes per clock at
# 2.4 GHz = 39.3 T lane-operations/s (non-packed 32-bit; a wave64 VALU
# instruction occupies one SIMD for 4 clocks).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# The method's own integer operations per 8x8 block of a round trip without
# stored coefficients: level shift 1 (on the DC term), forward 16 x 14 = 224
# add/sub (Table 1's 14 per 8-point pass), quantiser 64 shifts (D^2 fold) +
# 64 rounding divisions, dequantiser 64 multiplies, inverse 224 add/sub,
# rounding offset 1 (on the DC term), 64 shifts by 6 and 128 clamp
# comparisons: 834 per 64 pixels.
ROUNDTRIP_ALG_OPS_PER_BLOCK = 1 + 224 + 64 + 64 + 64 + 224 + 1 + 64 + 128


def load_valu(name: str):
    """VALU instructions per launch from a committed rocprofv3 counter
    summary, or None when absent or taken from a different kernel source."""
    path = os.path.join(ROOT, "profiles", "valu_%s.json" % name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source") != kernel_source_hash():
        return None
    return d


def fused_leg(tdct, torch, W, stream, reps=10, tune=None):
    """Encode + decode in one pass with no coefficients in HBM (2 B/px) on the
    same 64 x 4096^2 batch. It runs near two bounds, HBM and VALU issue; its
    roofline gives both (the counted VALU instructions per launch over the
    launch time against the part's VALU issue peak, and 2 B/px against
    8 TB/s), the nearer one on top."""
    n = len(W["sizes"])
    side = W["sizes"][0][0]
    base = W["src"].data_ptr()
    descs = [tdct.image_desc(tdct.OP_ROUNDTRIP, side, side, qtab=i, keep=64, src=base + int(W["off"][i]),
                             src_stride=side, coef=None, dst=W["dst"][i], dst_stride=side)
             for i in range(n)]
    plan = tdct.tdct_batch_plan(descs, W["qs"], tune=tune)
    try:
        if tune is None:
            tune = tdct.tdct_autotune(plan, stream, reps=2)
        tdct.tdct_batch_run(plan, stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        for k in range(reps):
            ev[k].record(stream)
            tdct.tdct_batch_run(plan, stream)
        ev[reps].record(stream)
        torch.cuda.synchronize()
        ms = sum(ev[k].elapsed_time(ev[k + 1]) for k in range(reps)) / reps
    finally:
        tdct.tdct_plan_free(plan)
    px = W["pixels"]
    # both bounds: HBM (2 B/px) and VALU issue (the counted instructions per
    # launch over the launch time); the top level is the nearer one
    gbs = 2 * px / (ms / 1e3) / 1e9
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
           "frac": round(gbs / 8000.0, 4)}
    roof = dict(hbm)
    valu = load_valu("roundtrip_64x4096")
    if valu:
        lane_ops = valu["valu_insts_per_launch"] * 64
        achieved = lane_ops / (ms / 1e3) / 1e12
        alg = ROUNDTRIP_ALG_OPS_PER_BLOCK / 64
        alu = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TOPS, 2),
               "unit": "T VALU lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
               "valu_lane_ops_per_px": round(lane_ops / px, 3),
               # the method's own operation count at the same rate; above the
               # issued count because packed int16 codes two blocks per
               # instruction and the fp32 decoder half fuses multiply-adds and
               # round/clamp/pack
               "algorithmic_ops_per_px": round(alg, 3),
               "algorithmic_tops": round(alg * px / (ms / 1e3) / 1e12, 2)}
        roof = dict(alu, hbm=hbm) if alu["frac"] > hbm["frac"] else dict(hbm, valu=alu)
    return {"kernel": "batch_kernel<32, %s> (round trip, coefficients kept in registers)"
            % ("true" if tune.get("pixel_cache") else "false"), "tune": tune,
            "ms": round(ms, 4), "gpx_s": round(px / (ms / 1e3) / 1e9, 1),
            "gbs": round(2 * px / (ms / 1e3) / 1e9, 1), "bytes_per_px": 2, "roofline": roof}


def forward_leg(tdct, torch, W, stream, reps=10):
    """The int32 forward transform alone (Y = T X T^t, no quantiser) of the
    same 64 x 4096^2 batch: 1 B in + 4 B out per pixel, HBM-bound; the
    launch shape comes from the autotuner."""
    n = len(W["sizes"])
    side = W["sizes"][0][0]
    nblk = (side // 8) ** 2
    base = W["src"].data_ptr()
    Y = torch.empty((n, nblk, 64), dtype=torch.int32, device="cuda")
    descs = [tdct.image_desc(tdct.OP_FORWARD, side, side, src=base + int(W["off"][i]),
                             src_stride=side, coef=Y[i]) for i in range(n)]
    plan = tdct.tdct_batch_plan(descs, W["qs"])
    try:
        tune = tdct.tdct_autotune(plan, stream, reps=2)
        tdct.tdct_batch_run(plan, stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        for k in range(reps):
            ev[k].record(stream)
            tdct.tdct_batch_run(plan, stream)
        ev[reps].record(stream)
        torch.cuda.synchronize()
        ms = sum(ev[k].elapsed_time(ev[k + 1]) for k in range(reps)) / reps
    finally:
        tdct.tdct_plan_free(plan)
    del Y
    gbs = 5 * W["pixels"] / (ms / 1e3) / 1e9
    return {"kernel": "batch_kernel<16, %s> (int32 forward)" % ("true" if tune.get("pixel_cache") else "false"),
            "tune": tune, "ms": round(ms, 4),
            "gpx_s": round(W["pixels"] / (ms / 1e3) / 1e9, 1), "gbs": round(gbs, 1),
            "bytes_per_px": 5, "frac_of_8tbs": round(gbs / 8000.0, 4)}


def video_leg(tdct, torch, stream, frames=256, reps=5):
    """256 frames of 3840x2160 4:2:0: encoder with luma/chroma Q tables,
    int8-saturated zigzag coefficients; one persistent launch over all
    768 planes (graph replay) vs one plain launch per plane. Both bounds are
    reported: HBM (2 B/sample) and VALU issue (the counted instructions per
    launch over the launch time)."""
    import numpy as np

    import synth
    v = synth.Video420(frames=frames)
    w, h = v.w, v.h
    fbytes = w * h + 2 * (w // 2) * (h // 2)
    t0 = time.time()
    host = np.empty(frames * fbytes, np.uint8)
    for f in range(frames):
        o = f * fbytes
        Y = host[o:o + w * h].reshape(h, w)
        Cb = host[o + w * h:o + w * h + (w // 2) * (h // 2)].reshape(h // 2, w // 2)
        Cr = host[o + w * h + (w // 2) * (h // 2):o + fbytes].reshape(h // 2, w // 2)
        v.frame(f, out=(Y, Cb, Cr))
    log("generated %d 4:2:0 frames (%.2f G samples) in %.1fs" % (frames, host.size / 1e9, time.time() - t0))
    src = torch.from_numpy(host).cuda()
    out = torch.empty(host.size, dtype=torch.int8, device="cuda")
    descs, qtabs = [], []
    sb, ob = src.data_ptr(), out.data_ptr()
    for f in range(frames):
        qy, qc = v.qtables(f)
        qtabs += [qy, qc]
        o = f * fbytes
        for pw, ph, po, qi in ((w, h, 0, 2 * f), (w // 2, h // 2, w * h, 2 * f + 1),
                               (w // 2, h // 2, w * h + (w // 2) * (h // 2), 2 * f + 1)):
            descs.append(tdct.image_desc(tdct.OP_ENCODE_I8ZZ, pw, ph, qtab=qi, src=sb + o + po,
                                         src_stride=pw, coef=ob + o + po))
    plan = tdct.tdct_batch_plan(descs, qtabs)
    try:
        tune = tdct.tdct_autotune(plan, stream, reps=2)
        graph_s = graph_replay_ms(tdct, torch, plan, stream) / 1e3
        tdct.tdct_run_per_image(descs, qtabs, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            tdct.tdct_run_per_image(descs, qtabs, stream)
        torch.cuda.synchronize()
        per_s = (time.perf_counter() - t0) / reps
    finally:
        tdct.tdct_plan_free(plan)
    n = host.size
    del src, out
    ctx = (host, v, frames)
    gbs = 2 * n / graph_s / 1e9
    traffic = load_traffic("video_420x256")
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(gbs / 8000.0, 4),
            "traffic": traffic["hbm_bytes_per_launch"] if traffic else None}
    valu = load_valu("video_420x256")
    if valu:
        lane_ops = valu["valu_insts_per_launch"] * 64
        achieved = lane_ops / graph_s / 1e12
        roof["valu"] = {"achieved": round(achieved, 2), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "T VALU lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                        "valu_lane_ops_per_sample": round(lane_ops / n, 3)}
    return ctx, {"frames": frames, "samples": n, "tune": tune,
            "graph_gsamples_s": round(n / graph_s / 1e9, 1), "graph_ms": round(graph_s * 1e3, 3),
            "graph_gbs": round(gbs, 1),
            "per_plane_gsamples_s": round(n / per_s / 1e9, 1), "per_plane_ms": round(per_s * 1e3, 3),
            "speedup": round(per_s / graph_s, 2), "bytes_per_sample": 2, "roofline": roof}


def dct2_matrix():
    """Orthonormal 8-point DCT-II (the exact transform the paper compares with)."""
    import numpy as np
    k = np.arange(8)[:, None]
    n = np.arange(8)[None, :]
    M = np.cos((2 * n + 1) * k * np.pi / 16) * np.sqrt(2 / 8)
    M[0, :] = np.sqrt(1 / 8)
    return M


def quality_leg(tdct, torch, stream, n_images=45, side=512, rs=range(2, 46)):
    """The paper's image-compression experiment (zonal coding, Section 3) on a
    synthetic stand-in for its 45-image set: for every r, the integer codec
    (Q = 1, zonal keep r) runs on the GPU with an exact SSE per image; the
    exact DCT-II with the same zonal rule, rounding and clamp runs on the host
    in float64. Reported: mean PSNR, PSNR of the mean MSE, and the absolute
    percentage error of the average MSE relative to the DCT (Fig. 2 methodology)."""
    import numpy as np

    import synth
    rs = list(rs)
    one = np.ones(64, np.uint16)
    imgs = [synth.plane(side, side, 100 + i) for i in range(n_images)]
    src = torch.from_numpy(np.stack(imgs)).cuda()
    dst = torch.empty_like(src)
    sse = torch.zeros((n_images, len(rs)), dtype=torch.int64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(n_images):
        for k, r in enumerate(rs):
            tdct.tdct_roundtrip(src[i], side, side, side, one, r, None, dst[i], side, stream)
            tdct.tdct_sse(src[i], side, dst[i], side, side, side, sse[i, k].data_ptr(), stream)
    e1.record(stream)
    torch.cuda.synchronize()
    gpu_ms = e0.elapsed_time(e1)
    sse_ours = sse.cpu().numpy().astype(np.float64)
    # exact DCT reference on the host (float64), same zonal rule
    C = dct2_matrix()
    order = []
    for d in range(15):  # JPEG zigzag, as in the codec
        cells = [(i, d - i) for i in range(8) if 0 <= d - i < 8]
        order += cells if d % 2 else cells[::-1]
    rank = np.empty((8, 8), np.int64)
    for t, (i, j) in enumerate(order):
        rank[i, j] = t
    sse_dct = np.zeros((n_images, len(rs)))
    for i, img in enumerate(imgs):
        X = img.reshape(side // 8, 8, side // 8, 8).transpose(0, 2, 1, 3).astype(np.float64) - 128
        Y = C @ X @ C.T  # per block: C X C^t
        for k, r in enumerate(rs):
            Z = C.T @ (Y * (rank < r)) @ C
            rec = np.clip(np.floor(Z + 0.5) + 128, 0, 255)
            sse_dct[i, k] = ((rec - X - 128) ** 2).sum()
    npx = side * side
    rows = []
    for k, r in enumerate(rs):
        mse_o = sse_ours[:, k] / npx
        mse_d = sse_dct[:, k] / npx
        psnr_o = np.where(mse_o > 0, 10 * np.log10(255.0 ** 2 / np.maximum(mse_o, 1e-300)), np.inf)
        rows.append({"r": r, "compression_pct": round(100 * (64 - r) / 64, 4),
                     "psnr_mean": round(float(np.mean(psnr_o)), 3),
                     "psnr_of_mean_mse": round(float(10 * np.log10(255.0 ** 2 / mse_o.mean())), 3),
                     "psnr_dct_of_mean_mse": round(float(10 * np.log10(255.0 ** 2 / mse_d.mean())), 3),
                     "ape_mse_pct": round(float(abs(mse_o.mean() - mse_d.mean()) / mse_d.mean() * 100), 3)})
    return {"images": n_images, "side": side, "gpu_ms": round(gpu_ms, 2),
            "gpu_launches": 2 * n_images * len(rs), "table": rows}


SERVING_POOL = 4          # payload planes of the serving leg
SERVING_SIDE = 8192       # their side (the largest request side)


def serving_pool(tdct, torch):
    """Device-resident payloads of the serving leg: SERVING_POOL blob planes
    of 8192^2 (encode inputs; a request is the top-left w x h window) and the
    encoder's output of each under Q = 1 + (1 + k)(i + j) (decode inputs; a
    request decodes the first (w/8)(h/8) blocks as a w x h image)."""
    import synth
    log("serving: building a payload pool of %d planes of %d^2" % (SERVING_POOL, SERVING_SIDE))
    host = [synth.plane(SERVING_SIDE, SERVING_SIDE, 5000 + k) for k in range(SERVING_POOL)]
    pool = [torch.from_numpy(p).cuda() for p in host]
    nblk = (SERVING_SIDE // 8) ** 2
    coefs = []
    for k in range(SERVING_POOL):
        c = torch.empty((nblk, 64), dtype=torch.int16, device="cuda")
        tdct.tdct_quantise(pool[k], SERVING_SIDE, SERVING_SIDE, SERVING_SIDE, synth.qtable(1, 1 + k), 64, c)
        coefs.append(c)
    torch.cuda.synchronize()
    return {"host": host, "pool": pool, "coefs": coefs}


def serving_requests(tdct, tr, P, idx=None, host_io=None):
    """The trace's requests (or those at `idx`) as one ctypes array: request k
    encodes or decodes a window of payload k mod SERVING_POOL with
    Q = 1 + s(i + j), keep 64. host_io: (pinned pool copies, pinned coefficient
    copies, pinned output buffers reused in turn)."""
    import synth
    qt = {s: tdct.qtable(synth.qtable(1, s)) for s in range(1, 9)}
    idx = range(len(tr["t"])) if idx is None else idx
    idx = list(idx)
    ra = tdct.request_array(len(idx))
    pin = [p.data_ptr() for p in P["pool"]]
    cin = [c.data_ptr() for c in P["coefs"]]
    if host_io:
        hp, hc, ho = host_io
        pin = [p.data_ptr() for p in hp]
        cin = [c.data_ptr() for c in hc]
        outs = [o.data_ptr() for o in ho]
    ops, ws, hs, ss = tr["op"], tr["w"], tr["h"], tr["s"]
    for j, k in enumerate(idx):
        r = ra[j]
        w, h, p = int(ws[k]), int(hs[k]), k % SERVING_POOL
        r.w, r.h, r.keep, r.Q = w, h, 64, qt[int(ss[k])]
        if ops[k] == 0:
            r.op, r.input, r.in_stride = tdct.OP_ENCODE, pin[p], SERVING_SIDE
        else:
            r.op, r.input, r.in_stride = tdct.OP_DECODE, cin[p], w
        if host_io:
            r.host_io, r.host_output = 1, outs[k % len(outs)]
    return ra


def _pct(v, q):
    import numpy as np
    return round(float(np.percentile(v, q)), 1) if len(v) else None


def serving_cfg(tdct, mode, streams=4, resident_workers=0):
    if mode == "resident":
        return tdct.server_cfg(64 << 30, resident=1, resident_workers=resident_workers,
                               resident_idle_us=100000)
    # requests have ragged widths: batch launches take cached pixel accesses
    # (burst capacity +5-8 % measured; lone requests use the plain kernel
    # either way)
    # batches take the autotune cache's shape for their class (tuned beforehand,
    # tune_serving_classes), else cached pixel accesses
    return tdct.server_cfg(64 << 30, streams=streams, max_batch=64, max_wait_us=0,
                           batching=0 if mode == "per_request" else 1, max_batch_px=MAX_BATCH_PX,
                           tune=dict(pixel_cache=1), tune_cache=1)


def tune_serving_classes(tdct, torch, P, rate=5000, seconds=4.0, sizes=(2, 4, 8, 16, 32, 64)):
    """Fills the autotune cache with the classes serving batches fall in:
    consecutive requests of the trace in groups of `sizes` requests (up to
    MAX_BATCH_PX pixels, as the server cuts its batches) become batch plans,
    and each is autotuned once. Servers created with tune_cache = 1 then
    launch each batch in the shape stored for its class (or the nearest size
    class). Returns the classes tuned."""
    import synth
    tr = synth.serving_trace(rate, seconds, seed=5)
    n = len(tr["t"])
    tuned, start = [], 0
    stream = torch.cuda.current_stream()
    for size in sizes:
        descs, qtabs, outs, px = [], [], [], 0
        k = start
        while k < n and len(descs) < size:
            w, h, s_, p = int(tr["w"][k]), int(tr["h"][k]), int(tr["s"][k]), k % SERVING_POOL
            if descs and px + w * h > MAX_BATCH_PX:
                break
            qtabs.append(synth.qtable(1, s_))
            if tr["op"][k] == 0:
                out = torch.empty(w * h * 2, dtype=torch.uint8, device="cuda")
                descs.append(tdct.image_desc(tdct.OP_ENCODE, w, h, qtab=len(qtabs) - 1, keep=64,
                                             src=P["pool"][p], src_stride=SERVING_SIDE, coef=out))
            else:
                out = torch.empty(w * h, dtype=torch.uint8, device="cuda")
                descs.append(tdct.image_desc(tdct.OP_DECODE, w, h, qtab=len(qtabs) - 1,
                                             coef=P["coefs"][p], dst=out, dst_stride=w))
            outs.append(out)
            px += w * h
            k += 1
        start = k
        if not descs:
            break
        plan = tdct.tdct_batch_plan(descs, qtabs)
        try:
            tune = tdct.tdct_autotune(plan, stream, reps=2)
            info = tdct.tdct_plan_info_get(plan)
        finally:
            tdct.tdct_plan_free(plan)
        tuned.append({"requests": len(descs), "mpx": round(px / 1e6, 1), "tiles": info["tiles"], "tune": tune})
        del outs
    torch.cuda.synchronize()
    return tuned


def serving_leg(tdct, torch, seconds, aux_seconds, rates=(200, 1000, 5000), streams=4,
                resident_workers=0,
                modes=("resident", "per_request", "batched", "per_request_short", "host_io_batched"),
                batched_seconds=None):
    """Poisson encode/decode requests (the serving workload: sides log-uniform
    multiples of 8 in [32, 8192], aspect <= 4, s in {1..8}) served by
    continuous batching and by one plain launch per request for `seconds`
    per rate, with device-resident payloads: the resident polling kernel
    (the served form) and one plain launch per request for `seconds`,
    continuous batching into launched batch kernels for `batched_seconds`,
    one plain launch per request again over that same shorter trace
    (per_request_short: the like-for-like comparison for batching),
    and batching with host payloads copied over PCIe (host_io_batched, the
    PCIe-inclusive rate) for `aux_seconds`. Per mode: latency
    percentiles, the tail's make-up (share of p99-and-above requests served in
    a batch of more than one, their mean size) and small-request percentiles.
    Returns (result, context for the oracle check)."""
    import numpy as np

    import synth
    P = serving_pool(tdct, torch)
    tuned = tune_serving_classes(tdct, torch, P)
    log("serving: tuned batch classes %s" % json.dumps(tuned))
    hp = hc = ho = None
    if "host_io_batched" in modes:
        # pinned copies of the payloads and a few pinned output buffers of the
        # largest size reused in turn (requests in flight may overwrite each
        # other's host copies: timing only)
        hp = [p.cpu().pin_memory() for p in P["pool"]]
        hc = [c.cpu().pin_memory() for c in P["coefs"]]
        ho = [torch.empty(2 * SERVING_SIDE ** 2, dtype=torch.uint8).pin_memory() for _ in range(4)]
    out, traces = {}, {}
    for rate in rates:
        res = {}
        for mode in modes:
            secs = {"resident": seconds, "per_request": seconds, "batched": batched_seconds or seconds,
                    "per_request_short": batched_seconds or seconds}.get(mode, aux_seconds)
            cfg_mode = "per_request" if mode == "per_request_short" else mode
            tr = synth.serving_trace(rate, secs, seed=5)
            traces[(rate, secs)] = tr
            px = (tr["w"] * tr["h"]).astype(np.int64)
            ra = serving_requests(tdct, tr, P, host_io=(hp, hc, ho) if mode == "host_io_batched" else None)
            arrival = (tr["t"] * 1e6).tolist()
            srv = tdct.tdct_server_create(serving_cfg(tdct, cfg_mode, streams, resident_workers))
            try:
                t0 = time.perf_counter()
                _, lat, st, bs = tdct.tdct_server_replay(srv, ra, arrival, with_batch=True)
                wall = time.perf_counter() - t0
                stats = tdct.tdct_server_stats(srv)
            finally:
                tdct.tdct_server_destroy(srv)
            ok = np.array(st) == 0
            lat, bs, pxo = np.array(lat)[ok], np.array(bs)[ok], px[ok]
            p99 = np.percentile(lat, 99) if len(lat) else 0
            tail = lat >= p99
            small = pxo < (1 << 20)
            res[mode] = {"seconds": secs, "requests": int(len(px)), "mpx_mean": round(float(px.mean()) / 1e6, 3),
                         "p50_us": _pct(lat, 50), "p99_us": _pct(lat, 99), "p999_us": _pct(lat, 99.9),
                         "failed": int((~ok).sum()),
                         "delivered_gpx_s": round(float(px.sum()) / wall / 1e9, 3),
                         "batches": stats["batches"], "mean_batch": round(stats["mean_batch"], 3),
                         "arena_high_water_gb": round(stats["arena_high_water"] / 1e9, 3),
                         "tail": {"requests": int(tail.sum()),
                                  "in_batches_share": round(float((bs[tail] > 1).mean()), 3) if tail.any() else None,
                                  "mpx_mean": round(float(pxo[tail].mean()) / 1e6, 2) if tail.any() else None},
                         "under_1mpx": {"requests": int(small.sum()), "p50_us": _pct(lat[small], 50),
                                        "p99_us": _pct(lat[small], 99)}}
            log("serving %d req/s %s: %s" % (rate, mode, json.dumps(res[mode])))
        if rate == max(rates):
            # capacity: the same requests all arriving at once (closed burst),
            # the aux-length trace
            tr = synth.serving_trace(rate, aux_seconds, seed=5)
            ra = serving_requests(tdct, tr, P)
            px = float((tr["w"] * tr["h"]).sum())
            for mode in modes:
                if mode in ("host_io_batched", "per_request_short"):
                    continue
                srv = tdct.tdct_server_create(serving_cfg(tdct, mode, streams, resident_workers))
                try:
                    t0 = time.perf_counter()
                    _, lat, st = tdct.tdct_server_replay(srv, ra, [0.0] * len(ra))
                    wall = time.perf_counter() - t0
                    stats = tdct.tdct_server_stats(srv)
                finally:
                    tdct.tdct_server_destroy(srv)
                res["burst_" + mode] = {"requests": len(ra), "gpx_s": round(px / wall / 1e9, 1),
                                        "wall_ms": round(wall * 1e3, 1),
                                        "mean_batch": round(stats["mean_batch"], 2),
                                        "failed": int(sum(1 for s_ in st if s_ != 0))}
        out[str(rate)] = res
    # the served form against one launch per request, per rate
    summary = {"served_form": "resident", "compared_with": "per_request", "rates": {}}
    for rate in rates:
        r = out[str(rate)]
        if "resident" in r and "per_request" in r:
            a, b = r["resident"], r["per_request"]
            summary["rates"][str(rate)] = {k: a[k] for k in ("p50_us", "p99_us", "p999_us")}
            summary["rates"][str(rate)].update({"per_request_" + k: b[k] for k in ("p50_us", "p99_us", "p999_us")})
    # continuous batching against one launch per request on the same trace
    summary["batched_vs_per_request_same_trace"] = {}
    for rate in rates:
        r = out[str(rate)]
        if "batched" in r and "per_request_short" in r:
            a, b = r["batched"], r["per_request_short"]
            d = {k: a[k] for k in ("p50_us", "p99_us", "p999_us")}
            d.update({"per_request_" + k: b[k] for k in ("p50_us", "p99_us", "p999_us")})
            d["seconds"] = a["seconds"]
            summary["batched_vs_per_request_same_trace"][str(rate)] = d
    burst = out[str(max(rates))]
    summary["burst_gpx_s"] = {m: burst["burst_" + m]["gpx_s"] for m in modes if "burst_" + m in burst}
    result = {"summary": summary,
              "seconds_per_rate": {"resident": seconds, "per_request": seconds,
                                   "batched": batched_seconds or seconds,
                                   "per_request_short": batched_seconds or seconds,
                                   "host_io_batched": aux_seconds},
              "batch_tune_classes": tuned,
              "streams": streams, "budget_gb": 64,
              "resident_workers": resident_workers or "four per CU", "rates": out}
    return result, {"P": P, "traces": traces, "seconds": seconds, "streams": streams}


def burst_leg(tdct, torch, modes, reps=3, seconds=4.0, rate=5000, resident_workers=0):
    """The serving trace's requests (`seconds` at `rate` req/s) all arriving
    at once, served `reps` times per mode: capacity of each served form in
    Gpx/s (wall time from the first submit to the last completion). A short,
    self-contained run for kernel traces and counters of the served forms."""
    import synth
    P = serving_pool(tdct, torch)
    out = {}
    if "batched" in modes:
        out["batch_tune_classes"] = tune_serving_classes(tdct, torch, P)
    tr = synth.serving_trace(rate, seconds, seed=5)
    ra = serving_requests(tdct, tr, P)
    px = float((tr["w"] * tr["h"]).sum())
    out.update({"requests": len(ra), "gpx": round(px / 1e9, 2)})
    for mode in modes:
        runs = []
        for _ in range(reps):
            srv = tdct.tdct_server_create(serving_cfg(tdct, mode, resident_workers=resident_workers))
            try:
                t0 = time.perf_counter()
                _, lat, st = tdct.tdct_server_replay(srv, ra, [0.0] * len(ra))
                wall = time.perf_counter() - t0
            finally:
                tdct.tdct_server_destroy(srv)
            runs.append({"gpx_s": round(px / wall / 1e9, 1), "wall_ms": round(wall * 1e3, 1),
                         "failed": int(sum(1 for s_ in st if s_ != 0))})
            log("burst %s: %s" % (mode, json.dumps(runs[-1])))
        out[mode] = runs
    return out


def _hip_copy_d2d():
    """A device-to-device copy ordered on torch's current stream (arena
    outputs into torch buffers for the checks). A plain hipMemcpy between
    device buffers runs on the null stream and may return before the copy
    ends, and torch's streams do not wait for the null stream: a comparison
    queued right after it could read the buffer half copied."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    lib.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p]
    lib.hipMemcpyAsync.restype = ctypes.c_int

    def copy(dst, src, nbytes):
        return lib.hipMemcpyAsync(dst, src, nbytes, 3, torch.cuda.current_stream().cuda_stream)
    return copy


def _oracle_threads():
    return max(1, min(os.cpu_count() or 1, 16))


def cpu_baseline_serving(tdct, torch, ctx, rates, frac=0.01, big_px=32 << 20, direct_n=64):
    """The served outputs against the oracle, outside the timed replays: for
    every rate, a seeded `frac` of the trace plus every request of at least
    32 Mpx is served again (same configuration, all at once, outputs kept),
    by the resident kernel, by batched launches and by one launch per
    request, and each output is compared
    in full with the oracle's.

    The oracle encodes every payload plane under every table the trace uses
    and decodes, block by block, its own encoding of each plane (what the
    decode requests of that payload carry) under every table; a request's
    expected output is then its window (blocks depend only on their own 64
    pixels). The GPU's decode inputs are checked against the oracle's
    encoding too. The oracle is also timed directly on `direct_n` sampled
    requests (its px/s on the request mix)."""
    import numpy as np

    import oracle as O
    import synth
    P = ctx["P"]
    threads = _oracle_threads()
    side = SERVING_SIDE
    nb = side // 8
    nblk = nb * nb
    t0 = time.perf_counter()
    E, D = {}, {}
    for p in range(SERVING_POOL):
        for s_ in range(1, 9):
            E[(p, s_)] = O.quantise(P["host"][p], synth.qtable(1, s_), 64, threads=threads)
    for p in range(SERVING_POOL):
        qin = E[(p, 1 + p)]
        for s_ in range(1, 9):
            plane = O.inverse(qin, synth.qtable(1, s_), side, side, threads=threads)
            D[(p, s_)] = np.ascontiguousarray(plane.reshape(nb, 8, nb, 8).transpose(0, 2, 1, 3))
    t_planes = time.perf_counter() - t0
    planes_px = 2 * len(E) * side * side
    Ed = {k: torch.from_numpy(v).cuda().view(nb, nb, 64) for k, v in E.items()}
    Dd = {k: torch.from_numpy(v).cuda().view(nblk, 8, 8) for k, v in D.items()}
    inputs_ok = all(torch.equal(P["coefs"][p], Ed[(p, 1 + p)].view(nblk, 64)) for p in range(SERVING_POOL))
    copy = _hip_copy_d2d()
    buf = torch.empty(2 * side * side, dtype=torch.uint8, device="cuda")

    def matches(tr, k, ptr, nbytes):
        w, h, s_, p = int(tr["w"][k]), int(tr["h"][k]), int(tr["s"][k]), k % SERVING_POOL
        assert copy(buf.data_ptr(), ptr, nbytes) == 0  # ordered before the comparison
        if tr["op"][k] == 0:
            got = buf[:nbytes].view(torch.int16).view(h // 8, w // 8, 64)
            return nbytes == 2 * w * h and torch.equal(got, Ed[(p, s_)][:h // 8, :w // 8])
        got = buf[:nbytes].view(h // 8, 8, w // 8, 8)
        want = Dd[(p, s_)][:(w // 8) * (h // 8)].view(h // 8, w // 8, 8, 8).permute(0, 2, 1, 3)
        return nbytes == w * h and torch.equal(got, want)

    out = {}
    direct_pool = []
    for rate in rates:
        tr = ctx["traces"][(rate, ctx["seconds"])]
        n = len(tr["t"])
        px = (tr["w"] * tr["h"]).astype(np.int64)
        rng = np.random.default_rng([5, rate, 1])
        rand = rng.choice(n, int(np.ceil(frac * n)), replace=False)
        big = np.nonzero(px >= big_px)[0]
        sample = np.union1d(rand, big)
        direct_pool += [(rate, int(k)) for k in rand[:direct_n]]
        outb = np.where(tr["op"] == 0, 2 * px, px)
        res = {"requests": int(len(sample)), "random": int(len(rand)), "at_least_32mpx": int(len(big)),
               "gpx": round(float(px[sample].sum()) / 1e9, 2)}
        for mode in ("resident", "batched", "per_request"):
            bad = 0
            srv = tdct.tdct_server_create(serving_cfg(tdct, mode, ctx["streams"]))
            try:
                start = 0
                while start < len(sample):
                    # outputs of one chunk stay in the 64 GB arena until compared
                    stop, acc = start, 0
                    while stop < len(sample) and (stop == start or acc + outb[sample[stop]] <= 48 << 30):
                        acc += (int(outb[sample[stop]]) + 255) // 256 * 256
                        stop += 1
                    chunk = [int(k) for k in sample[start:stop]]
                    ra = serving_requests(tdct, tr, P, idx=chunk)
                    tickets, _, st = tdct.tdct_server_replay(srv, ra, [0.0] * len(chunk), keep_outputs=True)
                    for k, t, st_ in zip(chunk, tickets, st):
                        r = tdct.tdct_server_poll(srv, t)
                        if st_ != 0 or not matches(tr, k, r.output, r.output_bytes):
                            bad += 1
                        tdct.tdct_server_release(srv, t)
                    start = stop
            finally:
                tdct.tdct_server_destroy(srv)
            res["mismatches_" + mode] = bad
        out[str(rate)] = res
        log("serving check %d req/s: %s" % (rate, json.dumps(res)))
    # the oracle directly on sampled requests: its px/s on the request mix
    dpx, t0 = 0, time.perf_counter()
    direct_bad = 0
    for rate, k in direct_pool:
        tr = ctx["traces"][(rate, ctx["seconds"])]
        w, h, s_, p = int(tr["w"][k]), int(tr["h"][k]), int(tr["s"][k]), k % SERVING_POOL
        Q = synth.qtable(1, s_)
        if tr["op"][k] == 0:
            q = O.quantise(P["host"][p][:h], Q, 64, w=w, threads=threads)
            direct_bad += not np.array_equal(q.reshape(h // 8, w // 8, 64), E[(p, s_)].reshape(nb, nb, 64)[:h // 8, :w // 8])
        else:
            nbk = (w // 8) * (h // 8)
            x = O.inverse(E[(p, 1 + p)][:nbk], Q, w, h, threads=threads)
            want = D[(p, s_)].reshape(nblk, 8, 8)[:nbk].reshape(h // 8, w // 8, 8, 8).transpose(0, 2, 1, 3)
            direct_bad += not np.array_equal(x.reshape(h // 8, 8, w // 8, 8), want)
        dpx += w * h
    t_direct = time.perf_counter() - t0
    del Ed, Dd, buf
    torch.cuda.empty_cache()
    return {"kind": "oracle", "cores": threads,
            "decode_inputs_equal_oracle": bool(inputs_ok), "rates": out,
            "oracle_direct": {"requests": len(direct_pool), "gpx_s": round(dpx / t_direct / 1e9, 4),
                              "mismatches_vs_planes": int(direct_bad)},
            "oracle_planes": {"gpx_s": round(planes_px / t_planes / 1e9, 4), "seconds": round(t_planes, 2)},
            "sample": "seeded %.0f %% of each %g-s trace plus every request of >= 32 Mpx, served again "
                      "(resident, batched and per-request modes) and compared in full with windows of the oracle's "
                      "whole-plane encodings and block-wise decodings (%d threads)"
                      % (100 * frac, ctx["seconds"], threads)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline_512(reps=20):
    """The oracle on the 512 x 512 image (seed 1) with the latency leg's
    calls: median time per call on all cores and on one core."""
    import numpy as np

    import oracle as O
    import synth
    img = synth.plane(512, 512, 1)
    one = np.ones(64, np.uint16)
    q10 = O.quantise(img, one, 10)
    out = {"side": 512, "reps": reps}
    for label, th in (("all_cores", _oracle_threads()), ("single_core", 1)):
        calls = {"forward_int32": lambda: O.forward(img, threads=th),
                 "quantise_keep10": lambda: O.quantise(img, one, 10, threads=th),
                 "inverse": lambda: O.inverse(q10, one, 512, 512, threads=th),
                 "roundtrip_keep10": lambda: O.roundtrip(img, one, 10, threads=th)}
        r = {}
        for name, f in calls.items():
            f()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                f()
                ts.append(time.perf_counter() - t0)
            r[name + "_us"] = round(1e6 * sorted(ts)[reps // 2], 1)
        out[label] = dict(r, cores=th)
    return out


def _pool_rate(fn, items, threads, min_s):
    """Runs fn(item) over items on `threads` host threads (one oracle call
    each, single-threaded) until min_s seconds have passed; returns
    (units done, seconds, items done)."""
    from concurrent.futures import ThreadPoolExecutor
    done, units = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while done < len(items) and time.perf_counter() - t0 < min_s:
            chunk = items[done:done + 4 * threads]
            units += sum(ex.map(fn, chunk))
            done += len(chunk)
    return units, time.perf_counter() - t0, done


def cpu_baseline_ragged(ctx, min_s=3.0):
    """The oracle on the ragged images (encode + decode with coefficients,
    as the batched leg), images spread over the host threads, and on one
    core."""
    import oracle as O
    import synth
    buf, off, strides, sizes, qs = ctx

    def one(i):
        img = synth.batch_view(buf, off, strides, sizes, i)
        O.roundtrip(img, qs[i], 64)
        return int(sizes[i][0]) * int(sizes[i][1])

    items = list(range(len(sizes)))
    th = _oracle_threads()
    px, dt, done = _pool_rate(one, items, th, min_s)
    px1, dt1, done1 = _pool_rate(one, items, 1, min_s / 3)
    return {"value": round(px / dt / 1e9, 4), "unit": "Gpixel/s", "cores": th, "kind": "oracle",
            "sample": "encode+decode of the first %d of the 10,000 ragged images (%.2f Gpx, %.1f s), "
                      "one image per thread" % (done, px / 1e9, dt),
            "single_core": {"value": round(px1 / dt1 / 1e9, 4), "unit": "Gpixel/s",
                            "sample": "first %d images in %.1f s" % (done1, dt1)}}


def cpu_baseline_video(ctx, min_s=3.0):
    """The oracle's int8 zigzag encoder on the 4:2:0 frames (luma and chroma
    tables as the video leg), planes spread over the host threads, and on
    one core."""
    import oracle as O
    host, v, frames = ctx
    w, h = v.w, v.h
    fbytes = w * h + 2 * (w // 2) * (h // 2)
    planes = []
    for f in range(frames):
        qy, qc = v.qtables(f)
        o = f * fbytes
        planes += [(o, w, h, qy), (o + w * h, w // 2, h // 2, qc),
                   (o + w * h + (w // 2) * (h // 2), w // 2, h // 2, qc)]

    def one(pl):
        o, pw, ph, Q = pl
        O.quantise_i8_zigzag(host[o:o + pw * ph].reshape(ph, pw), Q)
        return pw * ph

    th = _oracle_threads()
    n, dt, done = _pool_rate(one, planes, th, min_s)
    n1, dt1, done1 = _pool_rate(one, planes, 1, min_s / 3)
    return {"value": round(n / dt / 1e9, 4), "unit": "Gsample/s", "cores": th, "kind": "oracle",
            "sample": "int8 zigzag encode of the first %d of the 768 planes (%.2f G samples, %.1f s), "
                      "one plane per thread" % (done, n / 1e9, dt),
            "single_core": {"value": round(n1 / dt1 / 1e9, 4), "unit": "Gsample/s",
                            "sample": "first %d planes in %.1f s" % (done1, dt1)}}


def spin_cycles(torch, stream, ms):
    """Cycles of torch's spin kernel that hold `stream` for about `ms`
    milliseconds, from one timed spin."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        torch.cuda._sleep(1 << 20)
        a.record(stream)
        torch.cuda._sleep(1 << 22)
        b.record(stream)
    torch.cuda.synchronize()
    return int((1 << 22) * ms / max(a.elapsed_time(b), 1e-3))


def queued_run_ms(torch, stream, f, n, hold):
    """Device time of `n` back-to-back calls of f: queued behind a spin
    kernel, with one event before the first and one after the last, so that
    neither the host's launch time nor per-call event markers enter. Returns
    None if the spin ended before the last call was queued (the run then saw
    an idle queue)."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        torch.cuda._sleep(hold)
    a.record(stream)
    for _ in range(n):
        f()
    b.record(stream)
    in_time = not a.query()
    torch.cuda.synchronize()
    return a.elapsed_time(b) if in_time else None


def plain_leg(tdct, torch, stream, sides=(4096, 8192, 16384), rounds=5, reps=10):
    """One image per call through the plain C-ABI calls: tdct_quantise
    (encode, keep 64) and tdct_inverse (decode) on one blob-field image of
    4096^2, 8192^2 and 16384^2, Q = 1 + 3(i + j); 3 B/px algorithmic against
    8 TB/s. `ms` is the device time per call of a run of back-to-back calls
    (about 1.6 Gpx per run, at least 10 calls) timed with one event pair,
    median of `rounds` runs: the rate of a stream of plain calls. Beside it,
    `ms_event_per_call` is the median of `reps` calls each bracketed by its
    own events, which adds the event markers' overhead (a few microseconds)
    to every call. Both queue the calls behind a spin kernel, so they see
    device time only."""
    import synth
    Q = tdct.qtable(synth.qtable(1, 3))
    hold = spin_cycles(torch, stream, 20.0)
    out = {}
    for side in sides:
        src = torch.from_numpy(synth.plane(side, side, 4242)).cuda()
        q = torch.empty(((side // 8) ** 2, 64), dtype=torch.int16, device="cuda")
        dst = torch.empty_like(src)
        px = side * side
        n = max(10, min(100, int(1.6e9 / px)))
        calls = {"encode": lambda: tdct.tdct_quantise(src, side, side, side, Q, 64, q, stream),
                 "decode": lambda: tdct.tdct_inverse(q, Q, side, side, dst, side, stream)}
        r = {}
        for name, f in calls.items():
            f()
            torch.cuda.synchronize()
            runs, queued = [], True
            for _ in range(rounds):
                t, h = None, hold
                for _ in range(3):  # a slow host: a longer spin, at most twice
                    t = queued_run_ms(torch, stream, f, n, h)
                    if t is not None:
                        break
                    h *= 4
                if t is None:  # still not all queued in time: time it anyway, flagged
                    queued = False
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    for _ in range(n):
                        f()
                    b.record(stream)
                    torch.cuda.synchronize()
                    t = a.elapsed_time(b)
                runs.append(t / n)
            ms = sorted(runs)[rounds // 2]
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            with torch.cuda.stream(stream):
                torch.cuda._sleep(hold)
            ev[0].record(stream)
            for k in range(reps):
                f()
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            per_call = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))[reps // 2]
            gbs = 3 * px / (ms / 1e3) / 1e9
            if not queued:
                log("plain leg: %s at %d^2 was timed with calls the host could not queue ahead" % (name, side))
            r[name] = {"ms": round(ms, 4), "calls_per_run": n, "queued_ahead": queued,
                       "gpx_s": round(px / (ms / 1e3) / 1e9, 1),
                       "gbs": round(gbs, 1), "frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
                       "ms_event_per_call": round(per_call, 4)}
        out[str(side)] = r
        del src, q, dst
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--images", type=int, default=64)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and serving legs")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shape")
    ap.add_argument("--tune", default="",
                    help="fixed launch shapes instead of autotuning: "
                         "'WPG,GPC,TW[,XCD[,PC]]:WPG,GPC,TW[,XCD[,PC]]' for the encoder and the "
                         "decoder (PC: cached pixel accesses)")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="trace length per rate for the resident (served form) and per-request modes")
    ap.add_argument("--serving-batched-seconds", type=float, default=4.0,
                    help="trace length per rate for continuous batching into launched kernels "
                         "(at the workload's rates it takes the per-request path; its burst "
                         "capacity is measured apart)")
    ap.add_argument("--serving-aux-seconds", type=float, default=4.0,
                    help="trace length per rate for host payloads and the burst")
    ap.add_argument("--no-per-image", action="store_true",
                    help="leave out the ragged batch's per-image comparisons (120,000 plain "
                         "launches; for runs under a profiler)")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the zonal-coding quality sweep (PSNR and MSE APE vs the DCT)")
    ap.add_argument("--legs", default="",
                    help="comma-separated subset of the extra legs to run (default: all)")
    ap.add_argument("--config", type=int, choices=sorted(CONFIG_LEGS), default=None,
                    help="one workload beside the headline step: 1 the 512 x 512 latencies, 2 the "
                         "64 x 4096^2 step alone, 3 the 10,000 ragged images, 4 the 4:2:0 video "
                         "frames, 5 the serving streams")
    ap.add_argument("--fused-tune", default="",
                    help="fixed launch shape 'WPG,GPC,TW[,XCD[,PC]]' for the fused round trip")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file (default: $TDCT_TUNE_CACHE, else "
                         "~/.cache/tdct/autotune.json; '' turns it off): shapes tuned by an earlier "
                         "run of the same kernel sources on this GPU architecture are taken without "
                         "timing candidates again")
    ap.add_argument("--burst-only", default="",
                    help="only serve the 5000 req/s trace's requests arriving at once in these "
                         "comma-separated modes (batched, per_request, resident), for profiling")
    ap.add_argument("--burst-reps", type=int, default=3)
    ap.add_argument("--resident-workers", type=int, default=0,
                    help="worker waves of the resident kernel (0: four per compute unit)")
    ap.add_argument("--copy-only", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.config is not None:
        if args.legs or args.no_extras:
            ap.error("--config names the legs itself (no --legs or --no-extras with it)")
        args.legs = CONFIG_LEGS[args.config]
        args.no_extras = not args.legs

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the codec shards by image (or block range) with "
              "no cross-GPU exchange, so each GPU runs this same step on its share; "
              "--gpus %d is not run." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1702_00817_amd as tdct
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    cache_path = args.tune_cache
    if cache_path is None:
        cache_path = os.environ.get("TDCT_TUNE_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "tdct", "autotune.json")
    if cache_path:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        except OSError:
            pass  # the cache then counts write errors
        try:
            tdct.tdct_tune_cache_open(cache_path)
        except tdct.TdctError as e:  # a file not in the cache's format: tune without it
            log("autotune cache %s not used: %s" % (cache_path, e))
            tdct.tdct_tune_cache_open(None)
    else:
        tdct.tdct_tune_cache_open(None)
    cache_at_start = tdct.tdct_tune_cache_info()

    if args.burst_only:
        print(json.dumps({"burst": burst_leg(tdct, torch, args.burst_only.split(","), args.burst_reps,
                                             resident_workers=args.resident_workers)}), flush=True)
        return

    if args.copy_only:
        # A plain device copy of a known size: the calibration kernel for the
        # HBM counters and the practical copy ceiling of the part.
        n = args.copy_only << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        b.copy_(a)
        for k in range(5):
            ev[k].record(stream)
            b.copy_(a)
        ev[5].record(stream)
        torch.cuda.synchronize()
        ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(5))[2]
        print(json.dumps({"copy_bytes": n, "launches": 6, "median_ms": round(ms, 4),
                          "copy_gbs": round(2 * n / (ms / 1e3) / 1e9, 1)}))
        return

    t_start = time.perf_counter()
    W = make_large_batch(tdct, torch, args.images, args.side)
    fixed = [None, None]
    if args.tune:
        for k, part in enumerate(args.tune.split(":")):
            fixed[k] = parse_tune(part)
    pe = tdct.tdct_batch_plan(W["enc"], W["qs"], tune=fixed[0])
    pd = tdct.tdct_batch_plan(W["dec"], W["qs"], tune=fixed[1])
    tune_choice = None
    try:
        tune_e, tune_d = fixed
        if not args.no_tune and not args.tune:
            hits0 = tdct.tdct_tune_cache_info()["hits"]
            tune_e = tdct.tdct_autotune(pe, stream, reps=3)
            tune_d = tdct.tdct_autotune(pd, stream, reps=3)
            log("autotune: encode %s decode %s" % (tune_e, tune_d))
            if tdct.tdct_tune_cache_info()["hits"] > hits0:
                # shapes from the cache: the candidates' ~0.5 s of launches,
                # which also bring the clocks up, did not run; run as long
                # untimed before the warm-up steps
                t_end = time.perf_counter() + 0.5
                while time.perf_counter() < t_end:
                    tdct.tdct_batch_run(pe, stream)
                    tdct.tdct_batch_run(pd, stream)
                    torch.cuda.synchronize()
            ref = [parse_tune(x) for x in REFERENCE_TUNE.split(":")]
            if [tune_e, tune_d] != ref:
                # the autotuned pair against the reference pair, in whole steps
                k, med = step_choice(tdct, torch, W, [(tune_e, tune_d), tuple(ref)], stream)
                tune_choice = {"autotuned_ms_per_step": round(med[0], 4), "reference": REFERENCE_TUNE,
                               "reference_ms_per_step": round(med[1], 4),
                               "kept": ("autotuned", "reference")[k]}
                log("launch shapes in whole steps: %s" % json.dumps(tune_choice))
                if k == 1:
                    tdct.tdct_plan_free(pe)
                    tdct.tdct_plan_free(pd)
                    pe = pd = None
                    tune_e, tune_d = ref
                    pe = tdct.tdct_batch_plan(W["enc"], W["qs"], tune=tune_e)
                    pd = tdct.tdct_batch_plan(W["dec"], W["qs"], tune=tune_d)
        wall, enc_ms, dec_ms = time_steps(tdct, torch, pe, pd, args.steps, args.warmup, stream)
    finally:
        if pe is not None:
            tdct.tdct_plan_free(pe)
        if pd is not None:
            tdct.tdct_plan_free(pd)
    px = W["pixels"]
    ms_step = wall / args.steps * 1e3
    enc_avg, dec_avg = sum(enc_ms) / len(enc_ms), sum(dec_ms) / len(dec_ms)
    dom_name, dom_ms = ("encode", enc_avg) if enc_avg >= dec_avg else ("decode", dec_avg)
    bytes_launch = 3 * px
    achieved = bytes_launch / (dom_ms / 1e3) / 1e9
    traffic = load_traffic(dom_name + "_64x4096")
    # the part's practical rate for the dominant kernel's access mix: the
    # same bytes streamed with no arithmetic (1 read : 2 writes for the
    # encoder, 2 : 1 for the decoder)
    mix = "read1_write2" if dom_name == "encode" else "read2_write1"
    ceiling = ceiling_leg(tdct, torch, stream, names=(mix,))[mix]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
            "stream_ceiling": {"mix": mix, "gbs": ceiling, "frac": round(achieved / ceiling, 4)},
            "kernel": "batch_kernel (%s), 64 x 4096^2, %d B/px algorithmic" % (dom_name, 3),
            "encode_ms": round(enc_avg, 4), "decode_ms": round(dec_avg, 4),
            "encode_gbs": round(bytes_launch / (enc_avg / 1e3) / 1e9, 1),
            "decode_gbs": round(bytes_launch / (dec_avg / 1e3) / 1e9, 1)}
    result = {
        "metric": "Gpixel/s encode+decode (64 x 4096x4096 uint8, fused kernels), % HBM peak",
        "value": round(px / (ms_step / 1e3) / 1e9, 2),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic (seeded blob fields + noise)",
        "config": {"workload": "64 x 4096x4096 uint8 images, per-image Q_ij = 1 + s(i+j), "
                               "encode (int16 out) + decode (uint8 out)",
                   "images": args.images, "side": args.side, "pixels": px,
                   "tune": {"encode": tune_e, "decode": tune_d}, "tune_choice": tune_choice},
        "roofline": roof,
    }
    # wall seconds per part of the run
    leg_seconds = result["config"]["leg_seconds"] = {}
    clock = [t_start, "headline"]

    def mark(name):
        """Closes the running part's clock and starts `name`'s (None: stop)."""
        now = time.perf_counter()
        leg_seconds[clock[1]] = round(now - clock[0], 1)
        log("%s: %.1f s" % (clock[1], now - clock[0]))
        clock[:] = [now, name]

    if not args.no_cpu:
        mark("cpu_baseline")
        log("cpu baseline (oracle)...")
        result["cpu_baseline"] = cpu_baseline(W)
    legs = set(args.legs.split(",")) if args.legs else None

    def want(name):
        return not args.no_extras and (legs is None or name in legs)

    def cpu(name, f, *a):
        """An oracle timing beside a leg, under cpu_baseline."""
        if not args.no_cpu:
            log("cpu baseline (oracle) for %s..." % name)
            result.setdefault("cpu_baseline", {})[name] = f(*a)

    if want("fused_roundtrip"):
        mark("fused_roundtrip")
        log("fused round-trip leg...")
        ft = None
        if args.fused_tune:
            ft = parse_tune(args.fused_tune)
        result["fused_roundtrip"] = fused_leg(tdct, torch, W, stream, tune=ft)
    if want("per_image"):
        mark("per_image")
        log("per-image launches of the same batch...")
        result["per_image"] = per_image_leg(tdct, torch, W, stream)
    if want("forward"):
        mark("forward")
        log("int32 forward leg...")
        result["forward"] = forward_leg(tdct, torch, W, stream)
        torch.cuda.empty_cache()
    del W
    torch.cuda.empty_cache()
    if want("plain"):
        mark("plain")
        log("plain-call leg (one image per call)...")
        result["plain"] = plain_leg(tdct, torch, stream)
    if want("latency_512"):
        mark("latency_512")
        log("latency leg (512 x 512)...")
        result["latency_512"] = latency_leg(tdct, torch, stream)
        cpu("latency_512", cpu_baseline_512)
    ceil = {}
    if want("ceiling") or want("video") or want("batched"):
        mark("ceiling")
        log("ceiling leg...")
        ceil = ceiling_leg(tdct, torch, stream)
        if want("ceiling"):
            result["ceiling"] = ceil
    if want("video"):
        mark("video")
        log("video leg...")
        vctx, result["video"] = video_leg(tdct, torch, stream)
        roof = result["video"]["roofline"]
        roof["stream_ceiling"] = {"mix": "copy", "gbs": ceil["copy"],
                                  "frac": round(roof["achieved"] / ceil["copy"], 4)}
        torch.cuda.empty_cache()
        cpu("video", cpu_baseline_video, vctx)
        del vctx
    if want("batched"):
        mark("batched")
        log("batched leg...")
        bctx, result["batched"] = batched_leg(tdct, torch, stream, per_image=not args.no_per_image)
        roof = result["batched"]["roofline"]
        roof["stream_ceiling"] = {"mix": "read1_write3", "gbs": ceil["read1_write3"],
                                  "frac": round(roof["achieved"] / ceil["read1_write3"], 4)}
        torch.cuda.empty_cache()
        cpu("batched", cpu_baseline_ragged, bctx)
        del bctx
    if want("serving"):
        mark("serving")
        log("serving leg...")
        result["serving"], sctx = serving_leg(tdct, torch, args.serving_seconds, args.serving_aux_seconds,
                                              batched_seconds=args.serving_batched_seconds)
        mark("serving_check")
        cpu("serving", cpu_baseline_serving, tdct, torch, sctx, (200, 1000, 5000))
        del sctx
        torch.cuda.empty_cache()
    if want("quality") and not args.no_quality:
        mark("quality")
        log("quality leg...")
        result["quality"] = quality_leg(tdct, torch, stream)
    mark(None)
    leg_seconds.pop(None, None)
    leg_seconds["total"] = round(time.perf_counter() - t_start, 1)
    info = tdct.tdct_tune_cache_info()
    result["config"]["tune_cache"] = {"path": cache_path or None, "entries_at_start": cache_at_start["entries"],
                                      "hits": info["hits"], "misses": info["misses"], "stores": info["stores"],
                                      "write_errors": info["write_errors"], "batch_hits": info["batch_hits"],
                                      "batch_misses": info["batch_misses"]}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
