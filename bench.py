"""Benchmark: APAX profile + encode + decode of a 4096 x 4096 fp32 field
(Gaussian random field, k^-3 spectrum, scaled to [-1e3, 1e3], plus white
noise 1e-2) at a fixed 4:1 rate with the profiler's attenuation, 16x16 bricks,
on one MI355X.

One step = one pass of the whole hot path over one field: the profile
(operating point, stream mask, metrics, curve) and the encode at the profiled
operating point in one launch sequence (apax_profile_encode_async: the
profile's metrics pass runs the encoder's per-block gain search and stream
choice and records them, and the encode after it only quantizes, forms each
block's stream and packs -- the same bytes as apax_encode with
APAX_CODE_PROFILED), then apax_decode, enqueued with no host round trip.  The
profile's centred and curve passes run on a second stream from the end of
its metrics pass on, beside the encode and decode.  Inputs are resident in HBM before
timing; steps rotate over several copies so the 256 MB Infinity Cache cannot
serve them.  The steps are timed four ways: enqueued eagerly one after the
other, as hipGraphs of the same enqueue sequence (one per copy), and
pipelined (step i + 1's profile starts while step i's last profile passes
and its decode finish on the second stream; two profile workspaces
alternate), enqueued eagerly and as graph replays on two streams; the step
time is the fastest loop (all are reported, each
checked: every copy decodes to the same field).  After the timed loop the last
profile is read back and the decoded field checked against its correlation,
and every graph replay's decode against the eager one.  Also timed, outside
the step: encode and decode of the other workloads (the int16 time series,
the fp64 3-d field at fixed quality, the same field at 3:1 and 10:1).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "encode/decode GB/s (uncompressed bytes) and % HBM peak at fixed ratio, 1 GPU"


def read_traffic(kernel: str):
    """HBM bytes per launch from the rocprofv3 PMC summary, if it was taken on
    the current kernel sources (a source digest is recorded with it)."""
    path = os.path.join(ROOT, "profiles", "traffic_c1.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest():
        return None
    v = kv.get(f"{kernel}_hbm_bytes_per_launch")
    return float(v) if v else None


# the sources of the kernels a C1 step launches (the traffic summary holds
# for them as long as none of these changes)
C1_KERNEL_SOURCES = ("block.h", "codec.h", "kernels.h", "profile.hip", "encode.hip", "encode_tile.h",
                     "decode.hip", "decode_tile.h")


def source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1303_4994_amd", "csrc")
    for f in C1_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_KEYS = {  # kernel (trace name) -> key of its bytes per launch
    "apax::k_encode<float, 64, 2, 4, false>": "k_encode",
    "apax::k_decode<float, 64, 2, 4>": "k_decode",
    "apax::k_profile<float, 64, 2, 1>": "k_profile_metrics",
    "apax::k_profile<float, 64, 2, 5>": "k_profile_metrics_encode",
    "apax::k_profile<float, 64, 2, 4>": "k_profile_curve",
    "apax::k_profile<float, 64, 2, 3>": "k_profile_centred",
    "apax::k_profile<float, 64, 2, 2>": "k_profile_fits",
    "apax::k_probe_all<float, 64, 2>": "k_probe_all",
    "apax::k_pmax<float>": "k_pmax",
}


def traffic_summary(fetch_csv: str, write_csv: str, out_path: str, command: str):
    """HBM bytes per launch of the codec kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for the plain 64 MiB copy of --copy-probe."""
    import csv
    import collections

    def per_kernel(path, counter):
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                vals[r["Kernel_Name"].split("(")[0]].append(float(r["Counter_Value"]))
        return vals
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    field = 64 * 1024 * 1024

    def factor(vals, pick):
        """field bytes / the counter's mean reading (bytes) for the calibration kernel"""
        big = [v for k, vs in vals.items() if pick(k) for v in vs if v * 1024 > field / 4]
        return field / (sum(big) / len(big) * 1024) if big else None
    # reads: the plain copy of the field (its reads are whole 128-byte lines, as
    # the codec kernels' are); writes: the write-only fill of a field (the
    # copy's WRITE_SIZE reads about 1.4 times the bytes it writes)
    copyk = lambda k: "copy" in k.lower() and "apax" not in k
    ff = factor(f, copyk)
    fw = factor(w, lambda k: "FillFunctor" in k)
    f_sum = factor(f, lambda k: "reduce_kernel" in k)
    w_copy = factor(w, copyk)
    lines = ["# HBM traffic of the codec kernels, C1 workload (4096x4096 fp32, 16x16 bricks, 4:1)",
             f"# command (fetch): {command.format(c='FETCH_SIZE', d='fetch')}",
             f"# command (write): {command.format(c='WRITE_SIZE', d='write')}",
             f"# summary: python3 bench.py --traffic-from {fetch_csv} {write_csv}",
             "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch (raw_* below); the calibrated bytes scale",
             "# FETCH_SIZE by 64 MiB over its reading for a plain copy of a 64 MiB field and",
             "# WRITE_SIZE by 64 MiB over its reading for a write-only fill of a 64 MiB field",
             "# (for reference: the same factors from a read-only sum and from the copy's writes)",
             f"source_sha256: {source_digest()}",
             f"calibration_factor_fetch: {ff}", f"calibration_factor_write: {fw}",
             f"reference_factor_fetch_sum: {f_sum}", f"reference_factor_write_copy: {w_copy}"]
    for k in sorted(set(f) | set(w)):
        if not k.startswith("void apax::") and "apax::" not in k:
            continue
        fv = sum(f.get(k, [0])) / max(1, len(f.get(k, [0])))
        wv = sum(w.get(k, [0])) / max(1, len(w.get(k, [0])))
        name = k.split("apax::")[1].split("<")[0]
        fb = fv * 1024 * (ff or 1.0)
        wb = wv * 1024 * (fw or 1.0)
        lines.append(f"{name}<{k.split('<', 1)[1] if '<' in k else ''}: fetch_bytes={fb:.0f} write_bytes={wb:.0f} "
                     f"raw_fetch_KiB={fv:.0f} raw_write_KiB={wv:.0f}")
        key = TRAFFIC_KEYS.get(k.replace("void ", "").split("(")[0].strip())
        if key:
            lines.append(f"{key}_hbm_bytes_per_launch: {fb + wb:.0f}")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d /root/repo/gpurun_out/kt_c1 "
             "-o kt -- python3 /root/repo/bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-workloads")
TRACE_WL_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d /root/repo/gpurun_out/kt_wl "
                "-o kt -- python3 /root/repo/bench.py --steps 2 --warmup 1 --no-cpu-baseline")
INSTMIX_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 150 rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU "
               "SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM SQ_BUSY_CYCLES --output-format csv "
               "-d /root/repo/gpurun_out/pmc_sq -o p -- python3 /root/repo/bench.py --steps 2 --warmup 1 "
               "--no-cpu-baseline --no-workloads --copy-probe")


def trace_summary(db_path: str, out_path: str, workloads: bool = False):
    """Per-kernel durations from a rocprofv3 kernel-trace results database:
    all launches, and the launches that ran alone (the step overlaps two
    streams, so launches that shared the GPU run longer), plus one step's
    launch sequence.  workloads: the trace of a whole bench run (the step and
    the other workloads' encode and decode kernels)."""
    import collections
    import sqlite3
    rows = list(sqlite3.connect(db_path).execute("select name, start, end from kernels order by start"))
    every, alone = collections.defaultdict(list), collections.defaultdict(list)
    latest = 0
    for i, (n, a, b) in enumerate(rows):
        nm = n.split("(")[0].replace("void ", "")
        every[nm].append((b - a) / 1e3)
        nxt = rows[i + 1][1] if i + 1 < len(rows) else float("inf")
        if latest <= a and nxt >= b:
            alone[nm].append((b - a) / 1e3)
        latest = max(latest, b)
    if workloads:
        out = ["# rocprofv3 kernel trace of a whole bench run: the C1 step and, timed alone, the encode and",
               "# decode kernels of the int16 time series (2 MiB and 64 MiB, lossless, 256-sample blocks:",
               "# <short, 64, 1>), the C1 field at 3:1 and 10:1 (<float, 64, 2>) and the fp64 3-d field at",
               "# fixed quality (<double, 32, 3>, 4x4x8 bricks); variable-size encodes run",
               "# k_encode_reset, k_encode_size, k_encode_scan, k_encode_emit",
               f"# command: {TRACE_WL_CMD}",
               f"# summary: python3 bench.py --trace-workloads-from {db_path}",
               "# durations in microseconds; iso_avg_us: launches with no other kernel running",
               f"{'kernel':52s} {'calls':>6s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'total_us':>9s} "
               f"{'iso_n':>6s} {'iso_avg_us':>10s}"]
        for k, v in sorted(every.items(), key=lambda kv: -sum(kv[1])):
            if "apax::" not in k:
                continue
            w = alone.get(k, [])
            ia = f"{sum(w) / len(w):10.2f}" if w else f"{'-':>10s}"
            out.append(f"{k[:52]:52s} {len(v):6d} {sum(v) / len(v):8.2f} {min(v):8.2f} {max(v):8.2f} "
                       f"{sum(v):9.1f} {len(w):6d} {ia}")
        open(out_path, "w").write("\n".join(out) + "\n")
        print("\n".join(out))
        return
    out = ["# rocprofv3 kernel trace, C1 bench (4096x4096 fp32, 16x16 bricks, fixed rate 4:1)",
           f"# command: {TRACE_CMD}",
           f"# summary: python3 bench.py --trace-from {db_path}",
           "# durations in microseconds; per bench step: k_clear; k_pmax + k_pmax_reduce; 3 bisection probes",
           "# k_probe_all (all 8 codes of a launch per tile) + k_reduce<2, false>; histogram k_profile<.., 2>",
           "# + k_reduce<2, true>; metrics",
           "# k_profile<.., 5> (k_encode_header first: the stream header), which also writes every block of",
           "# the stream at its code and stream, then k_decode; curve k_profile<.., 4> + k_reduce<4, false>",
           "# beside it on a second stream, then there k_reduce<1, false> (the metrics' reduction), centred",
           "# k_profile<.., 3> + k_reduce<3, false>.",
           "# The run also times back-to-back standalone",
           "# k_encode / k_decode launches, event-bracketed profiles and the calls outside the step;",
           "# iso_avg_us is the mean over launches with no other kernel running (the per-launch figure",
           "# bench.py reports)",
           f"{'kernel':52s} {'calls':>6s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'total_us':>9s} "
           f"{'iso_n':>6s} {'iso_avg_us':>10s}"]
    for k, v in sorted(every.items(), key=lambda kv: -sum(kv[1])):
        if "apax::" not in k:
            continue
        w = alone.get(k, [])
        ia = f"{sum(w) / len(w):10.2f}" if w else f"{'-':>10s}"
        out.append(f"{k[:52]:52s} {len(v):6d} {sum(v) / len(v):8.2f} {min(v):8.2f} {max(v):8.2f} "
                   f"{sum(v):9.1f} {len(w):6d} {ia}")
    starts = [i for i, r in enumerate(rows) if "k_pmax<" in r[0]]
    if len(starts) > 3:
        seq = rows[starts[3]:starts[3] + 18]
        out += ["", "# one step of the timed loop (start offset and duration, us)"]
        for n, a, b in seq:
            nm = n.split("(")[0].replace("void ", "")
            if "apax::" in nm:
                out.append(f"{(a - seq[0][1]) / 1e3:9.1f} {(b - a) / 1e3:9.2f}  {nm}")
    open(out_path, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def instmix_summary(csv_path: str, out_path: str):
    """Instruction counts per wave and VALU issue time per dispatch from a
    rocprofv3 --pmc run of the SQ counters."""
    import collections
    import csv
    disp = collections.OrderedDict()
    for r in csv.DictReader(open(csv_path)):
        d = disp.setdefault((r["Dispatch_Id"], r["Kernel_Name"]), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    agg = collections.OrderedDict()
    for (_, name), d in disp.items():
        a = agg.setdefault(name.split("(")[0].replace("void ", ""), collections.Counter())
        a["n"] += 1
        for k, v in d.items():
            a[k] += v
    out = ["# rocprofv3 instruction counters per dispatch, C1 bench (4096x4096 fp32, 16x16 bricks, 4:1)",
           f"# command: {INSTMIX_CMD}",
           f"# summary: python3 bench.py --instmix-from {csv_path}",
           "# values are means over the dispatches of each kernel; per-wave figures divide by SQ_WAVES",
           "# (k_encode / k_decode: one wave per 256-sample block; the profile passes loop over blocks)",
           "# VALU_Ginstr: wave-level VALU instructions per dispatch (1e9); at one wave-instruction per CU",
           "# per clock (256 CUs x 2.4 GHz = 614 G/s) this is the VALU issue time",
           f"{'kernel':46s} {'n':>4s} {'waves':>8s} {'VALU/wave':>10s} {'SALU/wave':>10s} {'LDS/wave':>9s} "
           f"{'VMEM/wave':>10s} {'VALU_Ginstr':>12s} {'issue_us':>9s}"]
    for nm, a in agg.items():
        if "apax::" not in nm:
            continue
        n = a["n"]
        w = a["SQ_WAVES"] / n
        valu = a["SQ_INSTS_VALU"] / n
        out.append(f"{nm[:46]:46s} {n:4d} {w:8.0f} {valu / w:10.1f} {a['SQ_INSTS_SALU'] / n / w:10.1f} "
                   f"{a['SQ_INSTS_LDS'] / n / w:9.1f} {a['SQ_INSTS_VMEM'] / n / w:10.1f} {valu / 1e9:12.4f} "
                   f"{valu / 614e9 * 1e6:9.1f}")
    open(out_path, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def host_cpu():
    """Model name and logical core count of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count()}


def cpu_baseline(x, params):
    """The oracle (single-threaded C) on the full C1 field: profile, encode and
    decode each timed, and the whole pass."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    prof = O.profile_dict(O.profile(x, params))
    t1 = time.perf_counter()
    p = dict(params, code=prof["code"], stream_mask=prof["stream_mask"] & 0x7F)
    s = O.encode(x, p)
    t2 = time.perf_counter()
    O.decode(s)
    t3 = time.perf_counter()
    dt = t3 - t0
    mb = x.nbytes / 1e6
    return {"value": round(x.nbytes / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "the full 4096x4096 fp32 field, one profile+encode+decode pass, "
                      "single-threaded C oracle", "seconds": round(dt, 3),
            "profile_MBps": round(mb / (t1 - t0), 2), "encode_MBps": round(mb / (t2 - t1), 2),
            "decode_MBps": round(mb / (t3 - t2), 2), "host": host_cpu()}


# The paper's throughput figures for this path (other implementations and
# hardware: context, not the target)
PAPER_THROUGHPUT = {
    "software_encode_MBps": 130, "software_decode_MBps": 170,
    "software": "one x86 core at the profiler's operating points over the paper's datasets (Sec. 4, Sec. 7)",
    "table1_software_MBps_per_core": 150, "table1_software": "x86 core, about 50 instructions per sample",
    "table1_fpga_MBps_per_instance": 600, "table1_fpga": "FPGA netlist, encoder about 4000 and decoder about "
                                                          "3500 6-input LUTs",
    "table1_soc_GBps_per_instance": 1.5, "table1_soc": "SoC IP block, encoder + decoder about 220k gates "
                                                      "(under 0.1 mm^2 in 28 nm)",
}


def cpu_baseline_items(arrays, op, budget_bytes=192 << 20):
    """Oracle timed on the first items of a batch or request mix (about
    budget_bytes of input): encode (op "encode") or encode + decode of each."""
    from oracle import oracle as O
    sample, nb = [], 0
    for x, p in arrays:
        if nb >= budget_bytes:
            break
        sample.append((x.cpu().numpy(), p))
        nb += sample[-1][0].nbytes
    t0 = time.perf_counter()
    for xh, p in sample:
        st = O.encode(xh, p)
        if op != "encode":
            O.decode(st)
    dt = time.perf_counter() - t0
    what = "encode" if op == "encode" else "encode + decode"
    return {"value": round(nb / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {len(sample)} items ({nb / 1e6:.0f} MB), {what} of each, "
                      "single-threaded C oracle", "seconds": round(dt, 3)}


def codec_workload(A, dev, name, x, params, copies, reps, profile=True):
    """Encode and decode GB/s (input bytes) of one workload: the operating
    point from apax_profile (fixed rate / quality), then back-to-back
    launches over `copies` rotating device copies between HIP events."""
    import torch
    dtype = {1: torch.int8, 2: torch.int16, 4: torch.float32, 8: torch.float64}[x.itemsize]
    if x.dtype.kind == "i" and x.itemsize == 4:
        dtype = torch.int32
    xs = [torch.from_numpy(x).to(dev) for _ in range(copies)]
    ws = A.workspace(dtype, x.shape, params, dev)
    p = dict(params)
    prof = None
    if profile:
        prof = A.apax_profile(xs[0], params, ws=ws)
        p = dict(params, code=prof["code"], stream_mask=prof["stream_mask"] & (0x7F if params["mode"] ==
                                                                                 "fixed_rate" else 0xFF))
    bound = A.apax_encode_bound(dtype, x.shape, p)
    bufs = [torch.empty(bound, dtype=torch.uint8, device=dev) for _ in range(copies)]
    nbs = [torch.empty(1, dtype=torch.int64, device=dev) for _ in range(copies)]
    ys = [torch.empty_like(xs[0]) for _ in range(copies)]
    stream = torch.cuda.current_stream()
    A.apax_status_clear(ws)
    for k in range(copies):
        A.apax_encode(xs[k], p, out=bufs[k], nbytes=nbs[k], ws=ws, clear_status=False)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    nb = int(nbs[0].item())
    hdr = bytes(bufs[0][:64].cpu().numpy().tobytes())
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    for k in range(reps):
        A.apax_encode(xs[k % copies], p, out=bufs[k % copies], nbytes=nbs[k % copies], ws=ws,
                      clear_status=False)
    e1.record(stream)
    for k in range(reps):
        A.apax_decode(bufs[k % copies], nb, hdr=hdr, y=ys[k % copies], ws=ws, clear_status=False)
    e2.record(stream)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    for k in range(copies):  # every copy gave the same stream and decoded to the same array
        assert int(nbs[k].item()) == nb and torch.equal(bufs[k][:nb], bufs[0][:nb])
        assert torch.equal(ys[k], ys[0])
    if params["mode"] == "lossless":
        assert torch.equal(ys[0], xs[0])
    enc_ms, dec_ms = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
    # the same launches replayed as hipGraphs (one graph holds an encode of
    # every copy, another a decode of every copy): small arrays are bound by
    # the host's enqueue of eager launches, which a graph replay takes away
    enc_g = dec_g = None
    try:
        ge, gd = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(ge):
            for k in range(copies):
                A.apax_encode(xs[k], p, out=bufs[k], nbytes=nbs[k], ws=ws, clear_status=False)
        with torch.cuda.graph(gd):
            for k in range(copies):
                A.apax_decode(bufs[k], nb, hdr=hdr, y=ys[k], ws=ws, clear_status=False)
        nrep = max(1, reps // copies)
        ge.replay()
        gd.replay()
        torch.cuda.synchronize()
        g0, g1, g2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        g0.record(stream)
        for _ in range(nrep):
            ge.replay()
        g1.record(stream)
        for _ in range(nrep):
            gd.replay()
        g2.record(stream)
        torch.cuda.synchronize()
        assert A.apax_status(ws) == 0
        for k in range(copies):
            assert int(nbs[k].item()) == nb and torch.equal(bufs[k][:nb], bufs[0][:nb])
            assert torch.equal(ys[k], ys[0])
        enc_g = g0.elapsed_time(g1) / (nrep * copies)
        dec_g = g1.elapsed_time(g2) / (nrep * copies)
        del ge, gd
    except RuntimeError as exc:  # capture refused: the eager figures stand
        log(f"{name}: graph timing not used: {exc}")
    eager_enc_ms, eager_dec_ms = enc_ms, dec_ms
    if enc_g is not None:
        enc_ms, dec_ms = min(enc_ms, enc_g), min(dec_ms, dec_g)
    enc = x.nbytes / (enc_ms * 1e-3) / 1e9
    dec = x.nbytes / (dec_ms * 1e-3) / 1e9
    out = {"workload": name, "mode": params["mode"], "input_bytes": x.nbytes, "stream_bytes": nb,
           "ratio": round(x.nbytes / nb, 4), "encode_GBps": round(enc, 2), "decode_GBps": round(dec, 2),
           "encode_pct_hbm": round(100 * enc / HBM_PEAK_GBPS, 2),
           "decode_pct_hbm": round(100 * dec / HBM_PEAK_GBPS, 2),
           "encode_us": round(1e3 * enc_ms, 2), "decode_us": round(1e3 * dec_ms, 2),
           "eager_encode_us": round(1e3 * eager_enc_ms, 2), "eager_decode_us": round(1e3 * eager_dec_ms, 2),
           "timing": "faster of eager back-to-back launches and hipGraph replays of one launch per copy",
           "copies_rotated": copies, "launches": reps}
    if prof is not None:
        out["code"] = prof["code"]
        out["r"] = prof["metrics"]["r"]
    del xs, bufs, ys
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--copies", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="c1: skip the C0 / C2 / 3:1 / 10:1 encode and decode lines")
    ap.add_argument("--workload", choices=("c1", "batch", "serve"), default="c1",
                    help="c1: the headline single-array path; batch: many arrays per persistent "
                         "launch vs separate launches; serve: Poisson request stream")
    ap.add_argument("--items", type=int, default=4096, help="batch: number of arrays")
    ap.add_argument("--requests", type=int, default=200000, help="serve: number of requests")
    ap.add_argument("--serve-items", type=int, default=1000,
                    help="serve: distinct device-resident items the requests cycle over")
    ap.add_argument("--rho", type=float, default=0.8, help="serve: offered load / plain throughput")
    ap.add_argument("--pool", type=int, default=1 << 26, help="batch/serve: samples per pool")
    ap.add_argument("--copy-probe", action="store_true",
                    help="c1: also run a plain 64 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--trace-from", metavar="RESULTS_DB",
                    help="write profiles/kernels_c1_bench.txt from a rocprofv3 kernel-trace results database")
    ap.add_argument("--trace-workloads-from", metavar="RESULTS_DB",
                    help="write profiles/kernels_workloads.txt from the kernel trace of a whole bench run")
    ap.add_argument("--instmix-from", metavar="COUNTER_CSV",
                    help="write profiles/pmc_c1_instmix.txt from a rocprofv3 --pmc SQ counter CSV")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_c1.txt from two rocprofv3 --pmc counter CSVs")
    args = ap.parse_args()
    if args.trace_from:
        trace_summary(args.trace_from, os.path.join(ROOT, "profiles", "kernels_c1_bench.txt"))
        return
    if args.trace_workloads_from:
        trace_summary(args.trace_workloads_from, os.path.join(ROOT, "profiles", "kernels_workloads.txt"),
                      workloads=True)
        return
    if args.instmix_from:
        instmix_summary(args.instmix_from, os.path.join(ROOT, "profiles", "pmc_c1_instmix.txt"))
        return
    if args.traffic_from:
        cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 150 rocprofv3 --pmc {c} --output-format csv "
               "-d /root/repo/gpurun_out/pmc_{d} -o p -- python3 /root/repo/bench.py --steps 2 --warmup 1 "
               "--no-cpu-baseline --no-workloads --copy-probe")
        traffic_summary(args.traffic_from[0], args.traffic_from[1],
                        os.path.join(ROOT, "profiles", "traffic_c1.txt"), cmd)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU design is described, not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)

    import numpy as np
    import torch

    import synth
    from paper_1303_4994_amd import apax as A

    dev = torch.device("cuda:0")
    x = synth.grf2d(4096, 4096)
    params = {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}
    nbytes_in = x.nbytes
    R = max(1, args.copies)
    xs = [torch.from_numpy(x).to(dev) for _ in range(R)]
    ws = A.workspace(torch.float32, x.shape, params, dev)
    bound = A.apax_encode_bound(torch.float32, x.shape, dict(params, code=0))
    bufs = [torch.empty(bound, dtype=torch.uint8, device=dev) for _ in range(R)]
    ys = [torch.empty_like(xs[0]) for _ in range(R)]
    nbt = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    p_dev = dict(params, code=A.CODE_PROFILED)
    # two streams: the profile up to its metrics pass, then the encode (taken
    # from that pass's per-block results) and the decode of its stream on
    # `stream` (apax_profile_encode_async); the profile's centred and curve
    # passes on `side` from the end of the metrics pass on, beside the encode
    # and decode; `stream` joins `side` at the end.  The decode has its own
    # workspace.
    side = torch.cuda.Stream()
    ws_dec = A.workspace(torch.float32, x.shape, params, dev)
    ev_fork = torch.cuda.Event()

    def step(i, ev=None):
        xi = xs[i % R]
        if ev is not None:
            ev[0].record(stream)
        A.apax_profile_encode_async(xi, params, ws, out=bufs[i % R], nbytes=nbt, stream=stream, side=side,
                                    forked=ev_fork)
        A.apax_decode(bufs[i % R], bound, hdr=step.hdr, y=ys[i % R], ws=ws_dec, stream=stream,
                      clear_status=False)
        if ev is not None:
            ev[1].record(side)
        stream.wait_stream(side)

    # first pass: the fused profile + encode writes the stream of an encode at
    # the host-read operating point, byte for byte; its header serves the
    # decodes (the decoder compares it with each stream's own header on the
    # device)
    prof0 = A.apax_profile(xs[0], params, ws=ws)
    p0 = dict(params, code=prof0["code"], stream_mask=prof0["stream_mask"] & 0x7F)
    A.apax_encode(xs[0], p0, out=bufs[0], nbytes=nbt, ws=ws)
    torch.cuda.synchronize()
    step.hdr = bytes(bufs[0][:64].cpu().numpy().tobytes())
    A.apax_status_clear(ws)
    A.apax_status_clear(ws_dec)
    step(1)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0 and A.apax_status(ws_dec) == 0
    assert int(nbt.item()) == bound
    assert torch.equal(bufs[0], bufs[1 % R])
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0 and A.apax_status(ws_dec) == 0

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert A.apax_status(ws) == 0 and A.apax_status(ws_dec) == 0
    prof = A.apax_profile_read(xs[(args.steps - 1) % R], params, ws)
    assert prof["code"] == prof0["code"] and prof["stream_mask"] == prof0["stream_mask"]
    for k in range(1, min(R, args.steps)):  # every copy decoded to the same field
        assert torch.equal(ys[k], ys[0])
    y_serial = ys[0].clone()
    ms_step_eager = (t1 - t0) * 1e3 / args.steps

    # the same steps pipelined: step i + 1's profile starts on `stream` as
    # soon as step i's encode is enqueued, while step i's last profile
    # passes and its decode finish on `side`.  Two profile workspaces
    # alternate (a step waits until the step before last has released its
    # workspace); every decode reads its own copy's stream and writes its own
    # output, so no step's data is shared with the one beside it
    ws2 = A.workspace(torch.float32, x.shape, params, dev)
    wsp, nbp = [ws, ws2], [nbt, torch.empty(1, dtype=torch.int64, device=dev)]
    ev_encp = [torch.cuda.Event(), torch.cuda.Event()]
    ev_forkp = [torch.cuda.Event(), torch.cuda.Event()]
    ev_donep = [None, None]

    def pstep(i):
        k = i & 1
        if ev_donep[k] is not None:
            stream.wait_event(ev_donep[k])
        A.apax_profile_encode_async(xs[i % R], params, wsp[k], out=bufs[i % R], nbytes=nbp[k],
                                    encoded=ev_encp[k], stream=stream, side=side, forked=ev_forkp[k])
        side.wait_event(ev_encp[k])
        A.apax_decode(bufs[i % R], bound, hdr=step.hdr, y=ys[i % R], ws=ws_dec, stream=side,
                      clear_status=False)
        if ev_donep[k] is None:
            ev_donep[k] = torch.cuda.Event()
        ev_donep[k].record(side)

    A.apax_status_clear(ws2)
    for i in range(R):
        ys[i].zero_()
    for k in range(args.warmup):
        pstep(k)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for k in range(args.steps):
        pstep(k)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    p1 = time.perf_counter()
    assert A.apax_status(ws) == 0 and A.apax_status(ws2) == 0 and A.apax_status(ws_dec) == 0
    for w in wsp:
        pw = A.apax_profile_read(xs[0], params, w)
        assert pw["code"] == prof0["code"] and pw["stream_mask"] == prof0["stream_mask"]
        assert pw["metrics"]["r"] == prof0["metrics"]["r"]
    for k in range(min(R, max(args.warmup, args.steps))):  # every copy decoded as in the serial steps
        assert torch.equal(ys[k], y_serial), f"pipelined step of copy {k} differs from the serial steps"
    ms_step_pipelined = (p1 - p0) * 1e3 / args.steps
    # the same steps as hipGraphs (one per input copy, the two streams forked
    # and joined inside): the host enqueues one graph per step instead of
    # about twenty kernels, so the step time is the GPU's
    graph_ok, ms_step_graph = False, None
    try:
        y_eager = ys[0].clone()
        graphs = []
        for i in range(R):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                cap = torch.cuda.current_stream()
                A.apax_profile_encode_async(xs[i], params, ws, out=bufs[i], nbytes=nbt, stream=cap, side=side,
                                            forked=ev_fork)
                A.apax_decode(bufs[i], bound, hdr=step.hdr, y=ys[i], ws=ws_dec, stream=cap, clear_status=False)
                cap.wait_stream(side)
            graphs.append(g)
        for k in range(args.warmup):
            graphs[k % R].replay()
        torch.cuda.synchronize()
        for i in range(R):
            ys[i].zero_()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for k in range(args.steps):
            graphs[k % R].replay()
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        assert A.apax_status(ws) == 0 and A.apax_status(ws_dec) == 0
        # every replayed copy decoded to the eager result
        for i in range(min(R, args.steps)):
            assert torch.equal(ys[i], y_eager), f"graph replay of copy {i} differs from the eager step"
        ms_step_graph = (g1 - g0) * 1e3 / args.steps
        graph_ok = True
        del graphs
    except RuntimeError as exc:  # capture refused: report the eager steps
        log(f"step graph not used: {exc}")
    # the pipelined steps as hipGraphs: step i's graph (profile, encode,
    # decode of copy i with workspace pair i mod 2) replayed on stream i mod 2,
    # so step i + 1 runs beside step i and the host enqueues one graph per
    # step; step i + 2 follows step i on its stream, which orders the reuse
    # of the workspaces
    ms_step_graph_pipelined = None
    if graph_ok and R % 2 == 0:
        try:
            ws_decp = [ws_dec, A.workspace(torch.float32, x.shape, params, dev)]
            A.apax_status_clear(ws_decp[1])
            gstreams = [torch.cuda.Stream(), torch.cuda.Stream()]
            pgraphs = []
            for i in range(R):
                k = i & 1
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    cap = torch.cuda.current_stream()
                    A.apax_profile_encode_async(xs[i], params, wsp[k], out=bufs[i], nbytes=nbp[k], stream=cap,
                                                side=side, forked=ev_forkp[k])
                    A.apax_decode(bufs[i], bound, hdr=step.hdr, y=ys[i], ws=ws_decp[k], stream=cap,
                                  clear_status=False)
                    cap.wait_stream(side)
                pgraphs.append(g)
            torch.cuda.synchronize()

            def replay(k):
                with torch.cuda.stream(gstreams[k & 1]):
                    pgraphs[k % R].replay()

            for k in range(args.warmup):
                replay(k)
            torch.cuda.synchronize()
            for i in range(R):
                ys[i].zero_()
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            for k in range(args.steps):
                replay(k)
            torch.cuda.synchronize()
            q1 = time.perf_counter()
            assert all(A.apax_status(w) == 0 for w in wsp + ws_decp)
            for i in range(min(R, args.steps)):
                assert torch.equal(ys[i], y_serial), f"pipelined graph step of copy {i} differs from the serial steps"
            ms_step_graph_pipelined = (q1 - q0) * 1e3 / args.steps
            del pgraphs
        except RuntimeError as exc:
            log(f"pipelined step graphs not used: {exc}")
    ms_step_pipelined_eager = ms_step_pipelined
    if ms_step_graph_pipelined is not None and ms_step_graph_pipelined < ms_step_pipelined:
        ms_step_pipelined = ms_step_graph_pipelined
        pipelined_as_graph = True
    else:
        pipelined_as_graph = False
    # the step time: the faster of the two timed loops of the same steps (on
    # this runtime a graph replay does not always beat the eager enqueue of
    # the same kernels: its nodes can start later than the eager launches)
    ms_step_serial = ms_step_eager if ms_step_graph is None else min(ms_step_eager, ms_step_graph)
    ms_step = min(ms_step_serial, ms_step_pipelined)
    # in a step: the profile's span (enqueue start to its last pass, on the
    # side stream)
    prof_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps

    # per-launch kernel time: back-to-back launches over the rotating copies,
    # HIP events on the launch stream around the whole run
    reps = max(8, args.steps)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    for k in range(reps):
        A.apax_encode(xs[k % R], p_dev, out=bufs[k % R], nbytes=nbt, ws=ws, clear_status=False)
    e1.record(stream)
    for k in range(reps):
        A.apax_decode(bufs[k % R], bound, hdr=step.hdr, y=ys[k % R], ws=ws, clear_status=False)
    e2.record(stream)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    enc_ms = e0.elapsed_time(e1) / reps
    dec_ms = e1.elapsed_time(e2) / reps
    # kernel of each profile pass: HIP events around it on the launch stream
    # (apax_profile_timed), mean over `reps` profiles of the rotating copies
    pass_runs = {}
    for k in range(reps):
        _, pm = A.apax_profile_timed(xs[k % R], params, ws)
        for name, v in pm.items():
            pass_runs.setdefault(name, []).append(v)
    pass_ms = {name: sum(v) / len(v) for name, v in pass_runs.items()}
    # the step's fixed-rate metrics pass, which also writes the stream's
    # blocks: the profile-then-encode sequence on one stream with the same
    # events (apax_profile_encode_timed), the same bytes into the step's buffers
    menc_runs = []
    for k in range(reps):
        _, pm, _, _ = A.apax_profile_encode_timed(xs[k % R], params, ws, out=bufs[k % R], nbytes=nbt)
        menc_runs.append(pm["metrics"])
    menc_ms = sum(menc_runs) / len(menc_runs)
    assert int(nbt.item()) == bound

    # the 2-sigma S2R margin at the operating point (Sec. 4 Window 4; not part
    # of the step): the workspace holds the last timed profile of this field
    xl = xs[(reps - 1) % R]
    A.apax_s2r_margin(xl, params, ws)  # first call loads the kernels
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    s2r_ratio, s2r_db = A.apax_s2r_margin(xl, params, ws)
    s2r_ms = (time.perf_counter() - ts0) * 1e3

    # spectral metrics of the field and its decoded copy (Sec. 4 Windows 3-4;
    # not part of the step), warm call timed
    yl = ys[(reps - 1) % R]
    sws = torch.empty(A.lib.apax_spectral_workspace_bytes(), dtype=torch.uint8, device=dev)
    A.apax_spectral_metrics(xl, yl, ws=sws)
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    spec = A.apax_spectral_metrics(xl, yl, ws=sws)
    spec_ms = (time.perf_counter() - ts0) * 1e3

    # signal monitor of the field (Sec. 6; not part of the step), warm call timed
    A.apax_signal_monitor(xl, ws=sws)
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    mon = A.apax_signal_monitor(xl, ws=sws)
    mon_ms = (time.perf_counter() - ts0) * 1e3

    # decode-on-read (the "time to results" use, Sec. 1): a dot product with a
    # second field read from the 4:1 stream while decoding, against the same
    # consumer reading the uncompressed field; HIP events, back-to-back calls
    wf = torch.randn(xl.shape, dtype=torch.float32, device=dev)
    dout = torch.empty(1, dtype=torch.float64, device=dev)
    dws = torch.empty(A.DOT_WGS * 8, dtype=torch.uint8, device=dev)
    bl = bufs[(reps - 1) % R]
    A.apax_dot(xl, wf, out=dout, ws=dws)
    A.apax_decode_dot(bl, bound, step.hdr, wf, out=dout, ws=ws)
    f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    f0.record(stream)
    for _ in range(reps):
        A.apax_dot(xl, wf, out=dout, ws=dws)
    f1.record(stream)
    for _ in range(reps):
        A.apax_decode_dot(bl, bound, step.hdr, wf, out=dout, ws=ws)
    f2.record(stream)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    plain_dot_ms = f0.elapsed_time(f1) / reps
    fused_dot_ms = f1.elapsed_time(f2) / reps

    # the decoded field reproduces the profiler's correlation (checked outside timing)
    yd = ys[(args.steps - 1) % R].double()
    xd = xs[(args.steps - 1) % R].double()
    r_dec = float((xd * yd).sum() / torch.sqrt((xd * xd).sum() * (yd * yd).sum()))
    assert abs(r_dec - prof["metrics"]["r"]) < 1e-9, (r_dec, prof["metrics"]["r"])

    ratio = nbytes_in / bound
    enc_bytes = nbytes_in + bound          # read the field, write the stream
    dec_bytes = bound + nbytes_in          # read the stream, write the field
    enc_gbps = nbytes_in / (enc_ms * 1e-3) / 1e9
    dec_gbps = nbytes_in / (dec_ms * 1e-3) / 1e9
    # algorithmic bytes per launch: every kernel reads its samples once; the
    # subsample passes read every 16th block; the metrics pass writes, and the
    # centred pass reads, one 4-byte code per block
    nblocks = (4096 // 16) * (4096 // 16)
    sub_bytes = ((nblocks + 15) // 16) * 256 * 4
    probes = [v for name, v in pass_ms.items() if name.startswith("probe")]
    kernels = {  # name: (trace name, ms per launch, algorithmic bytes per launch)
        "k_encode": ("k_encode<float, 64, 2, 4, false>", enc_ms, enc_bytes),
        "k_decode": ("k_decode<float, 64, 2, 4>", dec_ms, dec_bytes),
        "k_profile_metrics": ("k_profile<float, 64, 2, 1>", pass_ms["metrics"], nbytes_in + 4 * nblocks),
        # read the field; write the stream's blocks and each block's code (4 B, for the centred pass)
        "k_profile_metrics_encode": ("k_profile<float, 64, 2, 5>", menc_ms, nbytes_in + (bound - 64) + 4 * nblocks),
        "k_profile_curve": ("k_profile<float, 64, 2, 4>", pass_ms["curve"], sub_bytes),
        "k_profile_centred": ("k_profile<float, 64, 2, 3>", pass_ms["centred"], nbytes_in + 4 * nblocks),
        "k_probe_all": ("k_probe_all<float, 64, 2>", sum(probes) / len(probes), sub_bytes),
        "k_pmax": ("k_pmax<float>", pass_ms["max"], nbytes_in),
    }
    dominant = max(kernels, key=lambda k: kernels[k][1])  # longest launch
    dom_name, dom_ms, dom_bytes = kernels[dominant]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = read_traffic(dominant)
    out = {
        "metric": METRIC,
        "value": round(nbytes_in / (ms_step * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_eager": round(ms_step_eager, 4),
        "ms_per_step_graph": None if ms_step_graph is None else round(ms_step_graph, 4),
        "ms_per_step_pipelined": round(ms_step_pipelined, 4),
        "ms_per_step_pipelined_eager": round(ms_step_pipelined_eager, 4),
        "ms_per_step_pipelined_graphs": None if ms_step_graph_pipelined is None else round(ms_step_graph_pipelined, 4),
        "pipelined_as_graphs": pipelined_as_graph,
        "ms_per_step_serial": round(ms_step_serial, 4),
        "step_pipelined": ms_step_pipelined <= ms_step_serial,
        "step_as_graph": graph_ok and ms_step_graph <= ms_step_eager,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C1: 2-D fp32 field 4096x4096 (GRF, k^-3, [-1e3,1e3] + noise 1e-2), "
                               "fixed rate 4:1, 16x16 bricks, profile + encode + decode per step",
                   "input_bytes": nbytes_in, "stream_bytes": bound, "copies_rotated": R,
                   "attenuation_arith": "f64", "stats_arith": "f64",
                   "streams": "profile and encode on one stream (the fixed-rate metrics pass writes the "
                              "stream's blocks itself), the curve pass beside the metrics pass and the "
                              "metrics reduction and centred pass beside the decode on a second"},
        "encode_GBps": round(enc_gbps, 2),
        "decode_GBps": round(dec_gbps, 2),
        "encode_pct_hbm": round(100 * enc_gbps / HBM_PEAK_GBPS, 2),
        "decode_pct_hbm": round(100 * dec_gbps / HBM_PEAK_GBPS, 2),
        "encode_ms": round(enc_ms, 4),
        "decode_ms": round(dec_ms, 4),
        "kernel_timing": f"mean of {reps} back-to-back launches between HIP events on the launch stream",
        "profile_ms": round(prof_ms, 4),
        "ratio": round(ratio, 4),
        "r": prof["metrics"]["r"],
        "code": prof["code"],
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_bytes},
        "kernels_us": {n: {"kernel": t, "us": round(1e3 * ms, 2),
                           "GBps": round(b / (ms * 1e-3) / 1e9, 1)}
                       for n, (t, ms, b) in kernels.items()},
        "profile_pass_us": {n: round(1e3 * v, 2) for n, v in pass_ms.items()},
        "s2r_margin": {"db": round(s2r_db, 4), "ratio": s2r_ratio, "ms_per_call": round(s2r_ms, 3),
                       "note": "2-sigma S2R margin at the operating point, five selection passes; "
                               "outside the step"},
        "decode_on_read": {"consumer": "dot product with a second 4096x4096 fp32 field",
                           "plain_us": round(1e3 * plain_dot_ms, 2), "fused_us": round(1e3 * fused_dot_ms, 2),
                           "time_to_results_speedup": round(plain_dot_ms / fused_dot_ms, 3),
                           "plain_GBps": round(2 * nbytes_in / (plain_dot_ms * 1e-3) / 1e9, 1),
                           "fused_GBps": round((bound + nbytes_in) / (fused_dot_ms * 1e-3) / 1e9, 1)},
        "spectral": {"dr_db": round(spec["dr"], 3), "srr_db": round(spec["srr"], 3),
                     "fft_s2r_margin_db": round(spec["fft_s2r_margin"], 3),
                     "segments": spec["segments"], "ms_per_call": round(spec_ms, 3),
                     "note": "Welch spectra of x, y, x - y (1024-sample Hann segments, hop 512); "
                             "outside the step"},
        "signal_monitor": {"peak_bin": mon["peak_bin"], "snr_db": round(mon["snr_db"], 3),
                           "stride": mon["stride"], "sign": mon["sign"], "gain_db": round(mon["gain_db"], 3),
                           "acf1": round(mon["acf"][1], 6), "ms_per_call": round(mon_ms, 3),
                           "note": "Welch spectrum of x and its lags 0..16 autocorrelation; outside the step"},
    }
    if args.copy_probe:
        # counter calibration: a plain copy of the field (reads and writes
        # input_bytes), a read-only sum over it and a write-only fill of a field
        for _ in range(3):
            ys[0].copy_(xs[1])
            float(xs[1].sum())
            ys[0].fill_(0.5)
        torch.cuda.synchronize()

    # the other workloads of the metric, each timed alone (not part of the step):
    # the lossless int16 time series, the fp64 3-d field at fixed quality, and
    # the C1 field at 3:1 and 10:1
    if not args.no_workloads:
        del xs, bufs, ys
        torch.cuda.empty_cache()
        wl = []
        x0 = synth.sinusoids(1 << 20)
        wl.append(codec_workload(A, dev, "C0: int16 time series 2^20 samples (2 MiB), lossless, 256-sample "
                                 "blocks; launch-latency bound at this size", x0,
                                 {"mode": "lossless", "brick": (256,)}, copies=256, reps=256, profile=False))
        x0l = synth.sinusoids(1 << 25)
        wl.append(codec_workload(A, dev, "C0 recipe at 2^25 samples (64 MiB): int16 time series, lossless, "
                                 "256-sample blocks", x0l, {"mode": "lossless", "brick": (256,)},
                                 copies=8, reps=max(8, args.steps), profile=False))
        for rate in (3.0, 10.0):
            wl.append(codec_workload(A, dev, f"C1 field at {rate:g}:1", x, dict(params, rate=rate),
                                     copies=8, reps=max(8, args.steps)))
        x2 = synth.blobs3d()
        wl.append(codec_workload(A, dev, "C2: fp64 field 256x512x512, fixed quality r >= 0.99996, 4x4x8 bricks",
                                 x2, {"mode": "fixed_quality", "brick": (4, 4, 8), "target_corr": 0.99996},
                                 copies=2, reps=8))
        out["workloads"] = wl
    out["paper_throughput"] = PAPER_THROUGHPUT
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, params)
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def item_params(spec, code):
    if spec["mode"] == "lossless":
        return {"mode": "lossless", "brick": (256,)}
    return {"mode": "fixed_rate", "brick": (256,), "rate": spec["rate"], "code": code}


def profiled_items(specs, pools, dev, A):
    """Cut each item from the device pools; fixed-rate items get the
    profiler's operating point and stream mask (untimed set-up)."""
    import torch
    out = []
    for k, spec in enumerate(specs):
        x = pools.item_device(spec, dev)
        p = item_params(spec, 0)
        if p["mode"] == "fixed_rate":
            prof = A.apax_profile(x, p)
            p = dict(p, code=prof["code"], stream_mask=prof["stream_mask"] & 0x7F)
        out.append((x, p))
        if k % 512 == 511:
            log(f"set-up {k + 1}/{len(specs)} items")
    torch.cuda.synchronize()
    return out


def bench_batch(args):
    """Many arrays (log-uniform 4 KB..64 MB, int16/int32/fp32/fp64, lossless
    or fixed rate 3:1..10:1, 1-D, 256-sample blocks) encoded and decoded by
    one persistent launch per block-shape class replayed from a hipGraph,
    against the same arrays encoded one apax_encode call at a time."""
    import torch

    import synth
    from paper_1303_4994_amd import apax as A
    from paper_1303_4994_amd import tune as T

    dev = torch.device("cuda:0")
    log(f"pools of {args.pool} samples")
    pools = synth.Pools(n=args.pool)
    specs = [synth.item_spec(i) for i in range(args.items)]
    arrays = profiled_items(specs, pools, dev, A)
    nbytes_in = sum(x.numel() * x.element_size() for x, _ in arrays)
    log(f"{len(arrays)} items, {nbytes_in / 1e9:.2f} GB; tuning")
    tune = T.tune(A.OP_ENCODE, arrays[:256], reps=2, verbose=True)
    b = A.Batch.encode(arrays, tune=tune)
    b.capture()
    for _ in range(args.warmup):
        b.launch()
    torch.cuda.synchronize()
    assert b.status() == 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.launch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    log(f"batched encode {t_batch * 1e3:.2f} ms")
    # plain: one apax_encode call per array, same outputs, one stream
    # one workspace, sized for the largest call, shared by the sequential calls
    ws = torch.empty(max(A.apax_workspace_size(x.dtype, tuple(x.shape), p) for x, p in arrays),
                     dtype=torch.uint8, device=dev)

    def plain():
        for i, (x, p) in enumerate(arrays):
            A.apax_encode(x, p, out=b.outs[i], nbytes=b.nbytes[i:i + 1], clear_status=False, ws=ws)
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / max(1, args.steps // 2)
    log(f"plain encode {t_plain * 1e3:.2f} ms")
    # batched decode of the batch's streams
    nb = b.nbytes.cpu().numpy()
    hdrs = [bytes(o[:64].cpu().numpy().tobytes()) for o in b.outs]
    d = A.Batch.decode([(b.outs[i], int(nb[i]), hdrs[i]) for i in range(len(arrays))], tune=tune)
    d.capture()
    d.launch()
    torch.cuda.synchronize()
    assert d.status() == 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d.launch()
    torch.cuda.synchronize()
    t_dec = (time.perf_counter() - t0) / args.steps
    ok = all(torch.equal(d.outs[i], arrays[i][0]) for i in range(len(arrays))
             if arrays[i][1]["mode"] == "lossless")
    stream_bytes = int(nb.sum())
    out = {
        "metric": "batched encode/decode GB/s (uncompressed bytes), 1 GPU",
        "value": round(nbytes_in / t_batch / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "mixed",
        "data": "synthetic",
        "config": {"workload": f"C3: {len(arrays)} arrays, log-uniform 4 KB..64 MB, int16/int32/fp32/fp64, "
                               "lossless or fixed rate 3:1..10:1 (profiler operating point), "
                               "1-D 256-sample blocks, one hipGraph replay per step",
                   "input_bytes": nbytes_in, "stream_bytes": stream_bytes, "pool_samples": args.pool,
                   "tune": tune},
        "encode_GBps_batched": round(nbytes_in / t_batch / 1e9, 2),
        "encode_GBps_plain": round(nbytes_in / t_plain / 1e9, 2),
        "batched_over_plain": round(t_plain / t_batch, 3),
        "decode_GBps_batched": round(nbytes_in / t_dec / 1e9, 2),
        "encode_pct_hbm": round(100 * nbytes_in / t_batch / 1e9 / HBM_PEAK_GBPS, 2),
        "lossless_roundtrip_exact": bool(ok),
        # one graph replay launches one persistent kernel per block-shape class
        # (1-D 256-sample blocks: k_encode_batch<64, 1, WP>); it reads every
        # array and writes every stream once
        "roofline": {"bound": "hbm", "kernel": "k_encode_batch (one hipGraph replay)",
                     "achieved": round((nbytes_in + stream_bytes) / t_batch / 1e9, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round((nbytes_in + stream_bytes) / t_batch / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "algorithmic_bytes_per_launch": nbytes_in + stream_bytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_items(arrays, "encode")
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson stream of encode/decode requests (payload log-uniform
    64 KB..256 MB, the batch generators and dtypes, 1:1 encode:decode) served
    by continuous batching under a 64 GB HBM budget.  The requests cycle over
    a set of device-resident items (each with its own output buffers, more
    items than requests can be in flight); the arrival rate is rho times the
    plain single-call throughput measured first on the same items."""
    import numpy as np
    import torch

    import synth
    from paper_1303_4994_amd import apax as A
    from paper_1303_4994_amd import serve as S

    dev = torch.device("cuda:0")
    log(f"pools of {args.pool} samples")
    pools = synth.Pools(n=args.pool)
    n_items = max(1, min(args.serve_items, args.requests))
    specs = synth.requests(n_items)
    arrays = profiled_items(specs, pools, dev, A)
    # decode requests read streams encoded in set-up
    items = []
    for spec, (x, p) in zip(specs, arrays):
        r = {"kind": spec["kind"], "x": x, "params": p, "bytes": x.numel() * x.element_size()}
        if r["kind"] == "decode":
            buf, nb = A.apax_encode(x, p)
            r["stream"], r["nbytes"] = buf, int(nb.item())
            r["hdr"] = bytes(buf[:64].cpu().numpy().tobytes())
            r["out"] = torch.empty_like(x)
        else:
            bound = A.apax_encode_bound(x.dtype, tuple(x.shape), p)
            r["out"] = (torch.empty(max(bound, 64), dtype=torch.uint8, device=dev),
                        torch.empty(1, dtype=torch.int64, device=dev))
        items.append(r)
    torch.cuda.synchronize()
    item_bytes = sum(r["bytes"] for r in items)
    log(f"{n_items} resident items, {item_bytes / 1e9:.2f} GB")
    ws = torch.empty(max(A.apax_workspace_size(r["x"].dtype, tuple(r["x"].shape), r["params"])
                         for r in items), dtype=torch.uint8, device=dev)

    def plain():
        for r in items:
            if r["kind"] == "encode":
                A.apax_encode(r["x"], r["params"], out=r["out"][0], nbytes=r["out"][1], ws=ws,
                              clear_status=False)
            else:
                A.apax_decode(r["stream"], r["nbytes"], hdr=r["hdr"], y=r["out"], ws=ws, clear_status=False)
    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    assert A.apax_status(ws) == 0
    T_plain = item_bytes / t_plain
    # reference copies of the plain results of every 16th item: the served
    # results must be byte-identical
    def result(r):
        if r["kind"] == "encode":
            return r["out"][0][: int(r["out"][1].item())].clone()
        return r["out"].clone()
    ref = {i: result(items[i]) for i in range(0, n_items, 16)}
    n = args.requests
    which = [k % n_items for k in range(n)]
    mean = sum(items[i]["bytes"] for i in which) / n
    lam = args.rho * T_plain / mean
    rng = np.random.default_rng(synth.seed_of(4, 7))
    arrivals = list(np.cumsum(rng.exponential(1.0 / lam, size=n)))
    log(f"plain {T_plain / 1e9:.1f} GB/s; {n} requests over {n_items} items, "
        f"arrival rate {lam:.1f}/s over {arrivals[-1]:.1f} s")
    srv = S.Server(budget_bytes=64 << 30, slots=4, max_group=64, ws_bytes=64 << 20)
    done = [0]

    def job(k):
        r = items[which[k]]
        if r["kind"] == "encode":
            return srv.submit_encode(r["x"], r["params"], r["out"][0], r["out"][1], tag=k), r["bytes"]
        return srv.submit_decode(r["stream"], r["nbytes"], r["hdr"], r["out"], tag=k), r["bytes"]

    step = max(100, n // 20)

    def on_done(k, c):
        done[0] += 1
        if done[0] % step == 0:
            log(f"served {done[0]}/{n}")
    st = S.drive(srv, [lambda k=k: job(k) for k in range(n)], arrivals, on_done=on_done,
                 deadline_s=arrivals[-1] + 300.0)
    srv.close()
    torch.cuda.synchronize()
    for i, v in ref.items():
        got = result(items[i])
        assert got.shape == v.shape and torch.equal(got, v), f"served item {i} differs from its plain call"
    # the served results of a bounded sample of those items (about 256 MB)
    # also equal the CPU oracle's stream or decoded array, byte for byte
    from oracle import oracle as O
    orc_bytes, orc_items = 0, 0
    for i in ref:
        r = items[i]
        if orc_bytes >= (256 << 20):
            break
        got = result(r).cpu().numpy()
        if r["kind"] == "encode":
            assert np.array_equal(got, O.encode(r["x"].cpu().numpy(), r["params"])), f"served item {i} != oracle"
        else:
            exp = O.decode(r["stream"][: r["nbytes"]].cpu().numpy())
            assert np.array_equal(got.view(np.uint8), exp.view(np.uint8)), f"served item {i} != oracle"
        orc_bytes += r["bytes"]
        orc_items += 1
    total = st["bytes"]
    out = {
        "metric": "served encode/decode GB/s (uncompressed bytes) with p50/p99 latency, 1 GPU",
        "value": round(st["GBps"], 2), "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(st["seconds"] * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "mixed", "data": "synthetic",
        "config": {"workload": f"C4: {n} requests, Poisson arrivals at rho={args.rho} of plain "
                               "throughput, payload log-uniform 64 KB..256 MB, encode:decode 1:1, "
                               f"cycling over {n_items} device-resident items, 64 GB HBM admission "
                               "budget, 4 slots x 64 requests",
                   "requests": n, "bytes": total, "items": n_items, "item_bytes": item_bytes,
                   "pool_samples": args.pool},
        "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
        "max_ms": round(st["max_ms"], 3), "groups": st["groups"],
        "plain_GBps": round(T_plain / 1e9, 2),
        "offered_GBps": round(args.rho * T_plain / 1e9, 2),
        "checked_items": len(ref),
        "oracle_checked_items": orc_items, "oracle_checked_bytes": orc_bytes,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_items([(r["x"], r["params"]) for r in items], "both")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
