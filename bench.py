#!/usr/bin/env python3
"""Throughput of the CKKS hot path on one MI355X.

Workload (the large-ring configuration the headline metric is quoted on):
N = 2^16, L = 24 ciphertext primes (60-bit q_0, then 50-bit), K = 6 special
60-bit primes, dnum = 4, scale 2^50; a batch of 16 ciphertexts with
unit-modulus complex slots.  One step = for every ciphertext of the batch a
depth-8 chain c <- RESCALE(HMult+relin(c, c)) (levels 24 -> 16) followed by
rotate-and-sum over all 2^15 slots (15 rotations + 15 additions).  That is
128 HMult+relin, 128 RESCALE and 240 ROTATE per step; inputs are resident in
HBM before the timed region starts.

`value` is whole-job HMult+relin/s: 128 * steps / timed seconds (the time
includes the rescales and rotations of the job).  Rates of the individual
operations, timed separately on the same data, are reported under
"breakdown"; the dominant kernel family's per-launch time is measured with
HIP events on the stream the kernels run on and reported under "roofline".

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published
ALU_PEAK_GOPS = 256 * 64 * 2.4  # int32 VALU lane-ops/s in G: 256 CUs x 64 lanes x 2.4 GHz
FAMILIES = ["ntt_fwd_pass", "ntt_inv_pass", "modup_bconv", "key_inner_product", "moddown_bconv",
            "moddown_final", "tensor", "automorphism", "rescale", "elementwise"]
KERNEL_NAMES = {2: "k_modup_mfma_b", 3: "k_key_inner_items", 4: "k_moddown_mfma_b", 5: "(fused into the forward NTT)",
                6: "k_tensor_b",
                7: "k_automorphism_b", 8: "k_rescale_expand_b"}


def kernel_name(kid, variant):
    """Demangled kernel name of one instantiation (see pft_prof_read_variants)."""
    if kid in (0, 1) and variant:
        v = variant - 1
        b = lambda x: "true" if x else "false"  # noqa: E731
        name = "k_ntt_pass<%d, %d, %s, %s, %s, %s, %s" % (v & 31, 3 if v & 256 else 4, b(kid == 1), b(v & 32),
                                                          b(v & 64), b(v & 128), b(v & 512))
        return name + (", true>" if v & 1024 else ">")  # X -> X^kappa folded into the pass
    if kid == 3 and variant >= 1024:  # inner product fused with the row pass of ModUp's rows
        v = variant - 1024
        return "k_row_inner<%d, 3, %s, %d>" % (v & 63, "true" if v & 64 else "false", 2 if v & 128 else 1)
    if kid == 8 and variant == 1:  # RESCALE's expansion fused with the first transform pass
        return "k_rescale_col_b"
    if kid in (2, 4) and variant >= 64:  # base conversion fused with the first (and last inverse) pass
        return "k_bconv_col_b<%du, %s, %s>" % ((variant - 64) & 15, "true" if kid == 4 else "false",
                                               "true" if (variant - 64) & 16 else "false")
    if kid in (2, 3, 4) and variant:  # templated on the k-block count / the number of digits
        return "%s<%du>" % (KERNEL_NAMES[kid], variant)
    return KERNEL_NAMES.get(kid, FAMILIES[kid])
CHAIN_DEPTH = 8
ROT_SLOTS = 1 << 15


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


class Roctx:
    """roctxProfilerResume/Pause around the timed region, for a profiler
    that limits itself to such regions (rocprofv3's --selected-regions; the
    stored profiles do not rely on it: they trace whole runs of
    --profile-steps / --profile-workload).  Without a profiler these calls
    do nothing."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("/opt/rocm/lib/librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so.1",
                     "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        log("roctx: %s" % ("loaded" if self.lib is not None else "not found (profiler regions unavailable)"))
        if self.lib is not None:
            for fn in ("roctxProfilerResume", "roctxProfilerPause"):
                getattr(self.lib, fn).argtypes = [ctypes.c_uint64]
                getattr(self.lib, fn).restype = ctypes.c_int

    def resume(self):
        if self.lib is not None:
            rc = self.lib.roctxProfilerResume(0)
            if rc:
                log("roctxProfilerResume returned %d" % rc)

    def pause(self):
        if self.lib is not None:
            rc = self.lib.roctxProfilerPause(0)
            if rc:
                log("roctxProfilerPause returned %d" % rc)


# source files whose text determines the kernels (for the validity of stored
# counter figures: any change to device code invalidates them all)
KERNEL_SOURCES = ["ntt.hip", "ckks.hip", "sampler.hip", "pft_device.h", "bconv_device.h", "pft_kernels.h"]
PROFILE_DIR = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1908_06972_amd", "csrc")


def source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_profile(kernel):
    """Counter figures of `kernel` recorded under profiles/ (a `pft-profile:`
    JSON line), if they were taken on the current kernel source."""
    if not os.path.isdir(PROFILE_DIR):
        return None
    sha = source_sha()
    for f in sorted(os.listdir(PROFILE_DIR)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILE_DIR, f)):
            if line.startswith("pft-profile: "):
                rec = json.loads(line[len("pft-profile: "):])
                if rec.get("kernel") == kernel and rec.get("source_sha256") == sha:
                    return rec
    return None


def _csv_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, dirpath))


def _step_dispatches(rows, key_id, key_start):
    """Dispatches of the job steps after the first one: from the first HMUL
    tensor kernel of the second step on (a step launches CHAIN_DEPTH tensor
    kernels).  This excludes key generation, encryption and the first step,
    during which the NTT autotuner times its candidates; every later step
    launches the same kernels with the same shapes."""
    rows = sorted(rows, key=lambda r: int(r[key_id]))
    tensors = sorted({int(r[key_id]) for r in rows if "k_tensor_b" in r["Kernel_Name"]})
    if len(tensors) <= CHAIN_DEPTH:
        return []
    first = tensors[CHAIN_DEPTH]
    return [r for r in rows if int(r[key_id]) >= first]


def summarize(trace_dir, fetch_dir, write_dir, kernel, kid, commands, n_top=6, sq_dir=None, mix_dir=None):
    """Markdown summary of three rocprofv3 runs of bench.py: a kernel trace
    (durations) and two counter runs (FETCH_SIZE with SQ_INSTS_VALU, then
    WRITE_SIZE), each restricted to the dispatches of the job steps, with
    counter figures for the n_top longest kernels (or `kernel`).  The copy
    kernel k_copy_rows_b (8 bytes read and 8 written per work-item)
    calibrates the byte counters.  sq_dir: an optional fourth run with the
    SQ counters SQ_WAVE_CYCLES, SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_VALU,
    SQ_INSTS_LDS and SQ_LDS_BANK_CONFLICT, summarised per kernel; mix_dir:
    an optional fifth run with the instruction mix (SQ_INSTS_VALU_INT32,
    SQ_INSTS_VALU_INT64, SQ_INSTS_VALU_FMA_F64, SQ_INSTS_MFMA) and the
    matrix-core busy cycles (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE
    times the 1024 SIMDs)."""
    trace = _step_dispatches(_csv_rows(_find(trace_dir, "kernel_trace.csv")), "Dispatch_Id", "Start_Timestamp")
    short_name = lambda n: n.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")  # noqa: E731
    per = {}
    for r in trace:
        name = short_name(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        c, t = per.get(name, (0, 0.0))
        per[name] = (c + 1, t + d)
    total = sum(t for _, t in per.values())
    ranked = sorted(per.items(), key=lambda kv: -kv[1][1])
    targets = [k for k, _ in ranked[:n_top]] if kernel == "auto" else [kernel]
    out = ["# Kernels of the large-ring job step (N=2^16, L=24, batch 16): %s" % ", ".join(targets), ""]
    out.append("Commands (from the repository root on the measuring MI355X host, after `export TMPDIR=/tmp`):")
    out.append("")
    for c in commands:
        out.append("    " + c)
    out.append("")
    out.append("Kernel durations over the dispatches of the job steps after the first (the first settles the NTT "
               "autotuner; every later step launches the same kernels with the same shapes):")
    out.append("")
    out.append("| kernel | calls | total ms | avg us | share |")
    out.append("|---|---|---|---|---|")
    for name, (c, t) in ranked[:14]:
        out.append("| %s | %d | %.2f | %.1f | %.1f%% |" % (name, c, t / 1e3, t / c, 100 * t / total))

    def per_dispatch(dirpath, counter, target):
        rows = _step_dispatches(_csv_rows(_find(dirpath, "counter_collection.csv")), "Dispatch_Id", "Start_Timestamp")
        vals, cal = [], []
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            v = float(r["Counter_Value"])
            name = short_name(r["Kernel_Name"])
            if name == target:
                vals.append(v)
            elif name == "k_copy_rows_b":
                cal.append((v, 8.0 * float(r["Grid_Size"])))
        return vals, cal

    out.append("")
    out.append("Counters over the same dispatches, per launch (calibration factors: known bytes of k_copy_rows_b, a "
               "plain copy of 8 bytes read and 8 written per work-item, divided by 1024 x its counted KiB; traffic = "
               "1024 x (fetch x fetch factor + write x write factor); on the measured MI355X FETCH_SIZE counts half the bytes "
               "the copy reads, factor 2.0, and WRITE_SIZE is exact, factor 1.0):")
    out.append("")
    out.append("| kernel | avg us | fetch KiB | write KiB | traffic MB | VALU insts |")
    out.append("|---|---|---|---|---|---|")
    recs = []
    for target in targets:
        fetch, fcal = per_dispatch(fetch_dir, "FETCH_SIZE", target)
        valu, _ = per_dispatch(fetch_dir, "SQ_INSTS_VALU", target)
        write, wcal = per_dispatch(write_dir, "WRITE_SIZE", target)
        f_factor = sum(b for _, b in fcal) / (1024.0 * sum(v for v, _ in fcal)) if fcal else None
        w_factor = sum(b for _, b in wcal) / (1024.0 * sum(v for v, _ in wcal)) if wcal else None
        c, t = per.get(target, (0, 0.0))
        rec = {
            "kernel": target,
            "source_sha256": source_sha(),
            "avg_launch_us": t / c if c else None,
            "fetch_kib_per_launch": sum(fetch) / len(fetch) if fetch else None,
            "write_kib_per_launch": sum(write) / len(write) if write else None,
            "fetch_calibration": f_factor,
            "write_calibration": w_factor,
            "valu_insts_per_launch": sum(valu) / len(valu) if valu else None,
        }
        if None not in (rec["fetch_kib_per_launch"], rec["write_kib_per_launch"], f_factor, w_factor):
            rec["traffic_bytes_per_launch"] = 1024.0 * (rec["fetch_kib_per_launch"] * f_factor +
                                                        rec["write_kib_per_launch"] * w_factor)
        fmt = lambda v, f: (f % v) if v is not None else "-"  # noqa: E731
        out.append("| %s | %s | %s | %s | %s | %s |" % (
            target, fmt(rec["avg_launch_us"], "%.1f"), fmt(rec["fetch_kib_per_launch"], "%.0f"),
            fmt(rec["write_kib_per_launch"], "%.0f"),
            fmt(rec.get("traffic_bytes_per_launch") and rec["traffic_bytes_per_launch"] / 1e6, "%.1f"),
            fmt(rec["valu_insts_per_launch"], "%.4g")))
        recs.append(rec)
    out.append("")
    if sq_dir:
        out.append("Issue counters over the same dispatches, per launch (wave cycles summed over waves; `wait` = "
                   "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES, the share of a wave's life spent waiting on a counter; `valu` "
                   "= SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES per wave, times the waves resident per SIMD for the "
                   "SIMD's VALU share; `conflict/LDS` = SQ_LDS_BANK_CONFLICT cycles per LDS instruction):")
        out.append("")
        out.append("| kernel | LDS insts | bank-conflict cycles | conflict/LDS | wait | valu |")
        out.append("|---|---|---|---|---|---|")
        for target in targets:
            vals = {}
            for ctr in ("SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS",
                        "SQ_LDS_BANK_CONFLICT"):
                v, _ = per_dispatch(sq_dir, ctr, target)
                vals[ctr] = sum(v) / len(v) if v else None
            wc, lds, bc = vals["SQ_WAVE_CYCLES"], vals["SQ_INSTS_LDS"], vals["SQ_LDS_BANK_CONFLICT"]
            fmt = lambda v, f: (f % v) if v is not None else "-"  # noqa: E731
            out.append("| %s | %s | %s | %s | %s | %s |" % (
                target, fmt(lds, "%.3g"), fmt(bc, "%.3g"), fmt(bc / lds if lds and bc is not None else None, "%.2f"),
                fmt(vals["SQ_WAIT_INST_ANY"] / wc if wc and vals["SQ_WAIT_INST_ANY"] is not None else None, "%.2f"),
                fmt(vals["SQ_ACTIVE_INST_VALU"] / wc if wc and vals["SQ_ACTIVE_INST_VALU"] is not None else None,
                    "%.2f")))
        out.append("")
    if mix_dir:
        out.append("Instruction mix and matrix cores over the same dispatches, per launch (wave instructions; "
                   "`MFMA busy` = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x 1024 SIMDs)):")
        out.append("")
        out.append("| kernel | VALU int32 | VALU int64 | VALU fp64 FMA | MFMA insts | MFMA busy |")
        out.append("|---|---|---|---|---|---|")
        for target in targets:
            vals = {}
            for ctr in ("SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_MFMA",
                        "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE"):
                v, _ = per_dispatch(mix_dir, ctr, target)
                vals[ctr] = sum(v) / len(v) if v else None
            fmt = lambda v, f: (f % v) if v is not None else "-"  # noqa: E731
            busy = vals["SQ_VALU_MFMA_BUSY_CYCLES"]
            act = vals["GRBM_GUI_ACTIVE"]
            out.append("| %s | %s | %s | %s | %s | %s |" % (
                target, fmt(vals["SQ_INSTS_VALU_INT32"], "%.3g"), fmt(vals["SQ_INSTS_VALU_INT64"], "%.3g"),
                fmt(vals["SQ_INSTS_VALU_FMA_F64"], "%.3g"), fmt(vals["SQ_INSTS_MFMA"], "%.3g"),
                fmt(busy / (act * 1024.0) if busy is not None and act else None, "%.3f")))
        out.append("")
    # every kernel of the profiled steps: counted traffic per step
    def step_total(dirpath, counter):
        rows = _step_dispatches(_csv_rows(_find(dirpath, "counter_collection.csv")), "Dispatch_Id", "Start_Timestamp")
        tensors = {int(r["Dispatch_Id"]) for r in rows if "k_tensor_b" in r["Kernel_Name"]}
        steps = len(tensors) / float(CHAIN_DEPTH)
        tot = sum(float(r["Counter_Value"]) for r in rows if r.get("Counter_Name") == counter)
        return tot, steps
    f_tot, f_steps = step_total(fetch_dir, "FETCH_SIZE")
    w_tot, w_steps = step_total(write_dir, "WRITE_SIZE")
    f_factor = recs[0]["fetch_calibration"] if recs else None
    w_factor = recs[0]["write_calibration"] if recs else None
    if f_steps and w_steps and f_factor and w_factor:
        step_rec = {"source_sha256": source_sha(), "steps_profiled": f_steps,
                    "fetch_bytes_per_step": 1024.0 * f_tot * f_factor / f_steps,
                    "write_bytes_per_step": 1024.0 * w_tot * w_factor / w_steps}
        step_rec["traffic_bytes_per_step"] = step_rec["fetch_bytes_per_step"] + step_rec["write_bytes_per_step"]
        out.append("Every kernel of the profiled steps together (calibrated as above): %.2f GB fetched and %.2f GB "
                   "written per step, %.2f GB in all." % (step_rec["fetch_bytes_per_step"] / 1e9,
                                                          step_rec["write_bytes_per_step"] / 1e9,
                                                          step_rec["traffic_bytes_per_step"] / 1e9))
        out.append("")
        recs.append(None)
    for rec in recs:
        if rec is None:
            out.append("pft-step: " + json.dumps(step_rec))
        else:
            out.append("pft-profile: " + json.dumps(rec))
    return "\n".join(out) + "\n"


def stored_step():
    """Counted traffic per job step recorded under profiles/ (a `pft-step:`
    line), if taken on the current kernel source."""
    if not os.path.isdir(PROFILE_DIR):
        return None
    sha = source_sha()
    for f in sorted(os.listdir(PROFILE_DIR)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILE_DIR, f)):
            if line.startswith("pft-step: "):
                rec = json.loads(line[len("pft-step: "):])
                if rec.get("source_sha256") == sha:
                    return rec
    return None


def ct_bytes(level, n):
    """One ciphertext at `level`: 2 polynomials x level limbs x N residues x 8 bytes."""
    return 2 * level * n * 8


def key_bytes(lp, level):
    """The part of one switching key a key switch at `level` reads: beta
    digits x (b, a) x (level + K) rows."""
    beta = -(-level // lp.alpha)
    return 2 * beta * (level + lp.K) * lp.n * 8


def op_alg_bytes(lp, batch):
    """Algorithmic HBM bytes of one operation at the top level L: its
    operands read and its result written once, 8 bytes per residue; the
    switching key once per batch (every ciphertext of a batch uses it).
    HMult+relin reads two operand ciphertexts."""
    L, n = lp.L, lp.n
    return {"hmult_relin": 3 * ct_bytes(L, n) + key_bytes(lp, L) / batch,
            "rotate": 2 * ct_bytes(L, n) + key_bytes(lp, L) / batch,
            "rescale": ct_bytes(L, n) + ct_bytes(L - 1, n),
            "poly_ntt": ct_bytes(L, n)}  # one L-limb polynomial read and written: 2 L N 8 bytes


def step_alg_bytes(lp, batch):
    """Algorithmic HBM bytes of one job step over the batch: for each of the
    CHAIN_DEPTH links (levels L .. L - CHAIN_DEPTH + 1) an HMult+relin (two
    operands read, the product written, the key once) and a RESCALE (read,
    write), then the rotate-and-sum: per rotation the running sum read and
    written once (the addition folds into the rotation's last kernel) and
    the rotation key once."""
    n, tot = lp.n, 0
    for lvl in range(lp.L, lp.L - CHAIN_DEPTH, -1):
        tot += 3 * ct_bytes(lvl, n) * batch + key_bytes(lp, lvl)
        tot += (ct_bytes(lvl, n) + ct_bytes(lvl - 1, n)) * batch
    lvl = lp.L - CHAIN_DEPTH
    rotations = ROT_SLOTS.bit_length() - 1
    tot += rotations * (2 * ct_bytes(lvl, n) * batch + key_bytes(lp, lvl))
    return tot


def copy_bandwidth(gib=2, reps=5):
    """Device-to-device copy rate (read + write bytes per second) of a
    torch tensor copy of `gib` GiB: the practical HBM ceiling beside the
    published peak."""
    import torch
    n = (gib << 30) // 8
    a = torch.zeros(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="print the oracle's full CPU table (JSON) on this host and exit (no GPU needed)")
    ap.add_argument("--reps", type=int, default=10, help="runs per median of the CPU baseline")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many untimed steps (for rocprofv3) and exit")
    ap.add_argument("--profile-workload", choices=["bow", "predict", "batched"],
                    help="run only the bag-of-words inference, the encrypted-weight predict step or the "
                         "batched-primitives op list, then one more batch / eager executor run set apart by idle "
                         "time (1 s before, 3 s after; for a rocprofv3 kernel trace), and exit")
    ap.add_argument("--no-breakdown", action="store_true", help="skip the per-operation loops")
    ap.add_argument("--no-predict", action="store_true", help="skip the encrypted-weight predict measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-primitives op-list measurement")
    ap.add_argument("--no-bow", action="store_true", help="skip the bag-of-words inference measurement")
    ap.add_argument("--no-paper-inference", action="store_true",
                    help="skip the inference at the paper's shapes (N=8192, 123 inputs)")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving measurement (0 skips it)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the markdown summary of three rocprofv3 runs of the timed region and exit")
    ap.add_argument("--kernel", default="auto",
                    help="kernel the --summarize counters are collected for; auto = the longest in the trace")
    ap.add_argument("--family", type=int, default=0)
    ap.add_argument("--commands", nargs="*", default=[])
    ap.add_argument("--sq", default=None, help="with --summarize: directory of the SQ counter run")
    ap.add_argument("--mix", default=None, help="with --summarize: directory of the instruction-mix counter run")
    ap.add_argument("--tuning-in", default=DEFAULT_TUNING,
                    help="JSON table of NTT schedules (from --tuning-out) to use instead of tuning; the default is the "
                         "table the autotuner produced for this workload, so kernel choices repeat run to run")
    ap.add_argument("--retune", action="store_true", help="ignore --tuning-in and let the autotuner choose")
    ap.add_argument("--tuning-out", help="write the NTT schedules the run used (JSON)")
    return ap.parse_args()


def prof_variants(ctx, kid):
    """[(variant, total ms, launches, bytes, ops)] of every instantiation of
    family kid timed since prof_enable, largest total first."""
    import ctypes
    from paper_1908_06972_amd import native as N
    n = 64
    var = (ctypes.c_uint32 * n)()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_uint64 * n)()
    by = (ctypes.c_double * n)()
    op = (ctypes.c_double * n)()
    k = ctx.lib.pft_prof_read_variants(ctx.handle, kid, n, var, ms, cnt, by, op)
    if k < 0:
        N.check(k)
    return [(var[i], ms[i], cnt[i], by[i], op[i]) for i in range(min(k, n))]


def prof_read(ctx, kid):
    import ctypes
    from paper_1908_06972_amd import native as N
    ms, cnt, by, op = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
    N.check(ctx.lib.pft_prof_read(ctx.handle, kid, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by),
                                  ctypes.byref(op)))
    return ms.value, cnt.value, by.value, op.value


def prof_enable(ctx, mask):
    from paper_1908_06972_amd import native as N
    N.check(ctx.lib.pft_prof_enable(ctx.handle, mask))


KEY_SEED = 1                                  # pft_keygen seed of the workload's keys
ROT_STEPS = [1 << i for i in range(15)]       # rotation keys 2^0..2^14 (rotate-and-sum over 2^15 slots)
SLOT_SEED0 = 303                              # slots of ciphertext i from rng(SLOT_SEED0 + i)
ENC_SEED0 = 3000                              # encryption draws of ciphertext i from seed ENC_SEED0 + i
DEFAULT_TUNING = os.path.join(ROOT, "paper_1908_06972_amd", "tuning", "large_ring_n16_l24.json")


def make_context():
    """Large-ring parameters, a context on a stream of its own (graphs can
    be captured on it) and the workload's keys drawn on the device from
    KEY_SEED: secret, public key, relinearisation key, rotation keys
    2^0..2^14."""
    import synth as S
    from paper_1908_06972_amd import ckks as L

    import torch
    lp = L.Params.from_config(S.CONFIGS["C3"])
    ctx = L.Context(lp, 0, stream=torch.cuda.Stream())
    t0 = time.time()
    ctx.keygen(KEY_SEED, ROT_STEPS)
    log("keys from seed: rlk + %d rotation keys resident, %.2f GiB device, %.1fs" % (
        len(ROT_STEPS), ctx.device_bytes() / 2 ** 30, time.time() - t0))
    return lp, ctx


def batch_slots(n, batch):
    """Unit-modulus complex slots of the batch's ciphertexts."""
    import synth as S
    return [S.slots_unit(S.rng(SLOT_SEED0 + i), n // 2) for i in range(batch)]


def encrypt_batch(ctx, lp, plains):
    """Seeded encryptions of the integer plaintexts at the top level."""
    cts = [ctx.encrypt_seeded(m, lp.L, lp.scale, ENC_SEED0 + i) for i, m in enumerate(plains)]
    ctx.synchronize()
    return cts


def import_tuning(ctx, path):
    """Load a JSON table of NTT schedules (written by --tuning-out)."""
    with open(path) as fh:
        ctx.ntt_tuning_import([(e[0], e[1], (tuple(e[2]), int(e[3]))) for e in json.load(fh)])


def setup(batch):
    lp, ctx = make_context()
    cts = encrypt_batch(ctx, lp, [lp.encode(z) for z in batch_slots(lp.n, batch)])
    return lp, ctx, cts


def chain_link(ctx, cur):
    """One link of the chain on the whole batch: RESCALE(HMult+relin(c, c))."""
    return ctx.rescale_batch(ctx.mul_relin_batch(cur, cur))


def job_step(ctx, cts):
    """One step of the workload over the batch, eager calls with fresh
    output buffers; returns the final ciphertexts."""
    cur = cts
    for _ in range(CHAIN_DEPTH):
        cur = chain_link(ctx, cur)
    return ctx.total_sum_batch(cur, ROT_SLOTS)


class GraphStep:
    """The same step with preallocated buffers, captured once in a HIP graph
    and replayed: one graph launch per step instead of ~1000 kernel launches."""

    def __init__(self, ctx, cts):
        self.ctx, self.cts = ctx, cts
        self.muls, self.rss = [], []
        level = cts[0].level
        for _ in range(CHAIN_DEPTH):
            self.muls.append([ctx.empty_ct(level) for _ in cts])
            self.rss.append([ctx.empty_ct(level - 1) for _ in cts])
            level -= 1
        self.out = [ctx.empty_ct(level) for _ in cts]
        self.run()  # eager once: sizes the scratch the capture will use
        ctx.synchronize()
        self.graph = ctx.capture(self.run)

    def run(self):
        cur = self.cts
        for d in range(CHAIN_DEPTH):
            self.ctx.mul_relin_batch(cur, cur, out=self.muls[d])
            self.ctx.rescale_batch(self.muls[d], out=self.rss[d])
            cur = self.rss[d]
        self.ctx.total_sum_batch(cur, ROT_SLOTS, out=self.out)

    def launch(self):
        self.graph.launch()


C2_PAIRS = 64
C2_SEED = 202


def c2_op_list(ctx, inputs, steps):
    """The batched-primitives op list over pairs (a_i, b_i) of mixed levels:
    m = HMult+relin(a, b), r = RESCALE(m), t = ROTATE(r, step_i), s = t + r;
    every 4th pair also takes a copy of a through NTT and INTT.  Returns
    (ciphertexts: inputs then outputs, ops)."""
    cts = list(inputs)
    ops = []
    for i in range(len(inputs) // 2):
        a, b = 2 * i, 2 * i + 1
        lvl = inputs[a].level
        m, r, t, s = len(cts), len(cts) + 1, len(cts) + 2, len(cts) + 3
        cts += [ctx.empty_ct(lvl), ctx.empty_ct(lvl - 1), ctx.empty_ct(lvl - 1), ctx.empty_ct(lvl - 1)]
        ops += [("mul_relin", a, b, m, 0, 0), ("rescale", m, 0, r, 0, 0),
                ("rotate", r, 0, t, steps[i % len(steps)], 0), ("add", t, r, s, 0, 0)]
        if i % 4 == 0:
            x = len(cts)
            cts.append(ctx.empty_ct(lvl))
            cts[x].data.copy_(inputs[a].data)
            cts[x].level, cts[x].scale = inputs[a].level, inputs[a].scale
            ops += [("ntt", x, 0, 0, 0, 0), ("intt", x, 0, 0, 0, 0)]
    return cts, ops


def c2_per_op(ctx, cts, ops):
    """The op list issued one library call per operation and ciphertext."""
    for kind, a, b, out, step, mode in ops:
        if kind == "mul_relin":
            ctx.mul_relin(cts[a], cts[b], out=cts[out])
        elif kind == "rescale":
            ctx.rescale(cts[a], mode, out=cts[out])
        elif kind == "rotate":
            ctx.rotate(cts[a], step, out=cts[out])
        elif kind == "add":
            ctx.add(cts[a], cts[b], out=cts[out])
        elif kind == "ntt":
            ctx.ntt_forward(cts[a].data, cts[a].level)
        elif kind == "intt":
            ctx.ntt_inverse(cts[a].data, cts[a].level)


def c2_bench(reps=5, region=None):
    """The batched-primitives configuration: N = 2^14, 8 ciphertext primes +
    2 special primes (dnum 4), scale 2^40; 64 ciphertext pairs at levels
    drawn from U{3..8} with slots U[-1, 1]; 16 rotation steps drawn from
    U{1..N/2-1}; the op list of c2_op_list.  Timed four ways on identical
    inputs: one call per operation (eager, and captured in one HIP graph),
    and the op-list executor (eager, and replayed from one HIP graph).  All
    four leave bit-identical outputs (checked).  region (with resume() and
    pause()): one more eager executor run between them."""
    import numpy as np
    import torch

    import synth as S
    from paper_1908_06972_amd import ckks as L

    cfg = S.CONFIGS["C2"]
    lp = L.Params.from_config(cfg)
    side = torch.cuda.Stream()
    ctx = L.Context(lp, 0, stream=side)
    g = S.rng(C2_SEED + 1)
    steps = [int(x) for x in g.integers(1, lp.n // 2, size=16)]
    ctx.keygen(KEY_SEED, steps)
    g = S.rng(C2_SEED)
    levels = [int(x) for x in g.integers(3, lp.L + 1, size=C2_PAIRS)]
    inputs = []
    for i in range(C2_PAIRS):
        for k in range(2):
            z = S.slots_uniform(S.rng(C2_SEED * 1000 + 2 * i + k), lp.n // 2)
            top = ctx.encrypt_seeded(lp.encode(z), lp.L, lp.scale, C2_SEED * 1000 + 2 * i + k)
            inputs.append(ctx.mod_drop(top, levels[i]) if levels[i] < lp.L else top)
    ctx.synchronize()

    def fresh():
        return c2_op_list(ctx, inputs, steps)

    def reset(cts, ops, ref):
        # the NTT -> INTT copies are transformed in place: restore them
        for kind, a, *_ in ops:
            if kind == "ntt":
                with torch.cuda.stream(side):
                    cts[a].data.copy_(ref[a].data)

    def same(x, y):
        return all(p.level == q.level and bool((p.data[:, :p.level] == q.data[:, :q.level]).all())
                   for p, q in zip(x, y))

    sync = ctx.synchronize
    ref, ops = fresh()
    c2_per_op(ctx, ref, ops)
    sync()
    out = {"pairs": C2_PAIRS, "levels": "U{3..8}", "rotation_steps": steps, "ops": len(ops),
           "hmult_relin_per_list": C2_PAIRS}
    # one call per operation, eager
    po, _ = fresh()
    t_po = timed(lambda: (reset(po, ops, ref), c2_per_op(ctx, po, ops)), reps, sync)
    # one call per operation, captured
    pg, _ = fresh()
    c2_per_op(ctx, pg, ops)
    sync()
    gr_po = ctx.capture(lambda: c2_per_op(ctx, pg, ops))
    t_pg = timed(lambda: (reset(pg, ops, ref), gr_po.launch()), reps, sync)
    # the op-list executor, eager
    ex, _ = fresh()
    ctx.exec_batch(ex, ops)
    sync()
    t_ex = timed(lambda: (reset(ex, ops, ref), ctx.exec_batch(ex, ops)), reps, sync)
    if region is not None:
        reset(ex, ops, ref)
        sync()
        region.resume()
        ctx.exec_batch(ex, ops)
        sync()
        region.pause()
    # the op-list executor, captured
    eg, _ = fresh()
    ctx.exec_batch(eg, ops)
    sync()
    gr_ex = ctx.capture(lambda: ctx.exec_batch(eg, ops))
    t_eg = timed(lambda: (reset(eg, ops, ref), gr_ex.launch()), reps, sync)
    identical = same(po, ref) and same(pg, ref) and same(ex, ref) and same(eg, ref)
    if not identical:
        print("batched op list: outputs differ between launch modes", file=sys.stderr)
        sys.exit(1)
    gr_po.close()
    gr_ex.close()
    for name, t in (("per_op", t_po), ("per_op_graph", t_pg), ("exec_batch", t_ex), ("exec_batch_graph", t_eg)):
        out[name] = {"ms_per_list": round(1000.0 * t, 3), "hmult_relin_per_s": round(C2_PAIRS / t, 1)}
    out["identical_outputs"] = identical
    out["speedup_exec_graph_over_per_op"] = round(t_po / t_eg, 2)
    out["note"] = ("times include the device-to-device copies restoring the NTT/INTT operands (one small copy "
                   "per 4th pair, the same in every mode)")
    log("batched op list: %s" % {k: v for k, v in out.items() if isinstance(v, dict)})
    ctx.close()
    return out


SERVING_MIX = {"N=2^14": 3, "N=2^15": 2, "N=2^16": 1}


def serving_bench(n_requests, rate=200.0, level=4, pool=16, budget_gib=16, saturate_rate=2000.0):
    """Poisson stream of encrypted bag-of-words inferences (vocabulary 32768,
    embedding 64, 8 classes) over three parameter sets in the ratio 3:2:1
    (N = 2^14 / 2^15 / 2^16 with the batched / bag-of-words / large-ring
    prime chains), inputs encrypted at level 4 (depth 3), keys resident.
    Served twice on the same trace: continuous batching (one stream per
    parameter set, overlapping) and a plain per-op server (one request at a
    time, arrival order)."""
    import synth as S
    from paper_1908_06972_amd.serving import GpuExecutor, Scheduler, build_sets, poisson_trace

    specs = {"N=2^14": S.CONFIGS["C2"], "N=2^15": S.CONFIGS["C4"], "N=2^16": S.CONFIGS["C3"]}
    H, O = S.bow_weights(404, 32768, 64, 8)
    t0 = time.time()
    sets, policies, words, _ = build_sets(specs, H, O, pool_size=pool, level=level, draws=S)
    key_bytes = sum(ctx.device_bytes() for ctx, _, _ in sets.values())
    log("serving: 3 parameter sets ready in %.1fs, %.2f GiB resident" % (time.time() - t0, key_bytes / 2 ** 30))
    ex = GpuExecutor(sets)
    warm = Scheduler(ex, policies, budget_gib << 30).run(poisson_trace(1, 12, 1000.0, SERVING_MIX,
                                                                       {k: pool for k in specs}, words))
    assert warm.completed == 12
    out = {"rate_req_per_s": rate, "requests": n_requests, "mix": "3:2:1 over N=2^14/2^15/2^16", "level": level,
           "vocab": 32768, "dim": 64, "classes": 8, "hbm_budget_gib": budget_gib,
           "resident_gib": round(key_bytes / 2 ** 30, 3)}
    for mode, cont in (("continuous", True), ("per_op", False)):
        trace = poisson_trace(505, n_requests, rate, SERVING_MIX, {k: pool for k in specs}, words)
        st = Scheduler(ex, policies, budget_gib << 30, continuous=cont).run(trace)
        out[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.summary().items()}
        log("serving %s: %s" % (mode, out[mode]))
    # the same mix arriving faster than one-request-at-a-time serving keeps up with
    sat = {"rate_req_per_s": saturate_rate, "requests": n_requests}
    for mode, cont in (("continuous", True), ("per_op", False)):
        trace = poisson_trace(506, n_requests, saturate_rate, SERVING_MIX, {k: pool for k in specs}, words)
        st = Scheduler(ex, policies, budget_gib << 30, continuous=cont).run(trace)
        sat[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.summary().items()}
        log("serving at %.0f req/s, %s: %s" % (saturate_rate, mode, sat[mode]))
    out["saturated"] = sat
    for ctx, _, _ in sets.values():
        ctx.synchronize()
    # the same sets with a 2 GiB rotation-key budget: keys beyond each set's
    # share live in pinned host memory and are copied in on use
    kbudget = 2 << 30
    t0 = time.time()
    sets_c, policies_c, words_c, _ = build_sets(specs, H, O, pool_size=pool, level=level, draws=S,
                                                key_budget_bytes=kbudget)
    res_c = sum(ctx.device_bytes() for ctx, _, _ in sets_c.values())
    log("serving: key-cache sets ready in %.1fs, %.2f GiB resident" % (time.time() - t0, res_c / 2 ** 30))
    ex_c = GpuExecutor(sets_c)
    n_c = min(n_requests, 300)
    trace = poisson_trace(507, n_c, rate, SERVING_MIX, {k: pool for k in specs}, words_c)
    st = Scheduler(ex_c, policies_c, budget_gib << 30, continuous=True).run(trace)
    cache = {k: ctx.key_cache_stats() for k, (ctx, _, _) in sets_c.items()}
    out["keys_over_budget"] = {
        "rotation_key_budget_gib": kbudget / 2 ** 30, "resident_gib": round(res_c / 2 ** 30, 3), "requests": n_c,
        "continuous": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.summary().items()},
        "key_cache": {k: {"resident_keys": v["max_resident"], "misses": v["misses"], "hits": v["hits"],
                          "copied_ahead": v["prefetches"], "gib_copied": round(v["bytes_in"] / 2 ** 30, 2)}
                      for k, v in cache.items()}}
    log("serving keys over budget: %s" % out["keys_over_budget"])
    for ctx, _, _ in sets_c.values():
        ctx.synchronize()
        ctx.close()
    return out


def predict_bench(n_docs=32, level=6, reps=3, region=None):
    """The predict step of training with encrypted weights (Sec. 4.2) at the
    bag-of-words shapes (N = 2^15 prime chain, vocabulary 32768 = two input
    ciphertexts, embedding 64, 8 classes): both weight matrices encrypted
    (128 + 8 diagonal ciphertexts), a batch of documents at level `level`
    (five levels consumed), then the degree-2 softmax approximation.
    region (with resume() and pause()): one more batch runs between them."""
    import numpy as np

    import synth as S
    from paper_1908_06972_amd import ckks as L
    from paper_1908_06972_amd import training as T

    cfg = S.CONFIGS["C4"]
    lp = L.Params.from_config(cfg)
    ctx = L.Context(lp, 0)
    n, t = lp.n, lp.n // 2
    dim, classes, n_in = 64, 8, 2
    kd = S.key_draws(61, n, lp.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(61, 0, n, lp.key_moduli(), lp.dnum)
    ctx.gen_relin_key(a, e)
    for st in sorted(set(T.rotation_steps(dim, t) + T.rotation_steps(classes, dim))):
        a, e = S.switch_key_draws(61, 6000 + st, n, lp.key_moduli(), lp.dnum)
        ctx.gen_rotation_key(st, a, e)
    H, O = S.bow_weights(62, n_in * t, dim, classes)
    seed = [7000]

    def draws():
        seed[0] += 1
        d = S.enc_draws(seed[0], n)
        return d.v, d.e0, d.e1

    t0 = time.time()
    model = T.EncryptedBowModel(T.encrypt_diagonals(ctx, H.T, dim, t, n_in, level, draws),
                                T.encrypt_diagonals(ctx, O.T, classes, dim, 1, level - 2, draws),
                                dim, classes, n_in, t)
    counts, words = S.bow_documents(63, n_docs, n_in * t)
    docs = []
    for d in range(n_docs):
        row = []
        for c in range(n_in):
            v, e0, e1 = draws()
            row.append(ctx.encrypt(lp.encode(counts[d][c * t:(c + 1) * t].astype(np.float64), lp.scale), level,
                                   lp.scale, v, e0, e1))
        docs.append(row)
    ctx.synchronize()
    log("predict: model encrypted (%d + %d diagonals) and %d documents in %.1fs" % (
        len(model.stage1), len(model.stage2), n_docs, time.time() - t0))
    out = T.predict_encrypted(ctx, model, docs, list(words))
    sec = timed(lambda: T.predict_encrypted(ctx, model, docs, list(words)), reps, ctx.synchronize)
    if region is not None:
        ctx.synchronize()
        region.resume()
        T.predict_encrypted(ctx, model, docs, list(words))
        ctx.synchronize()
        region.pause()
    err = 0.0
    for d in range(2):
        got = lp.decode(ctx.decrypt(out[d]), out[d].scale, classes).real
        s = ((counts[d].astype(np.float64) @ H) / float(words[d])) @ O  # Alg. 1 steps 2-3 in fp64
        err = max(err, float(np.max(np.abs(got - (s * s / 8 + s / 2 + 0.25)))))
    res = {"docs_per_s": round(n_docs / sec, 2), "ms_per_batch": round(1000.0 * sec, 2), "batch": n_docs,
           "level": level, "n": n, "limbs": lp.L, "vocab": n_in * t, "dim": dim, "classes": classes,
           "max_abs_err_vs_fp64": err,
           "note": "encrypted H and O (diagonal BSGS, HMUL + one relinearisation per giant step), 1/w, then "
                   "X^2/8 + X/2 + 1/4; error of 2 documents against Alg. 1 steps 2-3 and the polynomial in fp64"}
    log("predict: %s" % res)
    ctx.close()
    return res


def bow_bench(n_docs=32, reps=3, singles=8, region=None):
    """The bag-of-words inference workload: N = 2^15, 16 ciphertext primes
    (+4 special, dnum 4), scale 2^40; vocabulary 32768 (two input
    ciphertexts per document), plaintext embedding 32768 x 64 and classifier
    64 x 8 with N(0, 0.1^2) weights; documents of Zipf-distributed counts,
    50-500 tokens each, encrypted at the top level; Alg. 1 steps 2-3 as
    diagonal BSGS PtMatVec + 1/w + PtMatVec, three levels.  Reports the
    batch of n_docs (documents/s), single-document latencies (median and
    worst of `singles`), the error against fp64 and argmax agreement.
    region (with resume() and pause()): one more batch runs between them."""
    import statistics

    import numpy as np
    import torch

    import synth as S
    from paper_1908_06972_amd import ckks as L
    from paper_1908_06972_amd.inference import BowModel, encrypted_inference, split_counts

    lp = L.Params.from_config(S.CONFIGS["C4"])
    ctx = L.Context(lp, 0, stream=torch.cuda.Stream())
    t0 = time.time()
    H, O = S.bow_weights(404, 32768, 64, 8)
    model = BowModel(ctx, H, O, lp.L)
    ctx.keygen(KEY_SEED, model.rotation_steps())
    counts, words = S.bow_documents(405, n_docs, 32768)
    docs = [[ctx.encrypt_seeded(lp.encode(v), lp.L, lp.scale, 40500 + 4 * d + c)
             for c, v in enumerate(split_counts(counts[d], model.n_in, model.t))] for d in range(n_docs)]
    ctx.synchronize()
    log("bag of words: model (%d + %d diagonals), keys and %d documents in %.1fs" % (
        model.stage1.b * model.stage1.G * model.n_in, model.stage2.b * model.stage2.G, n_docs, time.time() - t0))
    out = encrypted_inference(ctx, model, docs, list(words))
    sec = timed(lambda: encrypted_inference(ctx, model, docs, list(words)), reps, ctx.synchronize)
    if region is not None:
        ctx.synchronize()
        region.resume()
        encrypted_inference(ctx, model, docs, list(words))
        ctx.synchronize()
        region.pause()
    lat = []
    for d in range(singles):
        ctx.synchronize()
        t1 = time.perf_counter()
        encrypted_inference(ctx, model, [docs[d]], [words[d]])
        ctx.synchronize()
        lat.append(time.perf_counter() - t1)
    err, agree = 0.0, 0
    for d in range(n_docs):
        got = lp.decode(ctx.decrypt(out[d]), out[d].scale, 8).real
        ref = ((counts[d].astype(np.float64) @ H) / float(words[d])) @ O  # Alg. 1 steps 2-3 in fp64
        err = max(err, float(np.max(np.abs(got - ref))))
        agree += int(np.argmax(got) == np.argmax(ref))
    res = {"docs_per_s": round(n_docs / sec, 2), "ms_per_batch": round(1000.0 * sec, 2), "batch": n_docs,
           "single_doc_ms_p50": round(1000.0 * statistics.median(lat), 2),
           "single_doc_ms_max": round(1000.0 * max(lat), 2),
           "rotations_per_doc": len(model.rotation_order()) + (model.stage1.b - 1) * (model.n_in - 1),
           "n": lp.n, "limbs": lp.L, "vocab": 32768, "dim": 64, "classes": 8,
           "max_abs_err_vs_fp64": err, "argmax_agree": "%d/%d" % (agree, n_docs),
           "note": "plaintext weights, diagonal BSGS PtMatVec (Sec. 4.1); rotations per document: the baby steps of "
                   "each input ciphertext, giant steps and the sum steps of both stages"}
    log("bag of words: %s" % res)
    ctx.close()
    return res


def paper_inference_bench(batch=8, classes=14):
    """Encrypted fasttext inference at the paper's own inference shapes
    (Sec. 6, Table 4: N = 8192, five 40-bit primes = log q 200, scale 2^40;
    vocabulary m = 500000 -> 123 input ciphertexts, embedding n = 50), inputs
    at the top level, three levels consumed.  Two packings of the same
    products: the paper's column packing (one TotalSum per column of H,
    n log2(t) rotations) and the diagonal BSGS form (rotations planned per
    input count; H padded to 64 columns, O to 16 classes).  Per-example
    latency (one document) and throughput over a batch."""
    import numpy as np

    import synth as S
    from paper_1908_06972_amd import ckks as L
    from paper_1908_06972_amd import colpack as CPK
    from paper_1908_06972_amd.inference import BowModel, encrypted_inference
    from paper_1908_06972_amd.training import bsgs_plan

    lp = L.Params(13, 5, 40, 40, 1, 60, 5, 2 ** 40)
    ctx = L.Context(lp, 0)
    n, t = lp.n, lp.n // 2
    vocab, dim = 500000, 50
    n_in = -(-vocab // t)
    kd = S.key_draws(81, n, lp.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    t0 = time.time()
    H, O = S.bow_weights(82, vocab, dim, classes)
    col = CPK.ColPackModel(ctx, H, O, lp.L)
    Hp = np.zeros((vocab, 64))
    Hp[:, :dim] = H
    Op = np.zeros((64, classes))
    Op[:dim] = O
    diag = BowModel(ctx, Hp, Op, lp.L, n_in=n_in)
    for st in sorted(set(col.rotation_steps()) | set(diag.rotation_steps())):
        a, e = S.switch_key_draws(81, 8000 + st, n, lp.key_moduli(), lp.dnum)
        ctx.gen_rotation_key(st, a, e)
    counts, words = S.bow_documents(83, batch, vocab)
    docs = []
    for d in range(batch):
        v = np.zeros(n_in * t)
        v[:vocab] = counts[d]
        row = []
        for c in range(n_in):
            dr = S.enc_draws(8300 + n_in * d + c, n)
            row.append(ctx.encrypt(lp.encode(v[c * t:(c + 1) * t], lp.scale), lp.L, lp.scale, dr.v, dr.e0, dr.e1))
        docs.append(row)
    ctx.synchronize()
    log("paper inference: models (%d column + %d diagonal plaintexts), keys and %d documents in %.1fs" % (
        dim * n_in, 64 * n_in, batch, time.time() - t0))
    b1, G1 = bsgs_plan(64, n_in)
    b2, G2 = bsgs_plan(diag.c_pad, 1)
    rot_diag = (n_in * (b1 - 1) + G1 - 1 + int(np.log2(t // 64))) + (b2 - 1 + G2 - 1 + int(np.log2(64 // diag.c_pad)))
    out = {"n": n, "limbs": lp.L, "log_q": sum(int(q).bit_length() for q in lp.q), "vocab": vocab,
           "input_ciphertexts": n_in, "dim": dim, "classes": classes, "batch": batch}
    for name, run, rots in (("column", lambda ds: CPK.encrypted_inference(ctx, col, ds, list(words[:len(ds)])),
                             dim * int(np.log2(t))),
                            ("diagonal", lambda ds: encrypted_inference(ctx, diag, ds, list(words[:len(ds)])),
                             rot_diag)):
        res = run(docs[:1])
        one = timed(lambda: run(docs[:1]), 3, ctx.synchronize)
        many = timed(lambda: run(docs), 2, ctx.synchronize)
        got = lp.decode(ctx.decrypt(res[0]), res[0].scale, classes).real
        want = ((counts[0].astype(np.float64) @ H) / float(words[0])) @ O  # Alg. 1 steps 2-3 in fp64
        out[name] = {"s_per_example": round(one, 5), "examples_per_s": round(batch / many, 2),
                     "rotations_per_example": int(rots), "max_abs_err_vs_fp64": float(np.max(np.abs(got - want))),
                     "argmax_equal": bool(np.argmax(got) == np.argmax(want))}
        log("paper inference %s: %s" % (name, out[name]))
    out["note"] = ("paper Table 4 (V100, same shapes): 0.23-0.66 s per example; column = the paper's packing "
                   "(n TotalSums), diagonal = BSGS with %d baby x %d giant steps over %d inputs" % (b1, G1, n_in))
    ctx.close()
    return out


def timed(fn, reps, sync):
    """Mean seconds per call of fn over reps calls, after one untimed call
    (which also lets the NTT autotuner settle the call's batch classes)."""
    fn()
    sync()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    sync()
    return (time.perf_counter() - t) / reps


def host_cpu():
    """(logical CPUs, model name, OpenMP threads the oracle uses) of this host."""
    import subprocess
    nproc = os.cpu_count() or 1
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return nproc, model, int(os.environ.get("OMP_NUM_THREADS", nproc))


def median_seconds(fn, reps):
    """Median wall time of reps calls of fn."""
    import statistics
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return statistics.median(ts)


class OracleWorld:
    """The oracle's keys and one encrypted input for a parameter set (from the
    shared seeded draws), for timing."""

    def __init__(self, cfg_name, rot_steps=(1,)):
        import synth as S
        from oracle import ckks as C
        self.C = C
        self.P = P = C.Params.from_config(S.CONFIGS[cfg_name])
        n = P.n
        C.set_mul_mode(0 if n <= 4096 else 1)  # schoolbook at N = 4096, the oracle's transform above
        kd = S.key_draws(1, n, P.q)
        self.pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
        a, e = S.switch_key_draws(1, 0, n, P.key_moduli(), P.dnum)
        self.rlk = C.relin_key(P, kd.s, a, e)
        self.rot = {}
        for st in rot_steps:
            a, e = S.switch_key_draws(1, 1000 + st, n, P.key_moduli(), P.dnum)
            self.rot[st] = C.rotation_key(P, kd.s, st, a, e)
        d = S.enc_draws(3000, n)
        self.ct = C.encrypt(P, self.pk, S.plaintext_coeffs(S.rng(5), n, int(P.scale)), P.L, d.v, d.e0, d.e1, P.scale)

    def hmult(self):
        return self.C.hmul_relin(self.P, self.ct, self.ct, self.rlk)

    def rescale(self):
        return self.C.rescale(self.P, self.ct)

    def rotate_add(self):
        return self.C.hadd(self.P, self.ct, self.C.rotate(self.P, self.ct, 1, self.rot[1]))


def limb_ntt_seconds(reps, threads):
    """Median seconds of the oracle's transform of one N = 2^16 limb, and of
    a 24-limb polynomial spread over `threads` host threads."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import synth as S
    from oracle import _ring
    from oracle import ckks as C
    P = C.Params.from_config(S.CONFIGS["C3"])
    lib = _ring.lib()
    g = S.rng(9)
    rows = [_ring.u64(g.integers(0, q, P.n, dtype=np.uint64)) for q in P.q]
    outs = [np.empty(P.n, dtype=np.uint64) for _ in P.q]

    def one(i):
        lib.or_ntt_fast(_ring.ptr(rows[i]), _ring.ptr(outs[i]), P.n, int(P.q[i]), int(P.psi[int(P.q[i])]))

    limb = median_seconds(lambda: one(1), reps)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        poly = median_seconds(lambda: list(ex.map(one, range(P.L))), reps)
    return limb, poly


def cpu_baseline(reps=10):
    """The oracle (never tuned) on a bounded sample of the same job, on this
    host's cores: medians of `reps` runs of one HMult+relin, one RESCALE and
    one ROTATE+HADD of one N = 2^16, L = 24 ciphertext (OpenMP over limbs),
    combined into the job's rate; the oracle's one-limb transform beside it."""
    nproc, model, threads = host_cpu()
    w = OracleWorld("C3")
    th = median_seconds(w.hmult, reps)
    tr = median_seconds(w.rescale, reps)
    tt = median_seconds(w.rotate_add, reps)
    limb, poly = limb_ntt_seconds(reps, threads)
    per_ct = CHAIN_DEPTH * (th + tr) + 15 * tt
    return {
        "value": CHAIN_DEPTH / per_ct,
        "unit": "HMult+relin/s",
        "cores": threads,
        "kind": "oracle",
        "nproc": nproc,
        "cpu_model": model,
        "sample": "medians of %d runs each of one HMult+relin, one RESCALE and one ROTATE+HADD of one N=2^16 L=24 "
                  "ciphertext (oracle, %d OpenMP threads); whole-job rate = 8 / (8 (t_hmult + t_rescale) + 15 "
                  "t_rotate_add) with t_hmult=%.3fs t_rescale=%.3fs t_rotate_add=%.3fs" % (reps, threads, th, tr, tt),
        "limb_ntt_per_s_1thread": round(1.0 / limb, 2),
        "poly_ntt_per_s": round(1.0 / poly, 3),
    }


def cpu_baseline_full(reps=10):
    """The full CPU table of the oracle on this host (run once, stored under
    profiles/): limb and 24-limb transforms, the single-op workload (N = 4096,
    schoolbook products) and the large-ring operations, medians of `reps`
    runs on all threads and on one thread (a child process with
    OMP_NUM_THREADS=1), and one bag-of-words inference (N = 2^15, 16 limbs,
    vocabulary 32768, 64 -> 8)."""
    import subprocess
    nproc, model, threads = host_cpu()
    res = {"nproc": nproc, "cpu_model": model, "threads": threads, "reps": reps}
    if threads > 1:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        log("cpu baseline: one-thread child process")
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-full", "--reps",
                              str(reps)], env=env, stdout=subprocess.PIPE, text=True, check=True).stdout
        res["one_thread"] = json.loads(out.strip().splitlines()[-1])
    limb, poly = limb_ntt_seconds(reps, threads)
    res["limb_ntt_s"], res["poly_ntt_s"] = limb, poly
    log("cpu baseline (%d threads): limb NTT %.4fs, 24-limb NTT %.4fs" % (threads, limb, poly))
    for name in ("C1", "C3"):
        w = OracleWorld(name)
        r = reps if name == "C1" or threads > 1 else max(3, reps // 3)
        res[name] = {"runs": r}
        for op, fn in (("hmult_relin_s", w.hmult), ("rescale_s", w.rescale), ("rotate_add_s", w.rotate_add)):
            res[name][op] = median_seconds(fn, r)
            log("cpu baseline (%d threads): %s %s %.3fs (median of %d)" % (threads, name, op, res[name][op], r))
    if threads > 1:
        res["C4_inference_s"] = oracle_inference_seconds()
        log("cpu baseline (%d threads): one bag-of-words inference %.1fs" % (threads, res["C4_inference_s"]))
    return res


def oracle_inference_seconds():
    """One encrypted bag-of-words inference on the oracle at the bag-of-words
    shapes (stage 1, 1/w, stage 2 with BSGS PtMatVec; the diagonals encoded by
    the oracle's encoder), wall seconds of one run."""
    import numpy as np

    import synth as S
    from oracle import ckks as C
    from oracle import ptmatvec as PM
    P = C.Params.from_config(S.CONFIGS["C4"])
    C.set_mul_mode(1)
    n, t, L = P.n, P.n // 2, P.L
    kd = S.key_draws(1, n, P.q)
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    steps = sorted(set(PM.rotation_steps(64, t, 2) + PM.rotation_steps(8, 64, 1)))
    keys = {}
    for st in steps:
        a, e = S.switch_key_draws(1, 1000 + st, n, P.key_moduli(), P.dnum)
        keys[st] = C.rotation_key(P, kd.s, st, a, e)
    H, O = S.bow_weights(404, 2 * t, 64, 8)
    s1, s2 = float(P.q[L - 1]), float(P.q[L - 3])
    p1 = [[[C.encode(d, n, s1) for d in g] for g in c] for c in PM.prerotated_diagonals(H.T, 64, t, 2, t)]
    p2 = [[[C.encode(d, n, s2) for d in g] for g in c] for c in PM.prerotated_diagonals(O.T, 8, 64, 1, t)]
    counts, words = S.bow_documents(405, 1, 2 * t)
    cts = []
    for c in range(2):
        d = S.enc_draws(4500 + c, n)
        cts.append(C.encrypt(P, pk, C.encode(counts[0][c * t:(c + 1) * t].astype(np.float64), n, P.scale), L,
                             d.v, d.e0, d.e1, P.scale))
    t0 = time.perf_counter()
    o = C.rescale(P, PM.ptmatvec(P, cts, p1, 64, t, keys, s1))
    m, ms = PM.constant_plain(P, 1.0 / float(words[0]), o.level)
    o = C.rescale(P, C.hmul_plain(P, o, m, ms))
    C.rescale(P, PM.ptmatvec(P, [o], p2, 8, 64, keys, s2))
    return time.perf_counter() - t0


def main():
    args = parse()
    if args.summarize:
        print(summarize(*args.summarize, args.kernel, args.family, args.commands, sq_dir=args.sq, mix_dir=args.mix),
              end="")
        return
    if args.cpu_baseline_full:
        print(json.dumps(cpu_baseline_full(args.reps)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requests would be sharded "
              "one process per GPU); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.profile_workload:
        class Pause:
            """Idle before (1 s) and after (3 s) the profiled run, so that its
            dispatches stand apart in a kernel trace: they follow the last
            gap of about a second before the first gap of three."""

            def resume(self):
                torch.cuda.synchronize()
                time.sleep(1.0)
                log("profiled run: start")

            def pause(self):
                torch.cuda.synchronize()
                log("profiled run: end")
                time.sleep(3.0)

        if args.profile_workload == "bow":
            bow_bench(reps=1, singles=1, region=Pause())
        elif args.profile_workload == "predict":
            predict_bench(reps=1, region=Pause())
        else:
            c2_bench(reps=1, region=Pause())
        return

    lp, ctx, cts = setup(args.batch)
    sync = torch.cuda.synchronize
    if args.tuning_in and not args.retune and os.path.exists(args.tuning_in):
        import_tuning(ctx, args.tuning_in)
        log("NTT schedules imported from %s" % args.tuning_in)

    def save_tuning():
        table = [[inv, cls, list(sched[0]), sched[1]] for inv, cls, sched in ctx.ntt_tuning_export()]
        if args.tuning_out:
            with open(args.tuning_out, "w") as fh:
                json.dump(table, fh)
        return table

    if args.profile_steps:
        # one settling step (autotuner), then the profiled steps.  Timing the
        # key inner product's launches (HIP events) keeps its two row kinds
        # on one stream, one after the other, so that the trace gives each
        # launch its own duration (the timed steps run them concurrently).
        prof_enable(ctx, 1 << FAMILIES.index("key_inner_product"))
        for i in range(1 + args.profile_steps):
            job_step(ctx, cts)
            sync()
            log("profile step %d done" % i)
        save_tuning()
        return

    # rank kernel families over one untimed step
    prof_enable(ctx, (1 << len(FAMILIES)) - 1)
    job_step(ctx, cts)
    sync()
    totals = {k: prof_read(ctx, k) for k in range(len(FAMILIES))}
    kernels = [(k,) + v for k in range(len(FAMILIES)) for v in prof_variants(ctx, k)]
    prof_enable(ctx, 0)
    step_total = sum(v[0] for v in totals.values())
    log("kernel families over one step: " + ", ".join(
        "%s %.1fms (%d)" % (FAMILIES[k], v[0], v[1]) for k, v in sorted(totals.items(), key=lambda kv: -kv[1][0])
        if v[1]))
    # the dominant kernel: the single instantiation with the largest total time
    kernels.sort(key=lambda r: -r[2])
    dom, dom_variant = kernels[0][0], kernels[0][1]
    top_kernels = [{"kernel": kernel_name(k, v), "share_of_step": round(ms / step_total, 3), "launches": c,
                    "avg_launch_us": round(1000.0 * ms / max(c, 1), 1),
                    "alg_gbs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
                   for k, v, ms, c, by, op in kernels[:6]]
    log("top kernels: " + ", ".join("%s %.1f%%" % (t["kernel"], 100 * t["share_of_step"]) for t in top_kernels))

    for i in range(args.warmup):
        job_step(ctx, cts)
        sync()
        log("warmup step %d done" % i)

    # timed region: batched eager launches, each step enqueued while the
    # previous one runs; the dominant kernel family is bracketed with HIP
    # events (on the stream of each launch) during the last timed step only,
    # so that the events' own cost touches one step
    prof_enable(ctx, 0)
    roctx = Roctx()
    sync()
    roctx.resume()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            sync()  # the stream idle before the events are switched on
            if i:
                log("timed steps 0..%d done" % (i - 1))
            prof_enable(ctx, 1 << dom)
        job_step(ctx, cts)
    sync()
    log("timed step %d done" % (args.steps - 1))
    elapsed = time.perf_counter() - t0
    roctx.pause()
    dom_ms = prof_read(ctx, dom)[0]
    rows = [r for r in prof_variants(ctx, dom) if r[0] == dom_variant] or [(dom_variant, 0.0, 0, 0.0, 0.0)]
    variant, d_ms, d_cnt, d_bytes, d_ops = rows[0]
    prof_enable(ctx, 0)

    hmults = args.batch * CHAIN_DEPTH * args.steps
    ms_per_step = 1000.0 * elapsed / args.steps
    value = hmults / elapsed

    breakdown = None
    if not args.no_breakdown:
        # the same step captured once in a HIP graph and replayed; its output
        # must equal the eager step's output bit for bit
        gstep = GraphStep(ctx, cts)
        ref = job_step(ctx, cts)
        gstep.launch()
        sync()
        identical = all(torch.equal(a.data, b.data) for a, b in zip(ref, gstep.out))
        if not identical:
            print("graph replay differs from the eager step", file=sys.stderr)
            sys.exit(1)
        t_graph = timed(gstep.launch, max(1, args.steps), sync)
        # the eager step again with no HIP events around any launch: what the
        # bracketing of the dominant family costs the timed region
        t_plain = timed(lambda: job_step(ctx, cts), max(1, args.steps), sync)
        gstep.graph.close()
        # separately timed per-operation rates at level 24 on the same batch
        reps = 3
        t_mul = timed(lambda: ctx.mul_relin_batch(cts, cts), reps, sync)
        t_rot = timed(lambda: ctx.rotate_batch(cts, 1), reps, sync)
        t_rs = timed(lambda: ctx.rescale_batch(cts), reps, sync)
        t_single = timed(lambda: [ctx.mul_relin(c, c) for c in cts], 1, sync)
        polys = torch.empty((2 * args.batch, lp.L, lp.n), dtype=torch.int64, device="cuda")
        for i, c in enumerate(cts):
            polys[2 * i:2 * i + 2].copy_(c.data)
        sync()
        t_ntt = timed(lambda: ctx.ntt_forward(polys, lp.L), reps, sync)
        t_intt = timed(lambda: ctx.ntt_inverse(polys, lp.L), reps, sync)
        breakdown = {
            "hmult_relin_per_s": args.batch / t_mul,
            "rotate_per_s": args.batch / t_rot,
            "rescale_per_s": args.batch / t_rs,
            "ntt_per_s": 2 * args.batch / t_ntt,
            "intt_per_s": 2 * args.batch / t_intt,
            "limb_ntt_per_s": 2 * args.batch * lp.L / t_ntt,
            "unbatched_hmult_relin_per_s": args.batch / t_single,
            "graph_ms_per_step": 1000.0 * t_graph,
            "eager_ms_per_step_without_events": 1000.0 * t_plain,
            "graph_hmult_relin_per_s": args.batch * CHAIN_DEPTH / t_graph,
            "graph_equals_eager": identical,
            "note": "level 24, batch of %d, per-operation loops after the timed region; ntt = forward NTT of one "
                    "24-limb polynomial; unbatched = one mul_relin call per ciphertext; graph = the timed step "
                    "replayed from one HIP graph; eager_ms_per_step_without_events = the timed step run again "
                    "without the HIP events that bracket the dominant kernel family" % args.batch,
        }

    avg_ms = d_ms / max(d_cnt, 1)
    gbs = d_bytes / (d_ms * 1e-3) / 1e9 if d_ms > 0 else 0.0
    kname = kernel_name(dom, variant)
    stored = stored_profile(kname)
    traffic = None
    alu = None
    if stored:
        traffic = stored.get("traffic_bytes_per_launch")
        if stored.get("valu_insts_per_launch") and avg_ms > 0:
            # one wave-level VALU instruction = 64 lane-ops; peak issue is one
            # wave instruction per CU per clock (4 SIMDs x 16 lanes)
            lane_ops = stored["valu_insts_per_launch"] * 64.0
            alu = {"achieved": round(lane_ops / (avg_ms * 1e-3) / 1e9, 1), "peak": ALU_PEAK_GOPS,
                   "unit": "G lane-op/s",
                   "frac": round(lane_ops / (avg_ms * 1e-3) / 1e9 / ALU_PEAK_GOPS, 4),
                   "source": "SQ_INSTS_VALU per launch from profiles/ over this launch time"}
    hbm_frac = gbs / HBM_PEAK_GBS
    roofline = {
        "kernel": kname,
        "family": FAMILIES[dom],
        "bound": "hbm",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(hbm_frac, 4),
        "traffic": traffic,
        "avg_launch_us": round(1000.0 * avg_ms, 2),
        "launches": d_cnt,
        "alg_bytes_per_launch": d_bytes / max(d_cnt, 1),
        "alg_ops_per_launch": d_ops / max(d_cnt, 1),
        "alg_bytes_note": "method bytes: operands read and results written once, 8 B per residue; words a "
                          "transform leaves between its passes are layout cost and not counted",
        "family_share_of_step": round(totals[dom][0] / step_total, 3) if step_total else None,
        "kernel_share_of_family": round(d_ms / dom_ms, 3) if dom_ms else None,
        "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_frac, 4)},
        "alu": alu,
        "top_kernels": top_kernels,
    }
    if alu and alu["frac"] > hbm_frac:
        # the kernel is further along its integer-ALU roof than its HBM roof
        roofline.update({"bound": "alu", "achieved": alu["achieved"], "peak": alu["peak"], "unit": alu["unit"],
                         "frac": alu["frac"]})
    elif not alu and d_bytes == 0:
        # no method bytes (it only reads and writes the middle of transforms)
        # and no stored counters taken on this kernel source: its roof is
        # unknown here, not an HBM fraction of zero
        roofline.update({"bound": "alu", "achieved": None, "peak": ALU_PEAK_GOPS, "unit": "G lane-op/s",
                         "frac": None, "note": "no counters under profiles/ for this kernel source"})
    # whole operations and the whole step against the HBM peak
    copy_gbs = copy_bandwidth()
    ops = op_alg_bytes(lp, args.batch)
    operations = None
    if breakdown:
        rates = {"hmult_relin": breakdown["hmult_relin_per_s"], "rotate": breakdown["rotate_per_s"],
                 "rescale": breakdown["rescale_per_s"], "poly_ntt": breakdown["ntt_per_s"]}
        operations = {k: {"rate_per_s": round(rates[k], 2), "alg_bytes": ops[k],
                          "achieved_gbs": round(rates[k] * ops[k] / 1e9, 1),
                          "frac": round(rates[k] * ops[k] / 1e9 / HBM_PEAK_GBS, 4)} for k in rates}
    sb = step_alg_bytes(lp, args.batch)
    st_rec = stored_step()
    step = {"alg_bytes": sb, "achieved_gbs": round(sb / (ms_per_step * 1e-3) / 1e9, 1),
            "frac": round(sb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "counted_bytes": st_rec["traffic_bytes_per_step"] if st_rec else None,
            "counted_over_alg": round(st_rec["traffic_bytes_per_step"] / sb, 3) if st_rec else None}
    roofline["operations"] = operations
    roofline["step"] = step
    roofline["copy_gbs"] = round(copy_gbs, 1)
    log("roofline: %s %.1f GB/s method (%.3f of HBM); step %.1f GB/s (%.4f); copy %.0f GB/s" % (
        kname, gbs, hbm_frac, step["achieved_gbs"], step["frac"], copy_gbs))

    tuning = save_tuning()
    batched = None
    if not args.no_batched:
        batched = c2_bench()
    serving = None
    if args.serve_requests > 0:
        serving = serving_bench(args.serve_requests)
    bow = None
    if not args.no_bow:
        bow = bow_bench()
    predict = None
    if not args.no_predict:
        predict = predict_bench()
    paper_inf = None
    if not args.no_paper_inference:
        paper_inf = paper_inference_bench()
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)...")
        cpu = cpu_baseline()

    out = {
        "metric": "HMult+relin/s and NTT/s at N=2^16,L=24; p50/p99 encrypted-inference latency",
        "value": round(value, 2),
        "unit": "HMult+relin/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "large ring: N=2^16, L=24 (+K=6, dnum=4), scale 2^50, batch %d; depth-8 "
                               "HMult+relin+rescale chain then rotate-and-sum over 2^15 slots" % args.batch,
                   "global_batch": args.batch, "log_n": 16, "levels": lp.L, "special_primes": lp.K, "dnum": lp.dnum,
                   "ntt_schedules": [{"inverse": bool(i), "class": c & 31, "column16_only": bool(c & 32),
                                      "radices": r, "direct_rows": bool(f & 1),
                                      "residues_per_thread": 8 if f & 2 else 16} for i, c, r, f in tuning]},
        "breakdown": breakdown,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "bag_of_words": bow,
        "serving": serving,
        "predict": predict,
        "paper_inference": paper_inf,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
