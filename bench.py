"""Benchmark: the p=17 bridge workload on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Step = one bridge pass over a batch of 256 encrypted inputs x in [0, 17) at
n = 16384 with eight 55-bit primes: 17 equality chains per input, each four
squarings with relinearization, then the bit combination into 5 bit
ciphertexts per input.  The library shares the first squaring's tensor,
rounding of the third component and key switching among the chains of an
input, and skips the test c = 0 (it enters no bit; the eq outputs are not
requested): 12,544 ciphertext squarings executed per step instead of 17,408.  Inputs are resident in HBM
(encrypted on the device) before the timed region.

Prints one JSON line with the metric (bridge conversions per second), the
executed ciphertext mul+relin per second, per-step p50/p99, the plain-vs-batched mul+relin
comparison at n = 16384 (one pair per call vs one batched call, for several
batch sizes), the headline step with the base conversions on the matrix cores and on the
vector ALU, the transform kernel alone at n = 4096 / 8192 / 16384, products
at n = 4096, 1024 products of mixed ring sizes (per-size calls vs one
multi-context call), depth-4 squaring chains (eager vs HIP graph), the
continuous-batching serving loop (Poisson arrivals, p50/p99), the roofline of the dominant kernel (timed live with HIP events on
the launch stream), and the CPU oracle timed on a bounded sample of the same
work.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ct mul+relin/s at n=16384 (batched vs plain GPU), bridge conversions/s, p50/p99"

# Peak figures (MI355X, gfx950): 256 CUs x 128 32-bit lanes at 2.4 GHz issue
# 78.6 T simple VALU lane-ops/s (the fp32 vector peak of 157.3 TFLOP/s counts an
# FMA as two); 32-bit integer multiplies (v_mul_lo_u32, v_mul_hi_u32,
# v_mad_u64_u32) issue at half that rate on gfx950 (measured by the calibration
# probe).
#
# Roofline of a 64-bit modular butterfly, algorithmic count: about 10
# multiply-class 32-bit operations (the 64 x 64-bit modular product built from
# 32-bit multiplies) and about 8 other 32-bit operations (the add, subtract and
# reduction), the multiplies at half rate: 10*2 + 8 = 28 issue slots, peak
# 78.6e12 / 28 = 2.81e12 butterflies/s.  This is the reported `peak`.
#
# Second figure, the model of the butterfly as implemented (Shoup product with a
# three-multiply quotient estimate): 9 multiplies (3 for the estimate, 3 each
# for the low halves of a*w and of quotient*q) and 18 full-rate slots of 64-bit
# adds, subtracts and the conditional subtraction: 36 slots, 2.18e12/s.
CUS, LANES_PER_CU, CLOCK = 256, 128, 2.4e9
VALU_LANE_OPS = CUS * LANES_PER_CU * CLOCK
SLOTS_PER_BFLY = 10 * 2 + 8
PEAK_BFLY = VALU_LANE_OPS / SLOTS_PER_BFLY
SLOTS_PER_BFLY_IMPL = 9 * 2 + 18
PEAK_BFLY_IMPL = VALU_LANE_OPS / SLOTS_PER_BFLY_IMPL
HBM_PEAK = 8.0e12

# HBM bytes per launch of the transform kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (scaled by 2.0 and 1.0, the factors a 1 GiB device copy and
# fill read back) averaged over the dispatches of one bridge group (one shared
# first-squaring launch of 32 ciphertexts and three launches of 512, the same
# mix as the timed run), together with the hash of the kernel sources they were
# taken on.  Reported only while the sources match.
TRAFFIC = {
    "relin_fused": {"bytes": 2371977.30 * 1024 * 2.0 + 1041152.00 * 1024 * 1.0, "src": "d37044ecbd169a83"},
    "square_tensor": {"bytes": 1374654.03 * 1024 * 2.0 + 3211323.16 * 1024 * 1.0, "src": "d37044ecbd169a83"},
}
KERNEL_SOURCES = ["paper_2204_12201_amd/csrc/kernels_ntt.hip", "paper_2204_12201_amd/csrc/ntt_core.hpp",
                  "paper_2204_12201_amd/csrc/modarith.hpp"]

# HBM bytes per 512-item launch of each kernel of a squaring (same counter
# passes and factors as TRAFFIC, taken with the matrix-core conversions), and
# the hash of the transform and conversion sources they were taken on.
PIPELINE = {
    "bytes_512": {"lift_q2p": (524397.9 * 2.0 + 1048576.1) * 1024,
                  "square_tensor": (1795473.2 * 2.0 + 4194382.5) * 1024,
                  "scale_round": (1574892.3 * 2.0 + 1572864.0) * 1024,
                  "relin_fused": (3098077.5 * 2.0 + 1359872.0) * 1024},
    "src": "2ec863cc6939fef6",
}
PIPELINE_SOURCES = KERNEL_SOURCES + ["paper_2204_12201_amd/csrc/kernels_conv.hip"]


def kernel_source_hash(files=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pipeline_bytes(ctx, squarings_per_s):
    """HBM bytes one squaring moves through lift, tensor, scale and key
    switching (counter figures of 512-item launches), against the 4 MiB of its
    input and output ciphertexts, while the sources match the counter run."""
    if kernel_source_hash(PIPELINE_SOURCES) != PIPELINE["src"]:
        return None
    per = {k: v / 512 for k, v in PIPELINE["bytes_512"].items()}
    total = sum(per.values())
    ct_bytes = 2 * ctx.k * ctx.n * 8
    return {"bytes_per_squaring": total, "per_kernel": per, "min_bytes_per_squaring": 2 * ct_bytes,
            "ratio_to_min": total / (2 * ct_bytes), "tb_per_s_at_measured_rate": total * squarings_per_s / 1e12}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(math.ceil(p / 100 * len(xs))) - 1))
    return xs[i]


def transform_rows(ctx, name: str):
    """Transform rows one item (one squaring) sends through kernel `name`."""
    k, K = ctx.k, ctx.k + ctx.aux_primes
    return {"mul_tensor": 7 * K, "square_tensor": 5 * K,
            "relin_fused": k * k + 2 * k}.get(name)


def same_launch_mix(args) -> bool:
    """The library groups the bridge chains by 32 inputs at n = 16384 (546
    products of workspace / p = 17): per group one shared first-squaring
    launch of 32 items and three launches of 512 (16 chains per input).  The counter runs use one
    group, so their per-dispatch averages hold for any whole number of groups."""
    return args.inputs % 32 == 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inputs", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip every leg after the headline bridge")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs after the headline (conv, powers, plain, autotune, ntt, mfma, c0, "
                         "mixed, chain, imputation, serving) or all")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival window of the serving leg (200 requests/s)")
    ap.add_argument("--saturate-rate", type=float, default=1000.0,
                    help="offered rate of the second serving run, above the loop's capacity")
    ap.add_argument("--saturate-seconds", type=float, default=10.0,
                    help="arrival window of the second serving run")
    ap.add_argument("--no-calib", action="store_true",
                    help="skip the VALU / copy calibration probe (M0) run beside the roofline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (HBM counter scale)")
    ap.add_argument("--conv", choices=("mfma", "valu"), default="mfma",
                    help="engine of the base conversions in the headline run (the library's default is mfma)")
    ap.add_argument("--cpu-oracle-only", type=float, default=None, metavar="SECONDS",
                    help="time only the CPU oracle (no GPU use) and print its JSON record")
    args = ap.parse_args()
    if args.cpu_oracle_only is not None:
        from paper_2204_12201_amd import inputs
        print(json.dumps(cpu_oracle_rate(inputs, args.cpu_oracle_only)))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the work shards by ciphertext across GPUs; this benchmark runs one)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_12201_amd import fhe, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs, t, nbits = cfg["n"], cfg["q"], cfg["t"], cfg["nbits"]
    count = args.inputs
    ctx = fhe.Context(n, qs, t, "coeff")
    ctx.set_conv_method(args.conv == "mfma")
    km = inputs.key_material(n, qs, 0)
    pk, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    xs = inputs.bridge_values(t, count, 0)
    pts = np.zeros((count, n), dtype=np.uint64)
    pts[:, 0] = xs
    r = inputs.encryption_randomness(n, count, 0)
    x_ct = ctx.encrypt(pk, pts, r["u"], r["e"])
    squarings = int(math.log2(t - 1))
    mul_per_step = count * (1 + (t - 1) * (squarings - 1))  # products executed per step
    print(f"[bench] setup done: {count} inputs, {mul_per_step} mul_relin per step", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        bits = ctx.bridge_to_bits(rlk, x_ct, nbits)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # correctness of the last output: decrypted bits equal the plain bits
    if args.warmup:
        dec = ctx.decrypt(km["s"], bits.reshape(-1, 2, len(qs), n)).reshape(count, nbits, n)[:, :, 0]
        want = (xs[:, None].astype(np.int64) >> np.arange(nbits)) & 1
        assert (dec.astype(np.int64) == want).all(), "bridge output does not decrypt to the bits of x"

    ctx.reset_kernel_stats()
    ctx.set_timing(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        evs[s][0].record(stream)
        bits = ctx.bridge_to_bits(rlk, x_ct, nbits)
        evs[s][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    step_ms = [a.elapsed_time(b) for a, b in evs]
    stats = ctx.kernel_stats()
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    conv_per_s = count * args.steps / elapsed
    value = conv_per_s

    # dominant kernel and its roofline: algorithmic butterflies over the timed
    # region (every executed product runs each transform kernel once per item)
    # divided by the kernel's summed launch time.
    kern = {k: v for k, v in stats.items() if v[1] > 0}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_launches = kern[dom]
    rows = transform_rows(ctx, dom)
    roofline = None
    if rows is not None:
        work_total = rows * (n // 2) * int(math.log2(n)) * mul_per_step * args.steps
        per_launch = work_total / dom_launches
        avg_s = dom_ms / 1e3 / dom_launches
        achieved = per_launch / avg_s
        tr = TRAFFIC.get(dom)
        traffic = tr["bytes"] if tr and tr["src"] == kernel_source_hash() and same_launch_mix(args) else None
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_BFLY / 1e12,
                    "unit": "Tbutterfly/s", "frac": achieved / PEAK_BFLY,
                    "peak_basis": "10 multiply-class (half rate) + 8 other 32-bit VALU ops per butterfly "
                                  "at 78.6 T lane-ops/s",
                    "peak_impl_model": PEAK_BFLY_IMPL / 1e12, "frac_impl_model": achieved / PEAK_BFLY_IMPL,
                    "traffic": traffic,
                    "traffic_unit": "bytes per launch",
                    "avg_launch_ms": avg_s * 1e3, "launches": dom_launches,
                    "butterflies_per_launch": per_launch}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "conversions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "bridge_p17_n16384_k8x55bit_256inputs", "n": n, "k": len(qs),
                   "q_bits": sum(int(q).bit_length() for q in qs), "p": t, "inputs": count,
                   "mul_relin_per_step": mul_per_step, "aux_primes": ctx.aux_primes,
                   "conversions_engine": args.conv,
                   "parallelism": "single-gpu"},
        "executed_mul_relin_per_s": mul_per_step * args.steps / elapsed,
        "step_p50_ms": percentile(step_ms, 50),
        "step_p99_ms": percentile(step_ms, 99),
        "kernel_ms": {k: round(v[0], 3) for k, v in kern.items()},
        "roofline": roofline,
        "pipeline_bytes": pipeline_bytes(ctx, mul_per_step * args.steps / elapsed) if args.conv == "mfma" else None,
    }

    legs = set(args.legs.split(",")) if args.legs != "all" else {
        "conv", "powers", "plain", "autotune", "ntt", "mfma", "c0", "mixed", "chain", "imputation", "serving"}
    if args.no_plain:
        legs = set()

    if "conv" in legs:
        out["conv_engines"] = conv_engine_leg(ctx, rlk, x_ct, nbits, torch)
        ctx.set_conv_method(args.conv == "mfma")
        print("[bench] conversion engines done", file=sys.stderr, flush=True)
    # the same bits from the powers of x (another circuit: t - 2 products per
    # input), on the same inputs and key; reported beside the headline
    if "powers" in legs:
        out["bridge_power_basis"] = power_basis_leg(ctx, rlk, x_ct, xs, km, nbits, args.steps, torch)
        print("[bench] power-basis bridge done", file=sys.stderr, flush=True)
    if "plain" in legs:
        out["plain_vs_batched"] = plain_vs_batched(ctx_factory=lambda: fhe.Context(
            n, qs, 65537, "slots"), fhe=fhe, inputs=inputs, torch=torch)
        print("[bench] plain vs batched done", file=sys.stderr, flush=True)

    if "autotune" in legs:
        out["autotune"] = autotune_leg(fhe, inputs, torch)
        print("[bench] autotune done", file=sys.stderr, flush=True)
    if "ntt" in legs:
        out["ntt_rows"] = ntt_rows_leg(fhe, inputs, torch)
    if "mfma" in legs:
        out["mfma_pass0"] = mfma_pass0_leg(fhe, inputs, torch)
        print("[bench] matrix-core pass comparison done", file=sys.stderr, flush=True)
    if "c0" in legs:
        out["c0_n4096"] = c0_leg(fhe, inputs, torch)
        print("[bench] transform rows and n=4096 products done", file=sys.stderr, flush=True)
    if "mixed" in legs:
        out["mixed_sizes"] = mixed_leg(fhe, inputs, torch)
    if "chain" in legs:
        out["square_chain_n16384"] = chain_leg(fhe, inputs, torch)
        print("[bench] mixed sizes and squaring chains done", file=sys.stderr, flush=True)
    if "imputation" in legs:
        out["imputation"] = imputation_leg(fhe, inputs, torch)
        print("[bench] imputation-shaped stages done", file=sys.stderr, flush=True)
    if "serving" in legs:
        setup = ServingSetup(fhe, inputs, torch)
        out["serving"] = serving_leg(fhe, inputs, torch, setup, seconds=args.serve_seconds)
        print("[bench] serving loop done", file=sys.stderr, flush=True)
        # offered load above capacity: queues build, batches fill
        out["serving_saturated"] = serving_leg(fhe, inputs, torch, setup, seconds=args.saturate_seconds,
                                               rate=args.saturate_rate, seed=8)
        print("[bench] saturated serving loop done", file=sys.stderr, flush=True)

    if not args.no_calib:
        cal = calibration()
        if cal:
            out["calibration"] = cal
            if "bfly_peak_calibrated" in cal and roofline.get("achieved"):
                roofline["frac_of_calibrated_issue"] = roofline["achieved"] * 1e12 / cal["bfly_peak_calibrated"]
        print("[bench] calibration done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inputs)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    print(json.dumps(out))


def plain_vs_batched(ctx_factory, fhe, inputs, torch, B=256, single_calls=200,
                     sweep=(1, 16, 64, 256, 341)):
    """n = 16384, eight 55-bit primes, t = 65537: for every batch size Bs in
    `sweep`, Bs single-pair calls against one call with count = Bs on the same
    ciphertexts; p50/p99 of single-call latency; per-kernel time of the
    batched call at B."""
    ctx = ctx_factory()
    n, qs = ctx.n, ctx.q
    km = inputs.key_material(n, qs, 4)
    pk, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    bmax = max(max(sweep), B)
    a = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, bmax, 4, "a"), "cuda")
    b = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, bmax, 4, "b"), "cuda")
    out = ctx.empty_ct(bmax)
    stream = torch.cuda.current_stream()
    # warm up both paths
    for _ in range(3):
        ctx.mul_relin(rlk, a[:B], b[:B], out=out[:B])
        ctx.mul_relin(rlk, a[:1], b[:1], out=out[:1])
    torch.cuda.synchronize()

    def rates(bs, reps):
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.mul_relin(rlk, a[:bs], b[:bs], out=out[:bs])
        torch.cuda.synchronize()
        batched = bs * reps / (time.perf_counter() - t0)
        views = [(a[j:j + 1], b[j:j + 1], out[j:j + 1]) for j in range(bs)]
        t0 = time.perf_counter()
        for x, y, o in views:
            ctx.mul_relin(rlk, x, y, out=o)
        torch.cuda.synchronize()
        return batched, bs / (time.perf_counter() - t0)

    rows = []
    for bs in sweep:
        bt, pl = rates(bs, 3 if bs >= 64 else 20)
        rows.append({"B": bs, "batched_mul_relin_per_s": bt, "plain_mul_relin_per_s": pl})
    batched, plain = rates(B, 3)
    ctx.reset_kernel_stats()
    ctx.set_timing(True)
    ctx.mul_relin(rlk, a[:B], b[:B], out=out[:B])
    torch.cuda.synchronize()
    ctx.set_timing(False)
    kern = {k: round(v[0], 3) for k, v in ctx.kernel_stats().items() if v[1] > 0}
    views = [(a[j:j + 1], b[j:j + 1], out[j:j + 1]) for j in range(B)]
    lat = []
    for j in range(single_calls):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        x, y, o = views[j % B]
        e0.record(stream)
        ctx.mul_relin(rlk, x, y, out=o)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    lat_ms = [e0.elapsed_time(e1) for e0, e1 in lat]
    return {"n": n, "k": len(qs), "t": 65537, "B": B, "batched_mul_relin_per_s": batched,
            "plain_mul_relin_per_s": plain, "batched_over_plain": batched / plain,
            "single_call_p50_ms": percentile(lat_ms, 50), "single_call_p99_ms": percentile(lat_ms, 99),
            "batched_kernel_ms": kern, "sweep": rows}


def autotune_leg(fhe, inputs, torch, sizes=(1, 4, 16, 256), reps=5):
    """fhe_autotune_mul_relin on the n = 16384, t = 65537 products: per batch
    size, the rate with the default launch shape, the shape the autotuner
    keeps (chunk cap, fused or unfused transforms) and the rate with it (each
    size on a fresh context)."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs = cfg["n"], cfg["q"]
    bmax = max(sizes)
    a = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, bmax, 5, "a"), "cuda")
    b = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, bmax, 5, "b"), "cuda")
    res = []
    for bs in sizes:
        ctx = fhe.Context(n, qs, 65537, "slots")
        km = inputs.key_material(n, qs, 5)
        _, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
        out = ctx.empty_ct(bs)

        def rate():
            ctx.mul_relin(rlk, a[:bs], b[:bs], out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.mul_relin(rlk, a[:bs], b[:bs], out=out)
            torch.cuda.synchronize()
            return bs * reps / (time.perf_counter() - t0)

        before = rate()
        chunk, fused = ctx.autotune_mul_relin(rlk, a[:bs], b[:bs])
        after = rate()
        res.append({"B": bs, "default_mul_relin_per_s": before, "chunk": chunk, "fused": fused,
                    "tuned_mul_relin_per_s": after})
        del ctx
    return res


def power_basis_leg(ctx, rlk, x_ct, xs, km, nbits, steps, torch):
    """The bits of the headline's inputs from the shared powers of x (t - 2
    products per input, another circuit than the per-test chains), timed over
    `steps` calls after one untimed call; the decryptions are checked."""
    n, k, t = ctx.n, ctx.k, ctx.t
    count = len(xs)
    ctx.bridge_to_bits_powers(rlk, x_ct, nbits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pbits = ctx.bridge_to_bits_powers(rlk, x_ct, nbits)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pdec = ctx.decrypt(km["s"], pbits.reshape(-1, 2, k, n)).reshape(count, nbits, n)[:, :, 0]
    want = (xs[:, None].astype(np.int64) >> np.arange(nbits)) & 1
    return {"conversions_per_s": count * steps / el, "ms_per_step": el * 1e3 / steps,
            "mul_relin_per_conversion": t - 2, "decrypts_to_bits": bool((pdec.astype(np.int64) == want).all())}


def conv_engine_leg(ctx, rlk, x_ct, nbits, torch, steps=2, rounds=2):
    """The headline step with the base conversions (lift, scale-and-round, the
    chains' first rounding) on the matrix cores and on the vector ALU, the two
    engines alternating over `rounds` rounds of `steps` steps: rate, kernel
    time per step by kind, and whether the bits are the same words."""
    el = {True: 0.0, False: 0.0}
    ms = {True: {}, False: {}}
    bits = {}
    for _ in range(rounds):
        for mfma in (True, False):
            ctx.set_conv_method(mfma)
            bits[mfma] = ctx.bridge_to_bits(rlk, x_ct, nbits)  # warm-up, kept for the comparison
            torch.cuda.synchronize()
            ctx.reset_kernel_stats()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.bridge_to_bits(rlk, x_ct, nbits)
            torch.cuda.synchronize()
            el[mfma] += time.perf_counter() - t0
            ctx.set_timing(False)
            for kind, (t, cnt) in ctx.kernel_stats().items():
                if cnt:
                    ms[mfma][kind] = ms[mfma].get(kind, 0.0) + t
    ctx.set_conv_method(True)
    res = {}
    for mfma in (True, False):
        res["mfma" if mfma else "valu"] = {
            "conversions_per_s": x_ct.shape[0] * steps * rounds / el[mfma],
            "kernel_ms_per_step": {kind: round(t / (steps * rounds), 3) for kind, t in ms[mfma].items()}}
    res["words_equal"] = bool(torch.equal(bits[True], bits[False]))
    return res


def ntt_rows_leg(fhe, inputs, torch, reps=4):
    """The transform kernel alone: forward then inverse transform of a batch of
    rows per launch (uniform residues) with the configured primes, at two batch
    sizes: 128 MiB (4096 / 2048 / 1024 rows at n = 4096 / 8192 / 16384), which
    the 256 MB last-level cache largely holds between the two launches, and
    512 MiB, which it does not (every row comes from and goes to HBM; each
    resident workgroup runs 16 rows).  Rows/s, butterflies/s and algorithmic
    bytes (each row read and written once, 16 bytes per coefficient) against
    the ALU and HBM peaks."""
    res = []
    for mib in (128, 512):
        for key in ("bfv_n4096", "bfv_n8192", "bfv_n16384"):
            cfg = inputs.CONFIGS[key]
            n, qs = cfg["n"], cfg["q"]
            k = len(qs)
            ctx = fhe.Context(n, qs, cfg["t"], cfg["encoding"])
            count = -(-(mib * 131072 // n) // k)
            polys = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 6, "ntt")[:, 0], "cuda")
            ctx.ntt(polys)
            ctx.ntt(polys, inverse=True)
            torch.cuda.synchronize()
            ctx.reset_kernel_stats()
            ctx.set_timing(True)
            for _ in range(reps):
                ctx.ntt(polys)
                ctx.ntt(polys, inverse=True)
            torch.cuda.synchronize()
            ctx.set_timing(False)
            ms, launches = ctx.kernel_stats()["ntt_rows"]
            rows = count * k * launches
            rows_s = rows / (ms / 1e3)
            bfly_s = rows_s * (n // 2) * int(math.log2(n))
            bytes_s = rows_s * n * 16
            res.append({"n": n, "batch_mib": mib, "rows_per_launch": count * k, "rows_per_s": rows_s,
                        "tbutterfly_per_s": bfly_s / 1e12, "alu_frac": bfly_s / PEAK_BFLY,
                        "alu_frac_impl_model": bfly_s / PEAK_BFLY_IMPL,
                        "gb_per_s": bytes_s / 1e9, "hbm_frac": bytes_s / HBM_PEAK})
            del polys
    return res


def mfma_pass0_leg(fhe, inputs, torch, launches=10):
    """The first radix-16 pass of the forward transform (butterfly levels
    0..3) at n = 16384 with the eight 55-bit primes, on the vector ALU and as
    an exact int8 matrix product on the matrix cores (fhe_ntt_pass0; the
    words are equal): once per launch over 64 MiB of rows (held by the 256 MB
    last-level cache between launches) and 512 MiB (from and to HBM), and 16
    times per launch on register-resident data over 512 MiB (the compute rate
    of the pass with its memory traffic amortised).  Per-launch time from HIP
    events on the launch stream; butterflies per second count the pass's
    4 n/2 butterflies per row and pass for both methods."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs = cfg["n"], cfg["q"]
    k = len(qs)
    ctx = fhe.Context(n, qs, cfg["t"], cfg["encoding"])
    res = []
    for mib, reps in ((64, 1), (512, 1), (512, 16)):
        count = mib * 131072 // n // k
        polys = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 9, "p0")[:, 0], "cuda")
        row = {"batch_mib": mib, "passes_per_launch": reps, "rows_per_launch": count * k}
        for name, mfma in (("valu", False), ("mfma", True)):
            ctx.ntt_pass0(polys, mfma, reps)
            torch.cuda.synchronize()
            ctx.reset_kernel_stats()
            ctx.set_timing(True)
            for _ in range(launches):
                ctx.ntt_pass0(polys, mfma, reps)
            torch.cuda.synchronize()
            ctx.set_timing(False)
            ms, nl = ctx.kernel_stats()["pass0_mfma" if mfma else "pass0_valu"]
            per = ms / nl
            rows_s = count * k / (per / 1e3)
            row[name] = {"ms_per_launch": per, "rows_per_s": rows_s,
                         "tbutterfly_per_s": rows_s * reps * 2 * n / 1e12, "gb_per_s": rows_s * n * 16 / 1e9}
        row["mfma_over_valu_time"] = row["mfma"]["ms_per_launch"] / row["valu"]["ms_per_launch"]
        res.append(row)
        del polys
    return res


def c0_leg(fhe, inputs, torch, reps=5):
    """n = 4096, three 36-bit primes, t = 65537: 64 products of uniform
    ciphertexts per call (the plain BFV workload's shape)."""
    cfg = inputs.CONFIGS["bfv_n4096"]
    n, qs, count = cfg["n"], cfg["q"], cfg["count"]
    ctx = fhe.Context(n, qs, cfg["t"], cfg["encoding"])
    km = inputs.key_material(n, qs, 0)
    pk, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    a = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 3, "a"), "cuda")
    b = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 3, "b"), "cuda")
    out = ctx.empty_ct(count)
    ctx.mul_relin(rlk, a, b, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.mul_relin(rlk, a, b, out=out)
    torch.cuda.synchronize()
    return {"n": n, "k": len(qs), "t": cfg["t"], "count": count,
            "mul_relin_per_s": count * reps / (time.perf_counter() - t0)}


def mixed_leg(fhe, inputs, torch, reps=4):
    """1024 ciphertext pairs of mixed ring sizes (342 at n=4096 with three 36-bit
    primes, 341 at n=8192 with five 43-bit, 341 at n=16384 with eight 55-bit;
    t = 65537): three per-size calls one after the other against one
    fhe_mul_relin_multi call whose parts overlap on the device, with each
    part's key switching on its own stream and with the key switching of all
    parts in one persistent launch (a (ciphertext, limb, ring size) work
    queue); words checked equal between the three."""
    parts = []
    for key, count in (("bfv_n4096", 342), ("bfv_n8192", 341), ("bfv_n16384", 341)):
        cfg = inputs.CONFIGS[key]
        n, qs = cfg["n"], cfg["q"]
        ctx = fhe.Context(n, qs, cfg["t"], cfg["encoding"])
        km = inputs.key_material(n, qs, 5)
        _, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
        a = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 5, "a"), "cuda")
        b = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 5, "b"), "cuda")
        parts.append((ctx, rlk, a, b, ctx.empty_ct(count)))
    total = sum(p[2].shape[0] for p in parts)
    lead = parts[0][0]
    for ctx, rlk, a, b, out in parts:
        ctx.mul_relin(rlk, a, b, out=out)
    torch.cuda.synchronize()
    want = [fhe.to_numpy_u64(p[4]) for p in parts]
    res = {"pairs": {"4096": 342, "8192": 341, "16384": 341}, "t": 65537}

    def sequential():
        for ctx, rlk, a, b, out in parts:
            ctx.mul_relin(rlk, a, b, out=out)

    def multi(persistent):
        def go():
            lead.set_multi_persistent(persistent)
            fhe.mul_relin_multi(parts)
        return go

    modes = (("sequential", sequential), ("multi_streams", multi(False)), ("multi_persistent", multi(True)))
    for name, fn in modes[1:]:  # warm-up, and the words of each mode
        for p in parts:
            p[4].zero_()
        fn()
        torch.cuda.synchronize()
        res[name + "_words_equal_sequential"] = all(
            (fhe.to_numpy_u64(p[4]) == w).all() for p, w in zip(parts, want))
    # the modes interleaved twice; the better pass of each is reported
    best = {}
    for _ in range(2):
        for name, fn in modes:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            best[name] = max(best.get(name, 0.0), total * reps / (time.perf_counter() - t0))
    for name, _ in modes:
        res[name + "_mul_relin_per_s"] = best[name]
    # the autotuner's choice between the two multi modes, kept in the leading context
    res["autotuned_persistent"] = fhe.autotune_mul_relin_multi(parts)
    res["multi_mul_relin_per_s"] = res["multi_persistent_mul_relin_per_s" if res["autotuned_persistent"]
                                       else "multi_streams_mul_relin_per_s"]
    lead.set_multi_persistent(False)
    return res


def chain_leg(fhe, inputs, torch, count=64, depth=4, reps=3):
    """Depth-4 squaring chains at n = 16384 (eight 55-bit primes, t = 65537) on
    64 ciphertexts: four eager mul_relin calls against the replayed HIP graph of
    fhe_square_chain."""
    cfg = inputs.CONFIGS["bfv_n16384"]
    n, qs = cfg["n"], cfg["q"]
    ctx = fhe.Context(n, qs, cfg["t"], cfg["encoding"])
    km = inputs.key_material(n, qs, 6)
    _, rlk = ctx.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    x = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, count, 6, "x"), "cuda")
    res = {}
    for name, graph in (("eager", False), ("graph", True)):
        ctx.square_chain(rlk, x, depth, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.square_chain(rlk, x, depth, graph=graph)
        torch.cuda.synchronize()
        res[f"{name}_mul_relin_per_s"] = count * depth * reps / (time.perf_counter() - t0)
    res.update({"n": n, "count": count, "depth": depth})
    return res


def imputation_leg(fhe, inputs, torch, reps=3, seed=11, subset=32):
    """The imputation-shaped workload (the paper's genotype-imputation case
    study), both stages on synthetic data.  Modular: n = 16384, eight 55-bit
    primes, t = 65537 (8192 samples per ciphertext in slots), 500 targets x 3
    classes = 1500 outputs, each an integer-weighted sum (weights uniform in
    [-8, 8]) of 24 encrypted tag genotypes (uniform words stand in for their
    encryptions), as one fhe_weighted_sum call; algorithmic HBM bytes = the 24
    inputs read once plus the 1500 outputs written.  Bit-level: per-class
    scores quantized to [0, 17) for a seeded subset of samples, encrypted at
    p = 17 (coefficient encoding), bridged to 5 bits each and reduced to a
    one-hot argmax over the 3 classes (fhe_argmax); decryptions checked."""
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs = cfg["n"], cfg["q"]
    nin, ntarget, ncls = 24, 500, 3
    ctx = fhe.Context(n, qs, 65537, "slots")
    g = fhe.from_numpy_u64(inputs.uniform_ciphertexts(n, qs, nin, seed, "g"), "cuda")
    W = np.random.default_rng(seed).integers(-8, 9, size=(ntarget * ncls, nin)).astype(np.int32)
    out = ctx.weighted_sum(g, W)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.weighted_sum(g, W, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t_ms = sorted(ms)[len(ms) // 2]
    ct_bytes = 2 * len(qs) * n * 8
    hbm = (nin + ntarget * ncls) * ct_bytes
    res = {"modular": {"n": n, "k": len(qs), "inputs": nin, "outputs": ntarget * ncls, "ms_per_call": t_ms,
                       "outputs_per_s": ntarget * ncls / (t_ms / 1e3), "gb_per_s": hbm / (t_ms / 1e3) / 1e9,
                       "hbm_frac": hbm / (t_ms / 1e3) / HBM_PEAK}}
    del out
    # bit-level stage on a subset: bridge the class scores, then argmax
    ctxb = fhe.Context(n, qs, cfg["t"], "coeff")
    km = inputs.key_material(n, qs, seed)
    pk, rlk = ctxb.keygen(km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    scores = inputs.bridge_values(cfg["t"], ncls * subset, seed).reshape(ncls, subset)
    pts = np.zeros((ncls * subset, n), dtype=np.uint64)
    pts[:, 0] = scores.reshape(-1)
    r = inputs.encryption_randomness(n, ncls * subset, seed)
    x = ctxb.encrypt(pk, pts, r["u"], r["e"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bits = ctxb.bridge_to_bits(rlk, x, cfg["nbits"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    oh = ctxb.argmax(rlk, bits.reshape(ncls, subset, cfg["nbits"], 2, len(qs), n))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dec = ctxb.decrypt(km["s"], oh.reshape(ncls * subset, 2, len(qs), n)).reshape(ncls, subset, n)
    best = [max(range(ncls), key=lambda c: (int(scores[c, j]), -c)) for j in range(subset)]
    ok = all(int(dec[c, j, 0]) == int(best[j] == c) for c in range(ncls) for j in range(subset))
    res["bridge_argmax"] = {"samples": subset, "classes": ncls, "bridge_ms": (t1 - t0) * 1e3,
                            "argmax_ms": (t2 - t1) * 1e3, "samples_per_s": subset / (t2 - t0),
                            "argmax_mul_relin": ncls * (ncls - 1) // 2 * (2 * cfg["nbits"] - 1) + ncls,
                            "decrypts_one_hot": ok}
    # signed casts of the same encrypted scores: SecureMod -> SecureInt (bridge,
    # constant adder, MUX) and back (linear)
    xs = x[:subset]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ybits = ctxb.mod_to_int(rlk, xs, cfg["nbits"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    back = ctxb.int_to_mod(ybits)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dec = ctxb.decrypt(km["s"], back)
    res["signed_casts"] = {"inputs": subset, "mod_to_int_ms": (t1 - t0) * 1e3, "int_to_mod_ms": (t2 - t1) * 1e3,
                           "round_trip_ok": bool((dec[:, 0] == scores.reshape(-1)[:subset]).all())}
    return res


class ServingSetup:
    """Contexts, resident keys and request pools of the serving legs: products
    at n = 8192 (t = 65537); p = 17 bridge conversions at n = 16384; imputation
    queries: one target's 3 class scores as weighted sums of 24 resident
    genotype ciphertexts (n = 16384, t = 65537), then 3 class scores at
    p = 17 (n = 16384, their own key) bridged to 5 bits and reduced to the
    one-hot argmax."""

    def __init__(self, fhe, inputs, torch, seed=7, pool=64):
        c8 = inputs.CONFIGS["bfv_n8192"]
        self.ctx8 = fhe.Context(c8["n"], c8["q"], c8["t"], "slots")
        km8 = inputs.key_material(c8["n"], c8["q"], seed)
        _, self.rlk8 = self.ctx8.keygen(km8["s"], km8["pk_a"], km8["pk_e"], km8["rlk_a"], km8["rlk_e"])
        cb = inputs.CONFIGS["bridge_n16384"]
        self.nbits = cb["nbits"]
        self.ctxb = fhe.Context(cb["n"], cb["q"], cb["t"], "coeff")
        kmb = inputs.key_material(cb["n"], cb["q"], seed)
        pkb, self.rlkb = self.ctxb.keygen(kmb["s"], kmb["pk_a"], kmb["pk_e"], kmb["rlk_a"], kmb["rlk_e"])
        self.pool = pool
        self.a = fhe.from_numpy_u64(inputs.uniform_ciphertexts(c8["n"], c8["q"], pool, seed, "a"), "cuda")
        self.b = fhe.from_numpy_u64(inputs.uniform_ciphertexts(c8["n"], c8["q"], pool, seed, "b"), "cuda")
        xs = inputs.bridge_values(cb["t"], pool, seed)
        pts = np.zeros((pool, cb["n"]), dtype=np.uint64)
        pts[:, 0] = xs
        r = inputs.encryption_randomness(cb["n"], pool, seed)
        self.xb = self.ctxb.encrypt(pkb, pts, r["u"], r["e"])
        self.ctxi = fhe.Context(cb["n"], cb["q"], 65537, "slots")
        self.gi = fhe.from_numpy_u64(inputs.uniform_ciphertexts(cb["n"], cb["q"], 24, seed, "g"), "cuda")
        self.wq = np.random.default_rng(seed + 1).integers(-8, 9, size=(pool, 3, 24)).astype(np.int32)
        self.ctx2 = fhe.Context(cb["n"], cb["q"], cb["t"], "coeff")
        km2 = inputs.key_material(cb["n"], cb["q"], seed + 2)
        pk2, self.rlk2 = self.ctx2.keygen(km2["s"], km2["pk_a"], km2["pk_e"], km2["rlk_a"], km2["rlk_e"])
        sv = inputs.bridge_values(cb["t"], 3 * pool, seed + 2)
        pts = np.zeros((3 * pool, cb["n"]), dtype=np.uint64)
        pts[:, 0] = sv
        r = inputs.encryption_randomness(cb["n"], 3 * pool, seed + 2)
        self.sc = self.ctx2.encrypt(pk2, pts, r["u"], r["e"]).view(pool, 3, 2, len(cb["q"]), cb["n"])
        # warm the lanes (workspaces, kernels)
        self.ctx8.mul_relin(self.rlk8, self.a[:64], self.b[:64])
        self.ctxb.bridge_to_bits(self.rlkb, self.xb[:8], self.nbits)
        self.ctxi.weighted_sum(self.gi, self.wq[:16].reshape(-1, 24))
        bits = self.ctx2.bridge_to_bits(self.rlk2, self.sc[:4].reshape(12, 2, len(cb["q"]), cb["n"]), self.nbits)
        self.ctx2.argmax(self.rlk2, bits.view(4, 3, self.nbits, 2, len(cb["q"]), cb["n"]).transpose(0, 1).contiguous())
        torch.cuda.synchronize()


def serving_leg(fhe, inputs, torch, setup, seconds=60.0, rate=200.0, seed=7):
    """Continuous batching (paper_2204_12201_amd/serving.py): Poisson arrivals at
    `rate` requests/s for `seconds`: 50 % products at n = 8192 (t = 65537), 30 %
    p = 17 bridge conversions at n = 16384, 20 % imputation queries (weighted
    sums, bridge of the 3 class scores, one-hot argmax); keys and genotype
    ciphertexts resident, 32 GiB in-flight budget.  Throughput and p50/p99
    latency from arrival to completion, per kind and overall; the loop runs
    until every arrived request is done (wall_s includes that drain)."""
    from paper_2204_12201_amd import serving
    S = setup
    rng = np.random.default_rng(seed)
    t, reqs, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        u, j = rng.random(), i % S.pool
        if u < 0.5:
            reqs.append(serving.Request(rid=i, kind="mul_n8192", arrival=t, x=S.a[j:j + 1], y=S.b[j:j + 1]))
        elif u < 0.8:
            reqs.append(serving.Request(rid=i, kind="bridge_n16384", arrival=t, x=S.xb[j:j + 1]))
        else:
            reqs.append(serving.Request(rid=i, kind="impute_n16384", arrival=t, w=S.wq[j], s=S.sc[j]))
        i += 1
    srv = serving.Server([serving.Lane("mul_n8192", S.ctx8, S.rlk8, "mul", max_batch=256),
                          serving.Lane("bridge_n16384", S.ctxb, S.rlkb, "bridge", max_batch=32, nbits=S.nbits),
                          serving.Lane("impute_n16384", S.ctxi, None, "impute", max_batch=64, shared=S.gi, rows=3,
                                       nbits=S.nbits, ctx2=S.ctx2, rlk2=S.rlk2)],
                         budget_bytes=32 << 30)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    el = time.perf_counter() - t0
    out = serving.summary(done, el)
    out.update({"offered_rate_req_per_s": rate, "seconds": seconds, "wall_s": el,
                "peak_in_flight_gib": srv.peak_bytes / 2**30, "max_concurrent_lanes": srv.max_concurrent})
    return out


def calibration():
    """M0: the calibration probe (paper_2204_12201_amd/calib/valu_calib, a
    child process) measures the issue rates of v_add_u32 and of the 32-bit
    integer multiplies, and the device copy rate.  From them, the butterfly
    peak of the same 36-slot model at the measured rates (9 multiplies at the
    slowest multiply rate, 18 other slots at the add rate)."""
    import re
    import subprocess
    exe = os.path.join(ROOT, "paper_2204_12201_amd", "calib", "valu_calib")
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    except (subprocess.TimeoutExpired, OSError):
        return None
    if r.returncode != 0:
        return None
    vals = {}
    for line in r.stdout.splitlines():
        m = re.match(r"(v_\w+)\s+([0-9.]+)\s+T lane-instr/s", line.strip())
        if m:
            vals[m.group(1)] = float(m.group(2))
        m = re.match(r"copy kernel\s+([0-9.]+)\s+GB/s", line.strip())
        if m:
            vals["copy"] = float(m.group(1))
    out = {"valu_add_tlane_per_s": vals.get("v_add_u32"), "mul_lo_tlane_per_s": vals.get("v_mul_lo_u32"),
           "mul_hi_tlane_per_s": vals.get("v_mul_hi_u32"), "mad_u64_tlane_per_s": vals.get("v_mad_u64_u32"),
           "copy_gb_per_s": vals.get("copy")}
    muls = [v for v in (out["mul_lo_tlane_per_s"], out["mul_hi_tlane_per_s"], out["mad_u64_tlane_per_s"]) if v]
    if muls and out["valu_add_tlane_per_s"]:
        t = 9 / (min(muls) * 1e12) + 18 / (out["valu_add_tlane_per_s"] * 1e12)
        out["bfly_peak_calibrated"] = 1.0 / t
    return out


def cpu_baseline(inputs, seconds=15.0):
    """The oracle on the host: one bridge chain (4 squarings with relinearization)
    at n = 16384, eight 55-bit primes, p = 17, repeated for about `seconds`,
    with every host thread the oracle's OpenMP loops get; then the same in a
    child process limited to one thread (OMP_NUM_THREADS=1)."""
    import subprocess
    res = cpu_oracle_rate(inputs, seconds)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-oracle-only", str(seconds)],
                           capture_output=True, text=True, timeout=seconds * 10 + 120, env=env)
        one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, OSError, ValueError, IndexError):
        one = None
    if one:
        res["one_thread"] = {k: one[k] for k in ("value", "unit", "cores", "sample", "mul_relin_per_s", "seconds")}
    return res


def cpu_oracle_rate(inputs, seconds=15.0):
    from oracle import bfv, clib
    cfg = inputs.CONFIGS["bridge_n16384"]
    n, qs, t = cfg["n"], cfg["q"], cfg["t"]
    P = bfv.Params(n, qs, t, "coeff")
    km = inputs.key_material(n, qs, 0)
    pk, rlk = bfv.keygen(P, km["s"], km["pk_a"], km["pk_e"], km["rlk_a"], km["rlk_e"])
    r = inputs.encryption_randomness(n, 1, 0)
    pt = np.zeros(n, dtype=np.uint64)
    pt[0] = 5
    ct = bfv.encrypt(P, pk, pt, r["u"][0], r["e"][0])
    done = 0
    t0 = time.perf_counter()
    y = bfv.sub_plain(P, ct, 3)
    while time.perf_counter() - t0 < seconds or done < 2:
        y = bfv.mul_relin(P, y, y, rlk)
        done += 1
    el = time.perf_counter() - t0
    # the oracle computes every chain on its own: 68 squarings per conversion
    return {"value": done / el / (17 * 4), "unit": "conversions/s", "cores": clib.max_threads(),
            "kind": "oracle",
            "sample": f"{done} squarings with relinearization of one bridge chain at n=16384, k=8 "
                      f"(55-bit primes), p=17 on the host CPU ({os.cpu_count()} logical CPUs visible), "
                      f"scaled by the oracle's 68 squarings per conversion",
            "mul_relin_per_s": done / el, "seconds": el}


if __name__ == "__main__":
    main()
