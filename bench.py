"""Benchmark: batched BootMMPM bootstraps per second at t = 2^12 on one MI355X.

One step = one call of the whole hot path (modulus switch, accumulator
initialisation, 630 CMux steps, sample extraction, key switch, final modulus
switch) over a batch of 4096 ciphertexts with n = 630, N = 1024, k = r = 4,
t = t' = 2^12, gadget 2^7 x 4, key switch 2^4 x 8, Q = 2^31 - 2^17 + 1, inputs
resident in device memory.  Alongside: the plain per-ciphertext path on the same
GPU, the blind-rotation kernel's roofline, and the CPU oracle on the host cores.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BATCH = 4096
# MI355X vector issue: the published fp32 vector rate 157.3 TFLOP/s is 256 CUs x
# 128 FMA lanes/clock x 2 flops x 2.4 GHz, i.e. 78.6 T lane-instructions/s; a
# 32-bit integer VALU instruction takes the same issue slot.
PEAK_LANE_OPS = 256 * 128 * 2.4e9
# One wave64 VALU instruction per 4 clocks per SIMD, without dual issue: the
# rate a stream of 64-bit multiply-adds can reach.
SINGLE_ISSUE_LANE_OPS = 256 * 64 * 2.4e9
# Issue rate of a register-only loop of lazy Montgomery butterflies (64-bit
# multiply-add, low-word multiply, multiply-add, subtract, min, add, subtract, add:
# 8 instructions), 16 independent chains per thread, 4096 workgroups, measured on
# the MI355X at the occupancy of each blind-rotation kernel: the ceiling that
# instruction mix can reach (4.817e12 butterflies/s at 2 waves per SIMD, 4.957e12
# at 5).
MIX_CEILING_LANE_OPS = {2: 38.5e12, 5: 39.7e12}
PEAK_HBM = 8.0e12
KERNEL_SOURCES = ("paper_2310_12441_amd/csrc/kernels.hip", "paper_2310_12441_amd/csrc/kernels_wide.hip",
                  "paper_2310_12441_amd/csrc/device_common.hpp")
# counter summaries of the two blind-rotation kernels the schedule can pick for the
# paper-shaped batch: the fused persistent kernel, and the global-accumulator kernel
# with four waves per component (one launch per CMux step)
COUNTERS = {"fused": os.path.join(ROOT, "profiles", "k_blind_rotate_paper_shaped_4096_counters.txt"),
            "global": os.path.join(ROOT, "profiles", "k_wide_step_paper_shaped_4096_counters.txt")}


def ops_per_bootstrap(n, N, l, r):
    """Algorithmic 32-bit VALU instructions (lane-ops) of one blind rotation.

    Op model, one lane-op per instruction of the shortest sequence in the
    representation used (residues in [0, Q), Q < 2^31, Montgomery twiddles):
    Cooley-Tukey butterfly 11 = Montgomery product 5 (64-bit product, low-word
    multiply, multiply-add, subtract, min) + modular add 3 + modular subtract 3;
    Gentleman-Sande butterfly 10 = modular add 3 + lazy subtract 2 + Montgomery
    product 5; NTT-domain multiply-accumulate 10 per pair of key products = two
    64-bit multiply-adds + Montgomery reduction 5 + modular add 3.  Per step and
    ring component: 2l forward and 2 inverse NTTs of (N/2) log2 N butterflies and
    2 N l product pairs.  Decomposition, rotation, data movement and address
    arithmetic are not counted.
    """
    logN = int(np.log2(N))
    bfly = (N // 2) * logN
    per_comp = 2 * l * bfly * 11 + 2 * bfly * 10 + 2 * N * l * 10
    return n * r * per_comp


# The paper's own times for the same workload (identity f by two bootstraps, n = 2^9,
# N = 2^11, log Q = 54, B = 2^15, q = 128 t), seconds per evaluation on one CPU
# thread: Table 1 (Intel i7-10700, log t = 5..11) and, for log t = 12, Table 2
# (Xeon Gold 6258R, n = 2^10).  Context for the paper-margin sweep, not a target.
PAPER_IDENTITY_SECONDS = {5: (0.7375, "Table 1"), 6: (1.3625, "Table 1"), 7: (2.6376, "Table 1"),
                          8: (5.2578, "Table 1"), 9: (10.203, "Table 1"), 10: (20.261, "Table 1"),
                          11: (41.795, "Table 1"), 12: (202.56, "Table 2, n = 2^10"),
                          13: (413.22, "Table 2, n = 2^10"), 14: (834.60, "Table 2, n = 2^10"),
                          15: (1676.3, "Table 2, n = 2^10")}


def ops_per_bootstrap_wide(n, N, l, r, keys=1):
    """The same op model at a ring modulus of two primes: every NTT, product and
    accumulation runs once per prime; with a ternary secret (keys = 2) each
    step has two sets of forward NTTs and products and one inverse NTT pair.
    Joining the residues, the decomposition, the rotation and data movement are
    not counted."""
    logN = int(np.log2(N))
    bfly = (N // 2) * logN
    per_prime = keys * (2 * l * bfly * 11 + 2 * N * l * 10) + 2 * bfly * 10
    return n * r * 2 * per_prime


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path):
    """HBM bytes per launch of a blind-rotation kernel from its committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != source_hash():
        return None
    try:
        return int(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bsk_bytes(n, N, l):
    return n * 2 * l * 2 * N * 4


def ksk_bytes(n, N, p):
    return N * p.l_ks * p.B_ks * (n + 1) * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--plain", type=int, default=20,
                    help="single-ciphertext plain-path runs (latency = their median)")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: one per host thread)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed", type=int, default=2048,
                    help="ciphertexts of the uneven-class batch (0: no mixed leg)")
    ap.add_argument("--compare", type=int, default=4096,
                    help="batch of the MMPM vs TFHE-shaped comparison per class (0: no comparison leg)")
    ap.add_argument("--compare-max-logt", type=int, default=16,
                    help="largest log2 t of the TFHE-shaped comparison (15: N = 16384, 16: 32768, 17: 65536)")
    ap.add_argument("--compare-only", default="",
                    help="comma-separated log2 t: run only these comparison rows (for profiling one ring)")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per arrival rate (0: no serving leg)")
    ap.add_argument("--serve-rates", default="5000,10000,20000,50000", help="Poisson arrival rates, req/s")
    ap.add_argument("--serve-max-latency", type=float, default=50.0,
                    help="admission bound on the expected latency, ms, for the load-shedding runs (0: none)")
    ap.add_argument("--margin", type=int, default=16384,
                    help="ring components per batch of the paper-margin sweep (0: no such leg)")
    ap.add_argument("--margin-logt", default="5,6,7,8,9,10,11,12,13,14,15", help="log2 t of the paper-margin sweep")
    ap.add_argument("--margin-serve-requests", type=int, default=64,
                    help="requests of the paper-margin serving run at t = 2^12 (0: none)")
    ap.add_argument("--margin-serve-rate", type=float, default=50.0, help="its Poisson arrival rate, req/s")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); ciphertexts are independent, "
              "so more GPUs would each bootstrap their own share with a replica of the keys", flush=True)
        sys.exit(2)
    t_start = time.perf_counter()

    import torch

    from paper_2310_12441_amd import binding
    from synth import PRESETS, enc_draws, key_draws, messages, negacyclic_table

    pre = PRESETS["paper_shaped"]
    p, t, r = pre["params"], pre["t"], pre["r"]
    q = 2 * p.N * r
    B = args.batch
    seeds = {"keys": 1, "table": 2, "messages": 3, "encryption": 4}
    draws = key_draws(p, seeds["keys"])
    ctx = binding.Context(p, draws)
    ctx.device_init(0)
    f = negacyclic_table(t, t, seeds["table"])
    tid = ctx.table_create(t, t, r, f)
    m = messages(t, B, seeds["messages"])
    ed = enc_draws(p.n, q, B, seeds["encryption"])
    ct = ctx.encrypt(q, t, m, ed["a"], ed["e"])
    ids = np.full(B, tid, dtype=np.int32)
    dev_in = torch.from_numpy(ct.view(np.int32)).cuda()
    dev_out = torch.empty_like(dev_in)

    # ---- schedule for this batch shape (not timed)
    schedule = ctx.autotune(ids, ct)
    sched = ctx.schedule_describe(ids)

    # ---- batched path (timed): the product's path, one captured graph per batch,
    # no events inside; wall clock over the steps
    ctx.set_timing(False)
    for _ in range(args.warmup):
        ctx.bootstrap(ids, dev_in, out=dev_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.bootstrap(ids, dev_in, out=dev_out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = B * args.steps / wall
    batched_out = dev_out.cpu().numpy().view(np.uint32).copy()
    # kernel split, separately: the blind-rotation and key-switch halves as two
    # graphs with HIP events between them on the stream they run on
    ctx.set_timing(True)
    ctx.bootstrap(ids, dev_in, out=dev_out)
    ctx.last_timing()
    br_ms, ks_ms = [], []
    t_ev = time.perf_counter()
    for _ in range(max(2, min(args.steps, 5))):
        ctx.bootstrap(ids, dev_in, out=dev_out)
        a, b = ctx.last_timing()
        br_ms.append(a)
        ks_ms.append(b)
    torch.cuda.synchronize()
    timed_wall_ms = (time.perf_counter() - t_ev) * 1e3 / len(br_ms)
    ctx.set_timing(False)
    split_same = bool(np.array_equal(dev_out.cpu().numpy().view(np.uint32), batched_out))

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.int32, device="cuda").fill_(7)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- plain path on the same GPU: one ciphertext per call, latency = median of the runs
    P = min(args.plain, B)
    plain_rate, plain_same, plain_lat = None, None, []
    if P > 0:
        ctx.bootstrap(ids[:1], dev_in[:1], plain=True)
        torch.cuda.synchronize()
        plain_outs = []
        for k in range(P):
            t1 = time.perf_counter()
            o = ctx.bootstrap(ids[k:k + 1], dev_in[k:k + 1], plain=True)
            torch.cuda.synchronize()
            plain_lat.append(time.perf_counter() - t1)
            plain_outs.append(o)
        plain_rate = 1.0 / float(np.median(plain_lat))
        plain_out = torch.cat(plain_outs).cpu().numpy().view(np.uint32)
        plain_same = bool(np.array_equal(plain_out, batched_out[:P]))

    # ---- roofline of the blind-rotation kernel the schedule picked: the fused
    # persistent kernel (one launch per batch) or the global-accumulator kernel (one
    # launch per CMux step, plus an initialisation and an extraction launch inside the
    # same HIP-event bracket, so the per-launch time below is slightly conservative)
    br_avg = float(np.mean(br_ms)) * 1e-3
    global_shape = sched[0] == 0
    launches = p.n if global_shape else 1
    per_launch = br_avg / launches
    ops = ops_per_bootstrap(p.n, p.N, p.l, r) * B // launches
    achieved = ops / per_launch
    waves_per_simd = 5 if global_shape else 2  # VGPR-bound occupancy of each kernel (94 and 256 VGPRs)
    mix = MIX_CEILING_LANE_OPS[waves_per_simd]
    hbm_alg = (bsk_bytes(p.n, p.N, p.l) + B * (p.n + 1) * 4 + B * (p.N + 1) * 4) // launches
    if global_shape:
        kname = f"k_wide_step<{p.N},1,1,{sched[3]},{2 if sched[5] == 4 else 1},false>"
    else:
        kname = f"k_blind_rotate<{p.N},{sched[0]},1,{sched[3]}" + (",true" if sched[5] == 1 else "") + ">"
    roofline = {
        "bound": "alu",
        "achieved": round(achieved / 1e12, 3),
        "peak": round(PEAK_LANE_OPS / 1e12, 3),
        "unit": "TOP/s",
        "frac": round(achieved / PEAK_LANE_OPS, 4),
        "peak_single_issue": round(SINGLE_ISSUE_LANE_OPS / 1e12, 3),
        "frac_single_issue": round(achieved / SINGLE_ISSUE_LANE_OPS, 4),
        "mix_ceiling": round(mix / 1e12, 3),
        "mix_ceiling_waves_per_simd": waves_per_simd,
        "frac_mix_ceiling": round(achieved / mix, 4),
        "traffic": measured_traffic(COUNTERS["global" if global_shape else "fused"]),
        "kernel": kname,
        "launches_per_batch": launches,
        "kernel_ms": round(per_launch * 1e3, 4),
        "blind_rotation_ms_per_batch": round(br_avg * 1e3, 3),
        "ops_per_launch": ops,
        "hbm_algorithmic_bytes": hbm_alg,
        "hbm_frac": round(hbm_alg / per_launch / PEAK_HBM, 6),
        "kernel_source_sha256_16": source_hash(),
    }

    legs = {"main_and_plain": round(time.perf_counter() - t_start, 1)}
    t_leg = time.perf_counter()

    def leg(name):
        nonlocal t_leg
        legs[name] = round(time.perf_counter() - t_leg, 1)
        t_leg = time.perf_counter()
        print(json.dumps({"leg_done": name, "seconds": legs[name]}), file=sys.stderr, flush=True)

    # ---- uneven classes: one table per (t, k), classes drawn uniformly per ciphertext
    from synth import CLASS_MIX, class_mix, poisson_arrivals
    tabs = []
    for k, (tt, rr) in enumerate(CLASS_MIX):
        tabs.append((ctx.table_create(tt, tt, rr, negacyclic_table(tt, tt, 100 + k)), tt, rr))

    def class_batch(count, mix_seed, enc_seed):
        cls = class_mix(count, mix_seed)
        c_ids = np.array([tabs[k][0] for k in cls], np.int32)
        c_ct = np.empty((count, p.n + 1), np.uint32)
        for k, (tid_k, tt, rr) in enumerate(tabs):
            sel = np.where(cls == k)[0]
            qq = 2 * p.N * rr
            edk = enc_draws(p.n, qq, sel.size, enc_seed + k)
            c_ct[sel] = ctx.encrypt(qq, tt, messages(tt, sel.size, enc_seed + 100 + k), edk["a"], edk["e"])
        return c_ids, c_ct

    mixed = None
    if args.mixed > 0:
        M = args.mixed
        x_ids, x_ct = class_batch(M, 8, 400)
        x_in = torch.from_numpy(x_ct.view(np.int32)).cuda()
        x_out = torch.empty_like(x_in)
        x_sched = ctx.autotune(x_ids, x_ct)
        x_desc = ctx.schedule_describe(x_ids)
        ctx.bootstrap(x_ids, x_in, out=x_out)
        torch.cuda.synchronize()
        reps = max(3, args.steps)
        x_times, x_br, x_ks = [], [], []
        for _ in range(reps):  # each call synchronised; the median resists a stray slow call
            t3 = time.perf_counter()
            ctx.bootstrap(x_ids, x_in, out=x_out)
            torch.cuda.synchronize()
            x_times.append(time.perf_counter() - t3)
        # the kernel split from two separate event-timed calls
        ctx.set_timing(True)
        for _ in range(2):
            ctx.bootstrap(x_ids, x_in, out=x_out)
            a_, b_ = ctx.last_timing()
            x_br.append(a_)
            x_ks.append(b_)
        ctx.set_timing(False)
        x_s = float(np.median(x_times))
        cls_x = class_mix(M, 8)
        rs = np.array([tabs[i][2] for i in cls_x])
        x_check = None
        if not args.no_cpu:
            # oracle on 4 ciphertexts of every class of this batch
            import oracle
            okeys = oracle.KeySet(p, draws)
            x_got = x_out.cpu().numpy().view(np.uint32)
            x_ok = True
            for k, (tid_k, tt, rr) in enumerate(tabs):
                sel = np.where(cls_x == k)[0]
                pick = sel[np.linspace(0, sel.size - 1, 4).astype(int)]
                Vk = oracle.test_vector(p.N, rr, p.Q, tt, tt, negacyclic_table(tt, tt, 100 + k))
                qq = 2 * p.N * rr
                want_k = oracle.bootstrap_many(p, rr, okeys.bsk, okeys.ksk, Vk, qq, qq, x_ct[pick])
                x_ok = x_ok and bool(np.array_equal(x_got[pick], want_k))
            x_check = {"oracle_samples": 4 * len(tabs), "equal": x_ok}
        mixed = {"batch": M, "classes": [list(c) for c in CLASS_MIX], "bootstraps_per_s": round(M / x_s, 1),
                 "ms_per_batch": round(x_s * 1e3, 3), "ms_per_batch_all": [round(v * 1e3, 3) for v in x_times],
                 "blind_rotation_ms": round(float(np.median(x_br)), 3), "keyswitch_ms": round(float(np.median(x_ks)), 3),
                 "components": int(rs.sum()), "parity": x_check,
                 "schedule": {"index": x_sched, "group_waves": x_desc[0], "ks_cts_per_wave": x_desc[1],
                              "ks_splits": x_desc[2], "waves_per_component": x_desc[3]}}

    leg("mixed")
    # ---- Sec. 5 comparison: each class (t, k) by MMPM (N = 1024, r = k) and by one
    # ring of degree N k (r = 1, TFHE-shaped), same n, gadget and key switch
    comparison = None
    if args.compare > 0:
        C = args.compare
        comparison = []

        def timed_batch(cx, tid_c, t_c, r_c, N_c, seed):
            qq = 2 * N_c * r_c
            edc = enc_draws(p.n, qq, C, seed)
            cts = cx.encrypt(qq, t_c, messages(t_c, C, seed + 1), edc["a"], edc["e"])
            ids_c = np.full(C, tid_c, np.int32)
            din = torch.from_numpy(cts.view(np.int32)).cuda()
            dout = torch.empty_like(din)
            cx.autotune(ids_c, cts)
            # 0 waves per fused group: the global-accumulator path (key-switch schedules only)
            path = "global accumulator" if cx.schedule_describe(ids_c)[0] == 0 else "fused"
            tw = time.perf_counter()
            cx.bootstrap(ids_c, din, out=dout)
            torch.cuda.synchronize()
            # batches of a second or more are timed once
            reps = 1 if time.perf_counter() - tw > 0.5 else max(1, min(args.steps, 3))
            tt0 = time.perf_counter()
            for _ in range(reps):
                cx.bootstrap(ids_c, din, out=dout)
            torch.cuda.synchronize()
            return round(C * reps / (time.perf_counter() - tt0), 1), path

        # the four classes of the uneven batch, then t = 2^15 and up (r = 16, 32, ...
        # components at N = 1024 against one ring of degree 1024 r): both on the
        # global-accumulator path, rings above 16384 split into sub-rings of 8192
        big = [(1 << lt, 1 << (lt - 11)) for lt in range(15, args.compare_max_logt + 1)]
        only = {int(x) for x in args.compare_only.split(",") if x}
        for k, (tt, rr) in enumerate(list(CLASS_MIX) + big):
            if only and tt.bit_length() - 1 not in only:
                continue
            row = {"t": tt, "k": rr}
            tid_m = tabs[k][0] if k < len(tabs) else ctx.table_create(tt, tt, rr, negacyclic_table(tt, tt, 100 + k))
            bps, path = timed_batch(ctx, tid_m, tt, rr, p.N, 700 + k)
            row["mmpm"] = {"N": p.N, "r": rr, "bootstraps_per_s": bps, "path": path,
                           "bsk_bytes": bsk_bytes(p.n, p.N, p.l), "ksk_bytes": ksk_bytes(p.n, p.N, p)}
            if rr == 1:
                row["tfhe"] = dict(row["mmpm"])  # the same ring: r = 1 at N = 1024
            else:
                from dataclasses import replace
                pt = replace(p, N=p.N * rr)
                cx = binding.Context(pt, key_draws(pt, seeds["keys"]))
                cx.device_init(0)
                tid_t = cx.table_create(tt, tt, 1, negacyclic_table(tt, tt, 100 + k))
                bps, path = timed_batch(cx, tid_t, tt, 1, pt.N, 700 + k)
                row["tfhe"] = {"N": pt.N, "r": 1, "bootstraps_per_s": bps, "path": path,
                               "bsk_bytes": bsk_bytes(pt.n, pt.N, pt.l), "ksk_bytes": ksk_bytes(pt.n, pt.N, pt)}
                cx.close()
                del cx
            row["mmpm_over_tfhe_speed"] = round(row["mmpm"]["bootstraps_per_s"] / row["tfhe"]["bootstraps_per_s"], 3)
            row["parity"] = {256: "same ring as the MMPM side", 1024: "tests: N = 2048 end to end",
                             4096: "tests: N = 4096 samples of a batch", 16384: "tests: the bench batch's samples "
                             "(stored oracle outputs) and N = 8192 end to end",
                             32768: "tests: r = 16 at N = 1024 and N = 16384 end to end",
                             65536: "tests: N = 32768 end to end (split ring)",
                             131072: "tests: N = 65536 end to end (split ring)"}[tt]
            comparison.append(row)
            print(json.dumps({"comparison_row": row}), file=sys.stderr, flush=True)

    leg("comparison")
    # ---- serving: Poisson arrivals of single bootstraps with mixed (t, k), keys resident
    serving = None
    if args.serve_requests > 0:
        R = args.serve_requests
        s_ids, s_ct = class_batch(R, 7, 200)
        alone = None
        serving = {"rates_req_s": [], "p50_ms": [], "p99_ms": [], "completed_per_s": [], "requests_per_rate": R,
                   "classes": [list(c) for c in CLASS_MIX], "chunk_steps": 63, "hbm_budget_bytes": 4 << 30}
        serving["admission"] = {"max_latency_ms": args.serve_max_latency, "rates_req_s": [], "admitted_fraction": [],
                                "p50_ms": [], "p99_ms": [], "completed_per_s": [], "identical_to_alone": True}
        for rate in [float(x) for x in args.serve_rates.split(",") if x]:
            srv = ctx.server_start(4 << 30, chunk_steps=63)
            warm = min(512, R)
            srv.replay(s_ids[:warm], s_ct[:warm], poisson_arrivals(rate, warm, 11))
            srv.stop()
            srv = ctx.server_start(4 << 30, chunk_steps=63)
            out_s, lat = srv.replay(s_ids, s_ct, poisson_arrivals(rate, R, 12))
            st = srv.stats()
            srv.stop()
            serving["rates_req_s"].append(rate)
            serving["p50_ms"].append(round(float(np.percentile(lat, 50)), 3))
            serving["p99_ms"].append(round(float(np.percentile(lat, 99)), 3))
            serving["completed_per_s"].append(round(st["boots_per_s"], 1))
            if alone is None:
                alone = ctx.bootstrap(s_ids, s_ct)
                serving["identical_to_alone"] = bool(np.array_equal(out_s, alone))
            if args.serve_max_latency > 0:
                # the same trace with load shedding: requests whose expected latency exceeds
                # the bound are refused at submission
                srv = ctx.server_start(4 << 30, chunk_steps=63)
                srv.set_admission(args.serve_max_latency)
                out_a, lat_a = srv.replay(s_ids, s_ct, poisson_arrivals(rate, R, 12))
                st_a = srv.stats()
                srv.stop()
                ok = lat_a >= 0
                adm = serving["admission"]
                adm["rates_req_s"].append(rate)
                adm["admitted_fraction"].append(round(float(ok.mean()), 4))
                adm["p50_ms"].append(round(float(np.percentile(lat_a[ok], 50)), 3))
                adm["p99_ms"].append(round(float(np.percentile(lat_a[ok], 99)), 3))
                adm["completed_per_s"].append(round(st_a["boots_per_s"], 1))
                adm["identical_to_alone"] = adm["identical_to_alone"] and bool(np.array_equal(out_a[ok], alone[ok]))

    leg("serving")
    # ---- the parameters of the experiments in Sec. 5 (Tables 1-2): n = 512, N = 2048,
    # ring modulus of 54 bits (two primes), gadget 2^15 x 4, q = 2Nr = 128 t, the
    # identity function on Z_t by two bootstraps (plaintext modulus 2t), noisy inputs
    margin = None
    if args.margin > 0:
        margin = margin_leg(args, binding, torch)

    leg("paper_margin")
    # ---- CPU oracle on the host cores, on a bounded sample of the same batch
    cpu = None
    if not args.no_cpu:
        import oracle
        nthr = oracle.num_threads()
        S = args.cpu_sample or max(64, 4 * nthr)
        keys = oracle.KeySet(p, draws)
        V = oracle.test_vector(p.N, r, p.Q, t, t, f)
        idx = np.linspace(0, B - 1, S).astype(int)
        t2 = time.perf_counter()
        want = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct[idx])
        cpu_s = time.perf_counter() - t2
        # one ciphertext runs on one thread: the single-core latency
        t3 = time.perf_counter()
        one = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct[idx[:1]])
        single_s = time.perf_counter() - t3
        cpu_model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")),
                         None) if os.path.exists("/proc/cpuinfo") else None
        cpu = {"value": round(S / cpu_s, 4), "unit": "bootstraps/s", "cores": nthr, "kind": "oracle",
               "cpu_model": cpu_model,
               "sample": f"{S} of the {B} ciphertexts (evenly spaced), one ciphertext per thread, schoolbook products",
               "seconds": round(cpu_s, 2), "single_thread_s_per_bootstrap": round(single_s, 3),
               "parity_with_gpu": bool(np.array_equal(want, batched_out[idx]) and np.array_equal(one, want[:1]))}

    leg("cpu_baseline")
    line = {
        "metric": "bootstraps/sec at t=2^12 (batched vs plain, bit-exact); serving p50/p99 ms",
        "value": round(value, 2),
        "unit": "bootstraps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"batched {B} x BootMMPM (n=630, N=1024, k=4, t=2^12, B=2^7 l=4, Bks=2^4 lks=8)",
                   "batch": B, "n": p.n, "N": p.N, "k": r, "t": t, "q": q, "Q": p.Q, "seeds": seeds},
        "plain_bootstraps_per_s": round(plain_rate, 3) if plain_rate else None,
        "plain_ms_per_bootstrap": round(1e3 / plain_rate, 3) if plain_rate else None,
        "plain_runs": len(plain_lat),
        "batched_vs_plain": round(value / plain_rate, 2) if plain_rate else None,
        "plain_equals_batched": plain_same,
        "kernel_split": {"blind_rotation_ms": round(float(np.mean(br_ms)), 3),
                         "keyswitch_ms": round(float(np.mean(ks_ms)), 3),
                         "wall_ms_per_batch_with_events": round(timed_wall_ms, 3),
                         "same_bits_as_timed_steps": split_same,
                         "how": "two graphs (blind rotation; key switch + final switch) with HIP events "
                                "between them on their stream, run after the timed steps"},
        "keyswitch_ms": round(float(np.mean(ks_ms)), 3),
        "schedule": {"index": schedule, "group_waves": sched[0], "ks_cts_per_wave": sched[1], "ks_splits": sched[2],
                     "waves_per_component": sched[3]},
        "mixed_classes": mixed,
        "mmpm_vs_tfhe_shaped": comparison,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "paper_margin": margin,
        "leg_seconds": legs,
    }
    print(json.dumps(line), flush=True)


def margin_leg(args, binding, torch):
    """Per log t: batched throughput of one nega-cyclic bootstrap and of the
    identity function (two bootstraps), the plain latency of the identity for one
    ciphertext, the blind-rotation / key-switch split and correct decryption."""
    from synth import PRESETS, enc_draws, key_draws, messages, negacyclic_table

    pre = PRESETS["paper_margin"]
    pw = pre["params"]
    seed = 31
    mctx = binding.Context(pw, key_draws(pw, seed))
    mctx.device_init(0)
    rows = []
    for logt in [int(x) for x in args.margin_logt.split(",") if x]:
        t = 1 << logt
        r = max(1, t * 128 // (2 * pw.N))  # q = 2Nr = 128 t
        q = 2 * pw.N * r
        Bm = max(8, min(4096, args.margin // r))
        row = {"log_t": logt, "r": r, "log_q": int(np.log2(q)), "batch": Bm}
        # one nega-cyclic bootstrap (2Nr / t = 128)
        tid = mctx.table_create(t, t, r, negacyclic_table(t, t, 500 + logt))
        edn = enc_draws(pw.n, q, Bm, 600 + logt)
        mn = messages(t, Bm, 700 + logt)
        ctn = mctx.encrypt(q, t, mn, edn["a"], edn["e"])
        din = torch.from_numpy(ctn.view(np.int32)).cuda()
        dout = torch.empty_like(din)
        ids = np.full(Bm, tid, np.int32)
        tw = time.perf_counter()
        mctx.bootstrap(ids, din, out=dout)
        torch.cuda.synchronize()
        reps = 1 if time.perf_counter() - tw > 0.5 else 2  # batches of a second or more are timed once
        t0 = time.perf_counter()
        for _ in range(reps):
            mctx.bootstrap(ids, din, out=dout)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        # the kernel split from one separate event-timed call
        mctx.set_timing(True)
        mctx.bootstrap(ids, din, out=dout)
        a_, b_ = mctx.last_timing()
        mctx.set_timing(False)
        br_ms, ks_ms = [a_], [b_]
        row["bootstraps_per_s"] = round(Bm / dt, 1)
        row["blind_rotation_ms"] = round(float(np.mean(br_ms)), 3)
        row["keyswitch_ms"] = round(float(np.mean(ks_ms)), 3)
        ops = ops_per_bootstrap_wide(pw.n, pw.N, pw.l, r, pw.keys_per_coord) * Bm
        row["blind_rotation_tops"] = round(ops / (row["blind_rotation_ms"] * 1e-3) / 1e12, 3)
        # the identity on Z_t: plaintext modulus 2t, two bootstraps
        ident = mctx.table_create_general(t, t, r, np.arange(t, dtype=np.uint32))
        mi = messages(t, Bm, 800 + logt)
        edi = enc_draws(pw.n, q, Bm, 900 + logt)
        cti = mctx.encrypt(q, 2 * t, mi, edi["a"], edi["e"])
        iin = torch.from_numpy(cti.view(np.int32)).cuda()
        iout = torch.empty_like(iin)
        iids = np.full(Bm, ident, np.int32)
        mctx.bootstrap(iids, iin, out=iout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mctx.bootstrap(iids, iin, out=iout)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        row["identity_per_s"] = round(Bm / dt, 1)
        outn = dout.cpu().numpy().view(np.uint32)
        outi = iout.cpu().numpy().view(np.uint32)
        row["correct"] = bool(np.array_equal(mctx.decrypt(q, t, outi), mi) and
                              np.array_equal(mctx.decrypt(q, t, outn), negacyclic_table(t, t, 500 + logt)[mn]))
        row["check"] = "every output decrypted (noisy keys and inputs); not compared with the oracle here"
        lat = []
        for k in range(3):
            t0 = time.perf_counter()
            mctx.bootstrap([ident], cti[k:k + 1], plain=True)
            lat.append(time.perf_counter() - t0)
        row["identity_plain_ms"] = round(float(np.median(lat)) * 1e3, 3)
        if logt in PAPER_IDENTITY_SECONDS:
            sec, where = PAPER_IDENTITY_SECONDS[logt]
            row["paper_identity_s"] = {"value": sec, "source": where, "hardware": "one CPU thread (PALISADE)"}
        rows.append(row)
        print(json.dumps({"paper_margin_row": row}), file=sys.stderr, flush=True)
    # serving at t = 2^12 (r = 128): continuous batching on the global-accumulator path
    serve = None
    if args.margin_serve_requests > 0:
        from synth import poisson_arrivals
        t, R = 1 << 12, args.margin_serve_requests
        r = t * 128 // (2 * pw.N)
        q = 2 * pw.N * r
        f = negacyclic_table(t, t, 512)
        tid = mctx.table_create(t, t, r, f)
        ed = enc_draws(pw.n, q, R, 950)
        m = messages(t, R, 951)
        cts = mctx.encrypt(q, t, m, ed["a"], ed["e"])
        ids = np.full(R, tid, np.int32)
        batched = mctx.bootstrap(ids, cts)
        srv = mctx.server_start(8 << 30, chunk_steps=64)
        try:
            out, lat = srv.replay(ids, cts, poisson_arrivals(args.margin_serve_rate, R, 952))
            st = srv.stats()
        finally:
            srv.stop()
        serve = {"t": t, "r": r, "requests": R, "rate_req_s": args.margin_serve_rate, "chunk_steps": 64,
                 "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                 "completed_per_s": round(st["boots_per_s"], 2),
                 "identical_to_batched": bool(np.array_equal(out, batched)),
                 "correct": bool(np.array_equal(mctx.decrypt(q, t, out), f[m]))}
        print(json.dumps({"paper_margin_serving": serve}), file=sys.stderr, flush=True)
    mctx.close()
    return {"params": {"n": pw.n, "N": pw.N, "log2_Q": int(pw.Q_ring).bit_length(), "Q": [pw.Q, pw.Q2],
                       "log2_B": pw.log2_B, "l": pw.l, "log2_Bks": pw.log2_Bks, "l_ks": pw.l_ks,
                       "secret": "ternary" if pw.ternary else "binary", "sigma": pw.sigma},
            "bsk_bytes": pw.keys_per_coord * pw.n * 2 * pw.l * 2 * pw.N * 8, "ksk_bytes": ksk_bytes(pw.n, pw.N, pw),
            "parity": ("rows are checked by decryption only; the kernels they time are compared bit for bit with "
                       "the oracle in tests/test_gpu_wide.py: this preset's r = 128 (3 CMux steps) and r = 1024 "
                       "(2 steps), and whole ternary bootstraps at N = 2048 with small n"),
            "rows": rows, "serving": serve}


if __name__ == "__main__":
    main()
