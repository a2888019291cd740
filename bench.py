"""Benchmark of the encrypted CutMax on one MI355X.

Default workload (one step = one encrypted CutMax, Alg. 2, on one ciphertext):
N = 2^16 RNS-CKKS at 128-bit security (30 Q primes, dnum = 3), 32000 LLM-like logits
(3 Gumbel - 1.1 ln rank, seeded, synthetic) zero-padded to 32768 slots, T = 3, p = 3, c = 5,
degree-3 Chebyshev inverse-square-root guess, Goldschmidt inverse with 3 squarings.
The ciphertext is resident in HBM before the timed region.

Also reported: batched argmaxes/s (16 requests: 8 x 32000 logits in 1 ciphertext and
8 x 128256 logits in 4 ciphertexts), one CutMax of 151936 logits (5 ciphertexts), NTT GB/s,
the roofline of the dominant kernel
(HIP events on the library's stream) and the CPU oracle timed on a bounded sample.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# hardware-counter summary of one CutMax (rocprofv3 FETCH_SIZE / WRITE_SIZE / VALU passes),
# valid only for the library sources it was taken with
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_cutmax_32k.json")
VOCAB2 = 32000
T, P, C = 3, 3, 5.0
VLO, VHI = [12.0, 0.4, 0.8], [24.0, 0.9, 16.0]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cfg_secure(he):
    return he.CutmaxCfg(T=T, p=[P] * T, c=[C] * T, var_lo=VLO, var_hi=VHI, init_degree=3, init_coef=None,
                        newton_steps=0, sum_lo=1.0, sum_hi=3.0, gold_d=3)


def src_digest() -> str:
    """sha256 (16 hex digits) over the library's HIP/C++ sources and its C header."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2509_08383_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(ROOT, "include", "he.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_entry(kernel: str, digest: str):
    """Counter summary of `kernel` if it was measured on these exact sources, else None."""
    try:
        with open(PMC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("src_digest") != digest:
        return None
    return next((e for e in d.get("kernels", []) if e["kernel"] == kernel), None)


def keyswitch_levels(L: int, T_: int, gold_d: int, slots: int):
    """Levels of every key switch of the schedule (rotations and relinearisations), in order."""
    lg = int(math.log2(slots))
    out = []
    lv = L
    for _ in range(T_):
        out += [lv] * lg                 # rotsum for the mean
        out += [lv - 1]                  # E^2
        out += [lv - 2] * lg             # rotsum for the variance
        out += [lv - 2, lv - 3]          # degree-3 initial guess: u^2, (g_3 u) u^2
        out += [lv - 4]                  # E * H
        out += [lv - 5, lv - 6]          # cube
        lv -= 7
    out += [lv] * lg                     # final rotsum
    e = lv - 1
    for i in range(gold_d):
        out += [e - i, e - i - 1]        # square, product
    out += [lv - gold_d - 2]             # Z = Y * P
    return out


def ks_cost(levels, alpha):
    """limb-NTT count of hybrid key switching at each level: INTT of the input, NTT of the
    converted digits, INTT of the 2 alpha P limbs, NTT of the 2 (l+1) ModDown limbs."""
    tot = 0
    for l in levels:
        beta = -(-(l + 1) // alpha)
        tot += (l + 1) + beta * (l + 1 + alpha) - (l + 1) + 2 * alpha + 2 * (l + 1)
    return tot


def _nucleus_mask(x: np.ndarray, top_p: float):
    """Membership of the smallest top-ranked set whose softmax mass reaches top_p, and the
    softmax mass outside it."""
    pr = np.exp(x - x.max())
    pr /= pr.sum()
    order = np.argsort(-pr)
    k = int(np.searchsorted(np.cumsum(pr[order]), top_p) + 1)
    m = np.zeros(x.size, dtype=bool)
    m[order[:k]] = True
    return m, 1.0 - float(pr[m].sum())


def violation_main(spec: str, graph: int):
    """Violation rate of the encrypted Gumbel-max and Beta-cut samplers (Sec. 4, "Nucleus
    Sampling", Fig. 4): S synthetic prompts x D draws each at top_p = 0.9 and temperature 1,
    16 requests per call; a pick is the argmax of the decrypted one-hot."""
    import torch
    from paper_2509_08383_amd import he
    from workloads import llm_logits_var, uniform_noise

    assert torch.cuda.is_available(), "no GPU"
    S, D = (int(v) for v in spec.split(","))
    top_p = 0.9
    ctx = he.Context(he.SECURE, device=0)
    if graph:
        ctx.set_option(he.HE_OPT_GRAPH, 1)
    # with the per-prompt Gumbel scale and Zipf exponent of this logit family, the variances
    # of the three iterations span about [6, 37], [0.33, 0.77] and [1, 116]
    vlo, vhi = [5.0, 0.3, 0.6], [48.0, 1.0, 128.0]
    cfg = he.CutmaxCfg(T=T, p=[P] * T, c=[C] * T, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=None,
                       newton_steps=0, sum_lo=1.0, sum_hi=4.0, gold_d=3, flags=he.HE_NOISE_PRESCALED)
    xs = [llm_logits_var(5000 + s) for s in range(S)]
    masks = [_nucleus_mask(x, top_p) for x in xs]
    cts = [ctx.encrypt(x) for x in xs]
    rate = {"gumbel": np.zeros(S), "beta_cut": np.zeros(S)}
    agree, calls, t_he, miss_gaps = 0, 0, 0.0, []
    for d in range(D):
        for b0 in range(0, S, 16):
            idx = list(range(b0, min(S, b0 + 16)))
            us = [uniform_noise(9000 + 1000 * s + d, xs[s].size) for s in idx]
            for kind in ("gumbel", "beta_cut"):
                gs = [he.gumbel_noise(u) if kind == "gumbel" else he.topp_noise(top_p, u) for u in us]
                nz = [ctx.encrypt(g) for g in gs]
                ins = [cts[s] for s in idx]
                ctx.sync()
                t0 = time.perf_counter()
                Z = ctx.gumbel_sample(ins, nz, 1.0, cfg) if kind == "gumbel" else \
                    ctx.topp_sample(ins, nz, top_p, 1.0, cfg)
                ctx.sync()
                t_he += time.perf_counter() - t0
                calls += len(idx)
                for j, s in enumerate(idx):
                    pick = int(np.argmax(ctx.decrypt(Z[j], xs[s].size)))
                    w = xs[s] + gs[j]
                    if pick == int(np.argmax(w)):
                        agree += 1
                    else:
                        top = np.sort(w)[-2:]
                        miss_gaps.append(float(top[1] - top[0]))
                    rate[kind][s] += float(not masks[s][0][pick]) / D
        log(f"[violation] draw {d + 1}/{D} done")
    out = {"metric": "violation rate outside the top-p nucleus", "top_p": top_p, "temperature": 1.0,
           "prompts": S, "draws_per_prompt": D, "data": "synthetic",
           "workload": "32000 LLM-like logits per prompt (Gumbel scale ~U[1.5,4.5], Zipf exponent ~U[0.9,1.3]), "
                       "N=2^16 RNS-CKKS 128-bit, T=3, p=3, c=5",
           "gumbel_max": {"mean": float(rate["gumbel"].mean()), "std": float(rate["gumbel"].std()),
                          "expected": float(np.mean([m[1] for m in masks]))},
           "beta_cut": {"mean": float(rate["beta_cut"].mean()), "std": float(rate["beta_cut"].std())},
           "encrypted_pick_equals_plaintext_pick": f"{agree}/{2 * S * D}",
           "top2_input_gap_of_mismatches": sorted(miss_gaps),
           "ms_per_sample": t_he * 1e3 / calls}
    print(json.dumps(out))


def boot_bench(he, args, x):
    from workloads import llm_logits as llm_logits_fn
    """CKKS bootstrapping at N = 2^16 (29 Q primes, the top 13 of 48 bits, sparse secret of
    weight 192, dnum = 3): one bootstrap of a ciphertext (16 levels, ratio 2^-6), and the T = 3
    CutMax on 32000 logits run on the 15 scaling levels below the wide primes, which hold two
    iterations, so the iterate is bootstrapped twice (HE_BOOT)."""
    log("[bench] bootstrappable context N=2^16")
    bctx = he.Context(he.BOOT, device=0)
    if args.graph:
        bctx.set_option(he.HE_OPT_GRAPH, 1)
    bc = he.BootCfg(ratio_bits=6)
    bctx.boot_setup(bc)
    rng = np.random.default_rng(5)
    v = rng.uniform(-1, 1, bctx.slots)
    ct = bctx.drop(bctx.encrypt(v), 2)
    out = bctx.bootstrap(ct, 1.0)
    bctx.sync()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        out = bctx.bootstrap(ct, 1.0)
    bctx.sync()
    boot_ms = (time.perf_counter() - t0) * 1e3 / reps
    err = float(np.abs(bctx.decrypt(out) - v).max())
    kern = None
    if not args.no_profile:
        bctx.profile_begin()
        bctx.bootstrap(ct, 1.0)
        kern = {k: {"launches": w[0], "ms": w[1], "bytes": w[2]} for k, w in bctx.profile_end().items()}
    log(f"[bench] bootstrap {boot_ms:.2f} ms, max err {err:.2e}")
    cfg = cfg_secure(he)
    cfg.flags = he.HE_BOOT
    ctb = bctx.encrypt(x)
    bctx.cutmax([ctb], cfg)
    bctx.sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        Zb = bctx.cutmax([ctb], cfg)[0]
    bctx.sync()
    cm_ms = (time.perf_counter() - t0) * 1e3 / reps
    cm_dev = bctx.last_cutmax_ms()
    ok = int(np.argmax(bctx.decrypt(Zb, x.size))) == int(np.argmax(x))
    log(f"[bench] bootstrapped CutMax {cm_ms:.2f} ms, argmax ok={ok}")
    zlevel = Zb.level
    del ctb, Zb
    # 16 requests of 32000 logits bootstrapped together (every launch covers all of them)
    xs = [llm_logits_fn(400 + r) for r in range(16)]
    cts = [bctx.encrypt(v) for v in xs]
    bctx.cutmax(cts, cfg)
    bctx.sync()
    t0 = time.perf_counter()
    Zs = bctx.cutmax(cts, cfg)
    bctx.sync()
    per_batch = time.perf_counter() - t0
    okb = sum(int(np.argmax(bctx.decrypt(Zs[r], xs[r].size)) == int(np.argmax(xs[r]))) for r in range(16))
    log(f"[bench] bootstrapped batch of 16: {per_batch * 1e3:.1f} ms, {okb}/16 argmax")
    del cts, Zs
    # the paper's largest vocabulary, 151936 logits in 5 ciphertexts, bootstrapped
    xq = llm_logits_fn(300, 151936)
    cq = bctx.encrypt(xq)
    bctx.cutmax([cq], cfg)
    bctx.sync()
    t0 = time.perf_counter()
    Zq = bctx.cutmax([cq], cfg)[0]
    bctx.sync()
    q_ms = (time.perf_counter() - t0) * 1e3
    okq = int(np.argmax(bctx.decrypt(Zq, xq.size))) == int(np.argmax(xq))
    log(f"[bench] bootstrapped 151936 logits: {q_ms:.1f} ms, argmax ok={okq}")
    del cq, Zq
    # error-corrected bootstrap: a second pass on the residual under bound 2^-6
    bctx.boot_setup(he.BootCfg(ratio_bits=6, correct_bits=6))
    out2 = bctx.bootstrap(ct, 1.0)
    bctx.sync()
    t0 = time.perf_counter()
    for _ in range(3):
        out2 = bctx.bootstrap(ct, 1.0)
    bctx.sync()
    corr_ms = (time.perf_counter() - t0) * 1e3 / 3
    corr_err = float(np.abs(bctx.decrypt(out2) - v).max())
    log(f"[bench] error-corrected bootstrap {corr_ms:.2f} ms, max err {corr_err:.2e}")
    table2 = table2_bench(he, bctx, args.table2_prompts) if args.table2_prompts > 0 else None
    res = {"params": "N=2^16, 29 Q primes (q0 48 bits, 15 x 40, 13 x 48), 10 P primes, dnum=3, "
                     "sparse ternary secret h=192",
           "levels_used": bc.levels(), "ratio_bits": bc.ratio_bits, "bootstrap_ms": boot_ms,
           "bootstrap_max_err_bound1": err, "out_level": out.level,
           "cutmax_T3_bootstrapped_ms": cm_ms, "cutmax_device_ms": cm_dev,
           "bootstraps_per_cutmax": 2, "cutmax_argmax_ok": bool(ok), "cutmax_out_level": zlevel,
           "batch16_ms": per_batch * 1e3, "batch16_argmaxes_per_s": 16.0 / per_batch, "batch16_argmax_ok": okb,
           "vocab_151936_ms": q_ms, "vocab_151936_argmax_ok": bool(okq),
           "corrected_bootstrap_ms": corr_ms, "corrected_bootstrap_max_err_bound1": corr_err,
           "table2_schedule": table2, "kernels": kern}
    bctx.close()
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(prm, x, ctx, args):
    """The oracle (plain C RNS-CKKS, OpenMP over limbs) timed on this host: the whole
    T = 3 encrypted CutMax on the bench input at the default thread count, and one
    top-level rotate-and-sum at one thread and at that thread count; the single-thread
    CutMax time is the sample's single-thread time scaled by the CutMax/sample ratio
    measured at the full thread count."""
    from oracle import ckks
    from oracle.cutmax_fp64 import chebyshev_invsqrt, slot_layout
    L = ckks.lib()
    threads = L.oc_num_threads()
    O = ckks.Oracle(ckks.Params(prm.log_n, prm.n_q, prm.q0_bits, prm.q_bits, prm.p_bits, prm.dnum,
                                prm.log2_scale, prm.seed, prm.hoist))
    O.keygen_cutmax()
    y, a, _ = slot_layout(x, O.slots)
    oc = O.encrypt(y)
    Ts = args.cpu_T
    coef = [list(chebyshev_invsqrt(VLO[t] / VHI[t], 3)) for t in range(Ts)]
    hc = ckks.HECfg(T=Ts, p=[P] * Ts, c=[C] * Ts, v_lo=VLO[:Ts], v_hi=VHI[:Ts], coef=coef, sum_lo=1.0,
                    sum_hi=3.0)
    c0 = time.perf_counter()
    ckks.cutmax_he(O, [oc], hc)
    sample_s = time.perf_counter() - c0
    full = ks_cost(keyswitch_levels(ctx.L, T, 3, ctx.slots), ctx.alpha)
    smp = ks_cost(keyswitch_levels(ctx.L, Ts, 3, ctx.slots), ctx.alpha)
    cm_ms = sample_s * 1e3 * full / smp
    what = ("the whole T=3 encrypted CutMax (Alg. 2)" if Ts == T else
            f"a T={Ts} encrypted CutMax scaled by the level-weighted key-switch work ({full}/{smp} limb-NTTs)")
    # one rotate-and-sum at the top level: all threads, then one thread
    t0 = time.perf_counter()
    O.rotsum(oc)
    rs_all = time.perf_counter() - t0
    L.oc_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.rotsum(oc)
        rs_one = time.perf_counter() - t0
    finally:
        L.oc_set_num_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": cm_ms, "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"{what} on the same 32000-logit input, one run, {sample_s:.2f} s at {threads} threads",
            "single_thread_ms": cm_ms * rs_one / rs_all,
            "single_thread_sample": f"one top-level rotate-and-sum (15 rotations as 5 hoisted steps): "
                                    f"{rs_one:.2f} s at 1 thread, {rs_all:.2f} s at {threads} threads; "
                                    f"the CutMax at 1 thread = CutMax at {threads} threads x that ratio",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": affinity}


def learned_bench(he, ctx, args):
    """The learned inverse-square-root initial guess against the fixed schedule.

    args.learned_runs plaintext CutMax runs (Alg. 1, T = 3, p = 3, c = 5) on LLM-like
    logits with a per-run Gumbel scale U[1.5, 4.5] and Zipf exponent U[0.9, 1.3] are
    logged on the GPU (one variance per iteration per run); per iteration one network
    (1-16-16-1, square activations, FP32, the library's kernels) is trained on 80% of the
    runs and collapsed to its quartic; the held-out 20% give each guess's RMS relative
    error of u^(-1/2) and the depth the fixed Chebyshev + Newton schedule needs to match
    the learned error.  Then 16 requests of 32000 logits at N = 2^16 (seeds disjoint from
    the logged runs) run the learned schedule (degree-4 guess, depth 3) and the fixed one
    (degree-3 Chebyshev guess, depth 2): levels left, ms per batch, argmax agreement."""
    from workloads import llm_logits_var
    vlo, vhi = [5.0, 0.4, 0.7], [48.0, 1.0, 64.0]
    t0 = time.perf_counter()
    v, _ = he.variance_log(seed=7, runs=args.learned_runs)
    t_log = time.perf_counter() - t0
    log(f"[bench] logged {v.size} variances in {t_log:.1f} s")

    def pe(c, u):
        acc = np.zeros_like(u)
        for a in c[::-1]:
            acc = acc * u + a
        return acc

    def rms(h, u):
        return float(np.sqrt(np.mean((h * np.sqrt(u) - 1.0) ** 2)))

    depth_of = {1: 1, 2: 2, 3: 2, 4: 3}
    coefs, per_t = [], []
    t_train = 0.0
    for t in range(3):
        inside = (v[:, t] >= vlo[t]) & (v[:, t] <= vhi[t])
        u = (v[inside, t] / vhi[t]).astype(np.float32)
        ntr = int(0.8 * u.size)
        M = he.InvSqrtMLP(seed=7 + t)
        t1 = time.perf_counter()
        loss = M.train(u[:ntr], epochs=args.learned_epochs, batch=1024, lr=1e-2, seed=7)
        t_train += time.perf_counter() - t1
        c = M.to_poly()
        coefs.append([float(a) for a in c])
        ut = u[ntr:].astype(np.float64)
        e_l = rms(pe(c, ut), ut)
        e_f = rms(pe(he.invsqrt_guess_fit(vlo[t] / vhi[t], 3), ut), ut)
        # the fixed schedule that reaches the learned error: Chebyshev degree d + k Newton steps
        match = None
        for d in (1, 2, 3, 4):
            h = pe(he.invsqrt_guess_fit(vlo[t] / vhi[t], d), ut)
            for k in range(4):
                if rms(h, ut) <= e_l and (match is None or depth_of[d] + 2 * k < match[0]):
                    match = (depth_of[d] + 2 * k, d, k)
                h = 1.5 * h - 0.5 * ut * h ** 3
        per_t.append({"iteration": t, "variances_in_domain": int(inside.sum()), "train_samples": ntr,
                      "train_loss": loss, "heldout_rms_learned_deg4": e_l, "heldout_rms_chebyshev_deg3": e_f,
                      "fixed_depth_to_match_learned": match[0] if match else None,
                      "fixed_schedule_to_match": f"degree {match[1]} + {match[2]} Newton" if match else None})
    log(f"[bench] learned guesses trained in {t_train:.1f} s: {per_t}")
    xs = [llm_logits_var(5000 + r) for r in range(16)]
    cts = [ctx.encrypt(x) for x in xs]
    out = {}
    for name, deg, coef in (("learned", 4, coefs), ("fixed", 3, None)):
        cfg = he.CutmaxCfg(T=3, p=[3] * 3, c=[5.0] * 3, var_lo=vlo, var_hi=vhi, init_degree=deg, init_coef=coef,
                           sum_lo=1.0, sum_hi=3.0, gold_d=2)
        ctx.cutmax(cts, cfg)
        ctx.sync()
        t1 = time.perf_counter()
        Z = ctx.cutmax(cts, cfg)
        ctx.sync()
        ms = (time.perf_counter() - t1) * 1e3
        picks = [int(np.argmax(ctx.decrypt(Z[r], xs[r].size))) for r in range(16)]
        ok = sum(int(picks[r] == int(np.argmax(xs[r]))) for r in range(16))
        out[name] = {"init_degree": deg, "guess_depth": depth_of[deg], "levels_used": ctx.L - Z[0].level,
                     "levels_left": Z[0].level, "ms_per_batch16": ms, "argmax_agreement": f"{ok}/16",
                     "picks": picks}
        del Z
    return {"logged_runs": args.learned_runs, "logged_variances": int(v.size), "log_s": t_log,
            "train_s": t_train, "epochs": args.learned_epochs, "domains": {"var_lo": vlo, "var_hi": vhi},
            "per_iteration": per_t, "batch16": out,
            "same_picks": out["learned"]["picks"] == out["fixed"]["picks"]}


# The paper's HE schedule (Table 2, Sec. 4 "HE CutMax"): T = 4, p = [16, 4, 4, 6], c = [5, 3, 3, 3].
# Variance domains and mean(y^(T)) bounds declared from 100 synthetic prompts per vocabulary
# size with margins; iterations 2-4 refine their guess with K scaled steps.
TABLE2 = {
    32768: dict(vlo=[12.0, 1e7, 4e6, 6e7], vhi=[24.0, 4e12, 1.6e10, 1.6e10], K=[0, 7, 5, 3],
                sum_lo=1.5e5, sum_hi=2.5e6, gold_d=6, paper_ms=3373.0, paper_max_z=0.994),
    151936: dict(vlo=[15.0, 2e6, 5e8, 2e10], vhi=[30.0, 8e10, 2e12, 2e12], K=[0, 6, 5, 3],
                 sum_lo=1e7, sum_hi=5e7, gold_d=5, paper_ms=4607.0, paper_max_z=0.989),
}


def table2_bench(he, bctx, prompts):
    """The Table 2 schedule encrypted on the bootstrappable set (error-corrected bootstraps
    where the 15 CutMax levels run out, also inside the wide-domain inverse square root), at
    32768 logits (1 ciphertext) and 151936 (5): ms per CutMax, mean max Z and argmax accuracy
    over `prompts` synthetic prompts, against the paper's H100 figures (context only)."""
    from workloads import llm_logits
    bctx.boot_setup(he.BootCfg(ratio_bits=6, correct_bits=6))
    out = {}
    for V, d in TABLE2.items():
        coef, steps, ranges = [], [], []
        for t in range(4):
            g, st, rg = he.invsqrt_scaled_plan(d["vlo"][t] / d["vhi"][t], 3, d["K"][t])
            coef.append(list(g))
            steps.append(st)
            ranges.append(rg)
        cfg = he.CutmaxCfg(T=4, p=[16, 4, 4, 6], c=[5.0, 3.0, 3.0, 3.0], var_lo=d["vlo"], var_hi=d["vhi"],
                           init_degree=3, init_coef=coef, sum_lo=d["sum_lo"], sum_hi=d["sum_hi"],
                           gold_d=d["gold_d"], flags=he.HE_BOOT | he.HE_REFINE_SCALED, ref_steps=steps,
                           ref_range=ranges)
        ms, mz, ok = [], [], 0
        for s in range(prompts):
            x = llm_logits(700 + s, V)
            ct = bctx.encrypt(x)
            bctx.cutmax([ct], cfg)            # first call: encodes the bootstrap's diagonals
            bctx.sync()
            t0 = time.perf_counter()
            Z = bctx.cutmax([ct], cfg)[0]
            bctx.sync()
            ms.append((time.perf_counter() - t0) * 1e3)
            z = bctx.decrypt(Z, V)
            mz.append(float(z.max()))
            ok += int(int(np.argmax(z)) == int(np.argmax(x)))
            del ct, Z
        out[str(V)] = {"ciphertexts": -(-V // bctx.slots), "ms_per_cutmax": float(np.median(ms)),
                       "mean_max_Z": float(np.mean(mz)), "argmax_accuracy": f"{ok}/{prompts}",
                       "refinement_steps": d["K"], "paper_ms_H100": d["paper_ms"], "paper_max_Z": d["paper_max_z"]}
        log(f"[bench] Table 2 schedule at {V} logits: {out[str(V)]}")
    bctx.boot_setup(he.BootCfg(ratio_bits=6))
    return out


def batch_bench(ctx, cfg, args):
    """Batched argmaxes/s: 16 requests, even ids 32000 logits (1 ciphertext), odd ids 128256
    logits (4 ciphertexts), all advancing through one schedule (every launch covers the 40
    ciphertexts)."""
    from workloads import llm_logits
    xs = [llm_logits(200 + r, 32000 if r % 2 == 0 else 128256) for r in range(16)]
    cts = [ctx.encrypt(v) for v in xs]
    ctx.cutmax(cts, cfg)
    ctx.sync()
    tb0 = time.perf_counter()
    for _ in range(args.batch_steps):
        Zb = ctx.cutmax(cts, cfg)
    ctx.sync()
    tb1 = time.perf_counter()
    per_batch = (tb1 - tb0) / args.batch_steps
    ok = sum(int(np.argmax(ctx.decrypt(Zb[r], xs[r].size)) == int(np.argmax(xs[r]))) for r in range(16))
    batch = {"requests": 16, "ciphertexts": sum(c.a for c in cts), "ms_per_batch": per_batch * 1e3,
             "argmaxes_per_s": 16.0 / per_batch, "device_ms": ctx.last_cutmax_ms(), "argmax_ok": ok}
    if not args.no_profile:
        ctx.profile_begin()
        ctx.cutmax(cts, cfg)
        kb = ctx.profile_end()
        batch["kernels"] = {k: {"launches": v[0], "ms": v[1], "bytes": v[2]} for k, v in kb.items()}
    log(f"[bench] batch {batch}")
    del cts, Zb
    return batch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched and the 151936-logit measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-boot", action="store_true",
                    help="skip the bootstrapping measurements (separate bootstrappable context)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 16-request batch (profiling runs of the batched kernels)")
    ap.add_argument("--boot-only", action="store_true",
                    help="only the bootstrapping measurements (profiling runs of the bootstrap)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess measurement")
    ap.add_argument("--learned-runs", type=int, default=1000000,
                    help="plaintext CutMax runs logged for the learned guess (one variance per iteration each)")
    ap.add_argument("--learned-epochs", type=int, default=10)
    ap.add_argument("--table2-prompts", type=int, default=4,
                    help="prompts per vocabulary size for the paper's Table 2 schedule (bootstrapped; 0 skips)")
    ap.add_argument("--graph", type=int, default=1,
                    help="replay each CutMax from a captured HIP graph (1) or launch eagerly (0)")
    ap.add_argument("--hoist", type=int, default=None,
                    help="rotate-and-sum radix log2 (default: the parameter set's)")
    ap.add_argument("--cpu-T", type=int, default=3, help="iterations of the oracle sample (1..3)")
    ap.add_argument("--violation", metavar="S,D", default=None,
                    help="instead of the CutMax benchmark, measure the violation rate of the encrypted "
                         "Gumbel-max and Beta-cut samplers over S prompts x D draws")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                          "(requests shard across GPUs with no exchange between them)"}))
        sys.exit(2)
    if args.violation:
        violation_main(args.violation, args.graph)
        return

    import torch
    from paper_2509_08383_amd import he
    from workloads import llm_logits

    assert torch.cuda.is_available(), "no GPU"
    digest = src_digest()
    if args.boot_only:
        print(json.dumps({"bootstrapping": boot_bench(he, args, llm_logits(0, VOCAB2))}))
        return
    log("[bench] context N=2^16")
    prm = he.SECURE if args.hoist is None else dataclasses.replace(he.SECURE, hoist=args.hoist)
    ctx = he.Context(prm, device=0)
    if args.graph:
        ctx.set_option(he.HE_OPT_GRAPH, 1)
    cfg = cfg_secure(he)
    if args.batch_only:
        bb = batch_bench(ctx, cfg, args)
        # the plain copy that calibrates the byte counters of profiling runs
        cms = ctx.bench_copy(64, 10)
        print(json.dumps({"batched": bb, "copy_ms": cms, "src_digest": digest}))
        return
    x = llm_logits(0, VOCAB2)
    ct = ctx.encrypt(x)
    log("[bench] warmup")
    for _ in range(args.warmup):
        ctx.cutmax([ct], cfg)
    torch.cuda.synchronize()
    ctx.sync()
    log(f"[bench] timing {args.steps} steps")
    dev_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Z = ctx.cutmax([ct], cfg)[0]
        dev_ms.append(ctx.last_cutmax_ms())
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    z = ctx.decrypt(Z, VOCAB2)
    argmax_ok = int(np.argmax(z)) == int(np.argmax(x))
    log(f"[bench] {ms_per_step:.3f} ms/step (device {np.median(dev_ms):.3f} ms), argmax ok={argmax_ok}")

    # --- per-kernel roofline (HIP events around every launch, one extra step)
    roof = None
    kern = {}
    if not args.no_profile:
        ctx.profile_begin()
        ctx.cutmax([ct], cfg)
        kern = ctx.profile_end()
        tot = sum(v[1] for v in kern.values())
        dom = max(kern.items(), key=lambda kv: kv[1][1])
        name = dom[0]
        launches, ms_total, bytes_total = dom[1]
        achieved = (bytes_total / (ms_total * 1e-3)) / 1e9 if bytes_total > 0 else None
        pm = pmc_entry(name, digest)
        traffic = None
        if pm and "fetch_MiB" in pm and "write_MiB" in pm:
            traffic = (pm["fetch_MiB"] + pm["write_MiB"]) * 2**20
        roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "alg_bytes_per_launch": bytes_total / launches, "launches": launches,
                "avg_launch_ms": ms_total / launches, "share_of_kernel_time": ms_total / tot,
                "valu_frac": pm.get("valu_util") if pm else None}
        log(f"[bench] dominant kernel {name}: {launches} launches, {ms_total:.3f} ms, {achieved} GB/s")

    # --- NTT GB/s (algorithmic 2 N 8 bytes per limb-NTT)
    ntt = {}
    for cts_n in (1, 8, 40):
        vec = cts_n * 2 * (ctx.L + 1)
        f, i = ctx.bench_ntt(vec, 5)
        alg = 2.0 * ctx.N * 8 * vec
        ntt[f"{cts_n}ct"] = {"vectors": vec, "fwd_ms": f, "inv_ms": i, "fwd_GBps": alg / (f * 1e-3) / 1e9,
                             "inv_GBps": alg / (i * 1e-3) / 1e9}
    log(f"[bench] ntt {ntt}")
    # the same transforms at N = 2^12 (the toy chain's ring degree, 36 limbs a polynomial)
    tctx = he.Context(he.TOY, device=0)
    ntt_4096 = {}
    for cts_n in (1, 8, 40):
        vec = cts_n * 2 * (tctx.L + 1)
        f, i = tctx.bench_ntt(vec, 5)
        alg = 2.0 * tctx.N * 8 * vec
        ntt_4096[f"{cts_n}ct"] = {"vectors": vec, "fwd_ms": f, "inv_ms": i, "fwd_GBps": alg / (f * 1e-3) / 1e9,
                                  "inv_GBps": alg / (i * 1e-3) / 1e9}
    del tctx
    log(f"[bench] ntt at N=2^12 {ntt_4096}")

    # --- plain copy of 64 limb vectors (32 MiB read + 32 MiB written per launch): the
    # achievable-bandwidth reference, and the known-size kernel that calibrates byte counters
    cms = ctx.bench_copy(64, 10)
    copy = {"vectors": 64, "bytes_per_launch": 2 * 64 * ctx.N * 8, "ms": cms,
            "GBps": 2 * 64 * ctx.N * 8 / (cms * 1e-3) / 1e9}
    log(f"[bench] copy {copy}")

    # --- the largest vocabulary of the paper's experiments (151936 logits, 5 ciphertexts)
    vocab_151936 = None
    if not args.no_batch:
        xq = llm_logits(300, 151936)
        ctq = ctx.encrypt(xq)
        ctx.cutmax([ctq], cfg)
        ctx.sync()
        tq0 = time.perf_counter()
        for _ in range(3):
            Zq = ctx.cutmax([ctq], cfg)[0]
        ctx.sync()
        tq1 = time.perf_counter()
        vocab_151936 = {"ciphertexts": ctq.a, "ms": (tq1 - tq0) * 1e3 / 3,
                        "argmax_ok": int(np.argmax(ctx.decrypt(Zq, xq.size))) == int(np.argmax(xq))}
        log(f"[bench] 151936 logits {vocab_151936}")
        del ctq, Zq

    # --- batched argmaxes/s (16 mixed-vocabulary requests)
    batch = None
    if not args.no_batch:
        batch = batch_bench(ctx, cfg, args)

    # --- the learned initial guess against the fixed schedule (16 requests)
    learned = None
    if not args.no_learned and not args.no_batch:
        learned = learned_bench(he, ctx, args)
        log(f"[bench] learned {learned['batch16']}")

    # --- CPU oracle: the whole encrypted CutMax on the host's cores, and a bounded
    # single-thread sample (one top-level rotate-and-sum) scaled by the same sample's
    # all-core time
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(prm, x, ctx, args)
        log(f"[bench] cpu {cpu}")

    boot = None
    if not args.no_boot:
        boot = boot_bench(he, args, x)

    out = {
        "metric": "ms per encrypted 32k-logit CutMax argmax",
        "value": ms_per_step,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "encrypted CutMax, N=2^16 RNS-CKKS 128-bit (30x Q, dnum=3), "
                               "one ciphertext of 32000 LLM-like logits in 32768 slots, T=3, p=3, c=5",
                   "global_batch": 1, "seq_len": VOCAB2, "parallelism": "none"},
        "device_ms_median": float(np.median(dev_ms)),
        "rotsum_hoist_log2": prm.hoist,
        "hip_graph": bool(args.graph),
        "src_digest": digest,
        "argmax_ok": bool(argmax_ok),
        "batched": batch,
        "learned_guess": learned,
        "vocab_151936": vocab_151936,
        "ntt": ntt,
        "ntt_n4096": ntt_4096,
        "copy": copy,
        "ntt_tuning": ctx.ntt_tuning(),
        "ntt_tuning_report": ctx.ntt_tuning_report(),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "ms": v[1], "bytes": v[2]} for k, v in kern.items()},
        "cpu_baseline": cpu,
        "bootstrapping": boot,
        "paper_reference": {"value_ms": 3373.0, "hardware": "1x NVIDIA H100 (HELayers)",
                            "note": "T=4, p=[16,4,4,6], c=[5,3,3,3], |V|=32768, unstated CKKS parameters; "
                                    "context only, not like-for-like"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
