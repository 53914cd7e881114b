#!/usr/bin/env python3
"""Benchmark of the fused-pack GEMM on one MI355X.

Headline workload (one "step" = one fused-pack GEMM call):
    binary64 C := 1.5 * A B + 0.5 * C, m = n = k = 8192, column-major, no transpose,
    lda = ldb = ldc = 8192, entries uniform [-1, 1] (seeded, synthetic).
value = GFLOP/s (2mnk flops per step) of the fused-pack path.  The JSON line also
carries the roofline position of the GEMM kernel, the oracle timed on the host
cores over a bounded sample of the same workload, and a size sweep comparing
fused-pack, pack-then-compute (fip_pack + CONSUME_ONLY) and unpacked (NONE)
paths in FP64 and FP32 (median over interleaved rounds; pack-then-compute time includes
its pack launch).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-cpu-baseline]
                    [--no-mx] [--no-autograd] [--no-batched]

With the sweep come cold-cache timings (a 512 MB write before each timed call) beside the
hot ones, and graph-replayed per-call times for tiny sizes.
Further sections of the same JSON line: the mixed-precision forms (bfloat16, FP8 E4M3,
3- and 2-term bfloat16 splits) at m = n = k in {1024, 4096, 16384} with their error
against the binary64 oracle; the bfloat16 autograd linear layer (8192 x 4096 x 4096,
forward and backward); the 10,000-problem batched binary32 GEMM (eager and graph).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X dense MFMA peaks
METRIC = "GFLOP/s & % of MFMA peak vs size: fused-pack vs pack-then-compute"
SWEEP_SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]
KERNEL_SOURCES = ["paper_2302_08417_amd/csrc/fipgemm_kernels.hip",
                  "paper_2302_08417_amd/csrc/fipgemm_api.cpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic(name):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernel."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _pmc_rows(folder, counter):
    """(kernel name, grid size, value) of every dispatch in a rocprofv3 --pmc csv output."""
    import csv
    path = os.path.join(folder, "run_counter_collection.csv")
    with open(path, newline="") as f:
        return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
                for r in csv.DictReader(f) if r["Counter_Name"] == counter]


def write_traffic_summary(args, fetch_dir, write_dir, cfetch_dir, cwrite_dir):
    """HBM bytes per launch of the headline GEMM kernel from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for a device copy of known size."""
    import statistics
    n, dt = args.size, args.dtype
    ctype = "double" if dt == "f64" else "float"

    def gemm_mean(folder, counter):
        rows = [r for r in _pmc_rows(folder, counter)
                if f"::gemm_kernel<{ctype}," in r[0]]
        if not rows:
            raise SystemExit(f"no gemm_kernel<{ctype}, ...> dispatch in {folder}")
        grid = max(r[1] for r in rows)          # the headline launch is the largest
        vals = [r[2] for r in rows if r[1] == grid]
        name = [r[0] for r in rows if r[1] == grid][0]
        return statistics.mean(vals), len(vals), name

    def copy_kib(folder, counter):
        rows = [r for r in _pmc_rows(folder, counter) if "copyBuffer" in r[0]]
        if not rows:
            raise SystemExit(f"no copy kernel dispatch in {folder}")
        return statistics.median(r[2] for r in rows)

    probe = 1 << 30
    fetch, nf, name = gemm_mean(fetch_dir, "FETCH_SIZE")
    write, nw, _ = gemm_mean(write_dir, "WRITE_SIZE")
    cf, cw = copy_kib(cfetch_dir, "FETCH_SIZE"), copy_kib(cwrite_dir, "WRITE_SIZE")
    fs, ws = probe / (cf * 1024), probe / (cw * 1024)
    rd, wr = fetch * 1024 * fs, write * 1024 * ws
    esize = 8 if dt == "f64" else 4
    rec = {
        "kernel": name.replace("void fip::(anonymous namespace)::", "").split("(")[0],
        "workload": f"fused-pack {'DGEMM' if dt == 'f64' else 'SGEMM'} m=n=k={n} column-major NN, "
                    "AUTO policy",
        "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1),
        "copy_probe_bytes": probe, "copy_fetch_kib": round(cf, 1), "copy_write_kib": round(cw, 1),
        "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
        "hbm_read_bytes_per_launch": int(rd), "hbm_write_bytes_per_launch": int(wr),
        "hbm_bytes_per_launch": int(rd + wr),
        "algorithmic_bytes_per_launch": esize * 4 * n * n,
        "dispatches_averaged": min(nf, nw),
        "kernel_source_sha256": kernel_source_hash(),
    }
    out = os.path.join(ROOT, "profiles", f"traffic_gemm_{dt}_{n}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


class Gemm:
    """One prepared GEMM (device operands + a handle per policy) timed with HIP events."""

    def __init__(self, F, torch, n, dtype, seed, layout=0, tA="N", tB="N", m=None, k=None,
                 ld_pad=0):
        import numpy as np
        from paper_2302_08417_amd import synth
        self.F, self.torch = F, torch
        self.m, self.n, self.k = (m or n), n, (k or n)
        np_dt = np.float64 if dtype == "f64" else np.float32
        c = synth.make_case(layout, self.m, self.n, self.k, tA, tB, ld_pad=ld_pad, alpha=1.5,
                            beta=0.5, dtype=np_dt, seed=seed)
        self.case = c
        self.A = torch.from_numpy(c.A).to("cuda")
        self.B = torch.from_numpy(c.B).to("cuda")
        self.C = torch.from_numpy(c.C).to("cuda")
        self.dt = F.FIP_F64 if dtype == "f64" else F.FIP_F32
        self.fn = F.fip_dgemm if dtype == "f64" else F.fip_sgemm
        self.handles = {}

    def handle(self, policy):
        F = self.F
        if policy not in self.handles:
            h = F.Handle(policy=policy)
            c = self.case
            p = h.plan(self.dt, c.layout, c.m, c.n, c.k, c.transA, c.transB)
            h.ensure_workspace(p.workspace_bytes)
            h.bind_stream()
            self.handles[policy] = h
        return self.handles[policy]

    def call(self, policy):
        c, F = self.case, self.F
        h = self.handle(policy)
        if policy == F.FIP_PACK_CONSUME_ONLY:
            rc = F.fip_pack(h.h, self.dt, c.layout, c.m, c.n, c.k, self.A, c.lda, c.transA, self.B,
                            c.ldb, c.transB)
            if rc:
                raise F.FipError("fip_pack", rc)
        rc = self.fn(h.h, c.layout, c.m, c.n, c.k, c.alpha, self.A, c.lda, c.transA, self.B, c.ldb,
                     c.transB, c.beta, self.C, c.ldc)
        if rc:
            raise F.FipError(self.fn.__name__, rc)

    def time(self, policy, reps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.call(policy)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            self.call(policy)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps  # ms per call

    def flops(self):
        return 2.0 * self.m * self.n * self.k

    def release(self):
        for h in self.handles.values():
            h.close()
        self.handles.clear()


def time_interleaved(g, policies, rounds=11, warmup=3, batch_s=0.01):
    """Median per-call time (ms) of each policy.  Every round times one batch of each policy,
    alternating the order between rounds, so that clock ramps and drift hit all of them alike."""
    import statistics
    est = g.flops() / (40e12 if g.case.A.dtype.itemsize == 8 else 80e12) + 5e-6
    reps = max(1, min(200, int(batch_s / est)))
    for pol in policies:
        g.time(pol, 1, warmup)
    times = {pol: [] for pol in policies}
    for r in range(rounds):
        for pol in (policies if r % 2 == 0 else policies[::-1]):
            times[pol].append(g.time(pol, reps, 0))
    return {pol: statistics.median(v) for pol, v in times.items()}, rounds * reps


# name, dtype code, MFMA peak (TFLOP/s), products, C tile (-1: the planner's choice)
MX_FORMS = [("bf16", 2, 2516.6, 1, -1), ("e4m3", 3, 5033.2, 1, -1), ("e4m3_tile256", 3, 5033.2, 1, 256),
            ("bf16x3", 4, 2516.6, 6, -1), ("bf16x3_fast", 5, 2516.6, 3, -1)]


def _median_times(torch, calls, rounds, reps):
    """Median per-call ms of each callable, interleaved over rounds (HIP events)."""
    import statistics
    times = {k: [] for k in calls}
    for r in range(rounds):
        for key in (list(calls) if r % 2 == 0 else list(calls)[::-1]):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                calls[key]()
            b.record()
            torch.cuda.synchronize()
            times[key].append(a.elapsed_time(b) / reps)
    return {k: statistics.median(v) for k, v in times.items()}


def mx_section(F, torch, sizes, forms=None):
    """Mixed-precision forms, square column-major NN, alpha = 1, beta = 0, C binary32:
    fused (AUTO) vs pack-then-compute vs unpacked, and the error of the fused result on a
    sampled 32 x 32 block of C against the binary64 oracle product of the binary32 values
    the operands were made from (max |dC| / max |A||B|)."""
    import numpy as np
    import oracle
    from paper_2302_08417_amd import synth
    out = []
    for n in sizes:
        for name, dt, peak, prods, tile in MX_FORMS:
            if forms and name not in forms:
                continue
            if tile == 256 and n < 4096:
                continue      # a forced 256 tile on fewer tiles than CUs says nothing
            A, B, sa, sb, A32, B32 = synth.mx_device_operands(dt, n, seed=synth.BASE_SEED + n)
            C = torch.zeros(n, n, device="cuda")
            hs = {pol: F.Handle(policy=pol) for pol in (F.FIP_PACK_AUTO, F.FIP_PACK_CONSUME_ONLY,
                                                         F.FIP_PACK_NONE)}
            for h in hs.values():
                h.set_attr(F.FIP_ATTR_MX_TILE, tile)

            def mk(pol):
                h = hs[pol]

                def call():
                    if pol == F.FIP_PACK_CONSUME_ONLY:
                        h.pack(0, n, n, n, A, n, "N", B, n, "N", dtype=dt)
                    h.gemm_mx(dt, 0, n, n, n, 1.0, A, n, "N", B, n, "N", 0.0, C, n, sa, sb)
                return call
            calls = {pol: mk(pol) for pol in hs}
            for c in calls.values():
                c()
            torch.cuda.synchronize()
            est = 2.0 * n ** 3 * prods / (peak * 0.25e12)
            med = _median_times(torch, calls, 5, max(1, min(50, int(0.01 / est))))
            calls[F.FIP_PACK_AUTO]()
            torch.cuda.synchronize()
            g = np.random.default_rng(n + dt)
            ri = np.sort(g.choice(n, 32, replace=False))
            ci = np.sort(g.choice(n, 32, replace=False))
            # A32[p, i] holds A(i, p) (column-major storage); B32[j, p] holds B(p, j)
            subA = A32[:, torch.as_tensor(ri, device="cuda")].double().cpu().numpy()  # k x 32
            subB = B32[torch.as_tensor(ci, device="cuda"), :].double().cpu().numpy()  # 32 x k
            got = C[torch.as_tensor(ci, device="cuda")][:, torch.as_tensor(ri, device="cuda")]
            got = got.double().cpu().numpy().T                                          # 32 x 32
            Aop = np.ascontiguousarray(subA.T).reshape(-1, order="F")                   # 32 x k
            Bop = np.ascontiguousarray(subB.T).reshape(-1, order="F")                   # k x 32
            ref, D = oracle.gemm(0, 32, 32, n, 1.0, Aop, 32, "N", Bop, n, "N", 0.0,
                                 np.zeros(32 * 32), 32)
            err = float(np.abs(got - ref.reshape(32, 32, order="F")).max() / D.max())
            fl = 2.0 * n ** 3
            row = {"form": name, "m": n, "n": n, "k": n,
                   "tile": hs[F.FIP_PACK_AUTO].last_plan().MT}
            for key, pol in (("fused", F.FIP_PACK_AUTO), ("pack_then_compute", F.FIP_PACK_CONSUME_ONLY),
                             ("no_pack", F.FIP_PACK_NONE)):
                row[key + "_us"] = round(med[pol] * 1e3, 2)
                row[key + "_tflops"] = round(fl / (med[pol] * 1e-3) / 1e12, 1)
            row["mfma_peak_tflops"] = peak
            row["fused_pct_mfma_peak"] = round(100 * row["fused_tflops"] * prods / peak, 2)
            if dt == F.FIP_E4M3 and tile == -1:
                # fip_quantize_fp8 of the binary32 operands (per row of op(A), per column of
                # op(B); four launches each), timed on its own
                hq = hs[F.FIP_PACK_AUTO]
                Qa = torch.empty(n * n, dtype=torch.uint8, device="cuda")
                Qb = torch.empty_like(Qa)
                qsa = torch.empty(n, device="cuda")
                qsb = torch.empty(n, device="cuda")

                def quant():
                    hq.quantize_fp8(0, n, n, A32, n, 0, Qa, n, qsa)
                    hq.quantize_fp8(0, n, n, B32, n, 1, Qb, n, qsb)
                quant()
                torch.cuda.synchronize()
                tq = _median_times(torch, {"q": quant}, 5, 5)["q"]
                row["quantize_both_us"] = round(tq * 1e3, 2)
                row["quantize_gbs"] = round(2 * n * n * (4 + 4 + 1) / (tq * 1e-3) / 1e9, 1)
                del Qa, Qb
            row["err_vs_fp64_oracle_rel_to_max_absAB"] = float(f"{err:.3e}")
            log(f"[mx] {row}")
            out.append(row)
            for h in hs.values():
                h.close()
            del A, B, A32, B32, C
            torch.cuda.empty_cache()
    return out


MX_DEEP_K = [(256, 256, 8192), (128, 512, 16384)]


def mx_deep_k_section(F, torch):
    """Mixed-precision forms on few tiles with a deep k (column-major NN, alpha = 1,
    beta = 0): fused with the planner's k split, fused unsplit, pack-then-compute and no-pack
    (both with the planner's split), in microseconds.  Operands: N(0, 1) binary32 (split
    forms) or rounded to bfloat16; E4M3 codes drawn uniformly from the finite codes of
    magnitude <= 120 with unit scales."""
    out = []
    for (m, n, k) in MX_DEEP_K:
        for name, dt, peak, prods, tile in MX_FORMS:
            if tile != -1:
                continue
            g = torch.Generator(device="cuda").manual_seed(m + n + k + dt)
            if dt == F.FIP_E4M3:
                A = torch.randint(0, 0x70, (m * k,), device="cuda", generator=g, dtype=torch.uint8)
                B = torch.randint(0, 0x70, (k * n,), device="cuda", generator=g, dtype=torch.uint8)
                A |= (torch.randint(0, 2, (m * k,), device="cuda", generator=g, dtype=torch.uint8) << 7)
                B |= (torch.randint(0, 2, (k * n,), device="cuda", generator=g, dtype=torch.uint8) << 7)
            else:
                A = torch.randn(m * k, device="cuda", generator=g)
                B = torch.randn(k * n, device="cuda", generator=g)
                if dt == F.FIP_BF16:
                    A, B = A.to(torch.bfloat16), B.to(torch.bfloat16)
            C = torch.zeros(m * n, device="cuda")
            legs = {"fused": (F.FIP_PACK_AUTO, -1), "fused_unsplit": (F.FIP_PACK_AUTO, 1),
                    "pack_then_compute": (F.FIP_PACK_CONSUME_ONLY, -1),
                    "no_pack": (F.FIP_PACK_NONE, -1)}
            hs = {}
            for key, (pol, split) in legs.items():
                hs[key] = F.Handle(policy=pol)
                hs[key].set_attr(F.FIP_ATTR_SPLIT_K, split)

            def mk(key):
                h, pol = hs[key], legs[key][0]

                def call():
                    if pol == F.FIP_PACK_CONSUME_ONLY:
                        h.pack(0, m, n, k, A, m, "N", B, k, "N", dtype=dt)
                    h.gemm_mx(dt, 0, m, n, k, 1.0, A, m, "N", B, k, "N", 0.0, C, m)
                return call
            calls = {key: mk(key) for key in legs}
            for c in calls.values():
                c()
            torch.cuda.synchronize()
            est = 2.0 * m * n * k * prods / (peak * 0.25e12)
            med = _median_times(torch, calls, 5, max(1, min(50, int(0.01 / est))))
            row = {"form": name, "m": m, "n": n, "k": k,
                   "split_k": hs["fused"].last_plan().split_k}
            for key in legs:
                row[key + "_us"] = round(med[key] * 1e3, 2)
            row["fused_speedup_vs_pack_then_compute"] = round(med["pack_then_compute"] / med["fused"], 3)
            log(f"[mx deep k] {row}")
            out.append(row)
            for h in hs.values():
                h.close()
            del A, B, C
            torch.cuda.empty_cache()
    return out


def autograd_section(F, torch):
    """bfloat16 linear layer, forward Y = X W^T and backward dX = dY W, dW = dY^T X, all
    through the fused-pack GEMM: X 8192 x 4096 ~ N(0,1), W 4096 x 4096 ~ N(0, 1/4096),
    dY ~ N(0,1)."""
    from paper_2302_08417_amd import autograd as AG
    g = torch.Generator(device="cuda").manual_seed(3)
    X = torch.randn(8192, 4096, device="cuda", generator=g).to(torch.bfloat16).requires_grad_()
    W = (torch.randn(4096, 4096, device="cuda", generator=g) / 64).to(torch.bfloat16)
    W.requires_grad_()
    dY = torch.randn(8192, 4096, device="cuda", generator=g).to(torch.bfloat16)

    def step():
        X.grad = None
        W.grad = None
        AG.fip_linear(X, W).backward(dY)
    step()
    torch.cuda.synchronize()
    t = _median_times(torch, {"s": step}, 7, 5)["s"]
    fl = 3 * 2.0 * 8192 * 4096 * 4096
    res = {"workload": "bf16 linear fwd+bwd X 8192x4096, W 4096x4096", "ms_per_step": round(t, 4),
           "tflops": round(fl / (t * 1e-3) / 1e12, 1),
           "pct_bf16_mfma_peak": round(100 * fl / (t * 1e-3) / 2516.6e12, 2)}
    log(f"[autograd] {res}")
    return res


def batched_section(F, torch, count=10000):
    """10,000 binary32 problems, m, n, k log-uniform in [4, 512], random transposes, ragged
    storage through device pointer arrays, alpha = 1.5, beta = 0.5; tile threshold from the
    autotuner; eager launch and graph replay."""
    from paper_2302_08417_amd import synth
    from paper_2302_08417_amd.batched import DeviceBatch
    b = synth.make_batch(count, synth.COL, lo=4, hi=512, seed=synth.BASE_SEED + 3)
    db = DeviceBatch(b)
    h = F.Handle()
    split = db.tune(h)
    db.run(h)
    db.run(h, graph=True)
    torch.cuda.synchronize()
    med = _median_times(torch, {"eager": lambda: db.run(h), "graph": lambda: db.run(h, graph=True)},
                        7, 10)
    m, n, k = (x.astype("float64") for x in (b.m, b.n, b.k))
    fl = float((2 * m * n * k).sum())
    nbytes = float((4 * (m * k + k * n + 2 * m * n)).sum())
    res = {"workload": f"{count} fp32 problems, m,n,k log-uniform [4,512], random transposes",
           "tuned_split": split, "total_gflop": round(fl / 1e9, 3),
           "algorithmic_gbytes": round(nbytes / 1e9, 4)}
    for key in ("eager", "graph"):
        t = med[key]
        res[key + "_us"] = round(t * 1e3, 1)
        res[key + "_tflops"] = round(fl / (t * 1e-3) / 1e12, 2)
        res[key + "_algorithmic_gbs"] = round(nbytes / (t * 1e-3) / 1e9, 1)
    res["pct_hbm_peak_graph"] = round(100 * res["graph_algorithmic_gbs"] / 8000.0, 2)
    log(f"[batched] {res}")
    return res


VARIANTS_ALL = [(layout, tA, tB, pad) for layout in (0, 1) for tA in "NT" for tB in "NT"
                for pad in (0, 7)]
VARIANTS_FEW = [(0, "N", "N", 0), (0, "T", "N", 7), (1, "N", "T", 0), (1, "T", "T", 7)]


def _policy_names(F):
    return {F.FIP_PACK_AUTO: "fused", F.FIP_PACK_CONSUME_ONLY: "pack_then_compute",
            F.FIP_PACK_NONE: "no_pack"}


def _time_row(F, torch, g, row, rounds, batch_s):
    names = _policy_names(F)
    med, calls = time_interleaved(g, list(names), rounds=rounds, batch_s=batch_s)
    row["calls_per_variant"] = calls
    for pol, name in names.items():
        t = med[pol]
        row[name + "_us"] = round(t * 1e3, 2)
        row[name + "_gflops"] = round(g.flops() / (t * 1e-3) / 1e9, 2)
    row["fused_speedup_vs_pack_then_compute"] = round(row["pack_then_compute_us"] / row["fused_us"], 3)
    return row


def sweep_section(F, torch, sizes, dtypes):
    """Square m = n = k sweep, fused vs pack-then-compute vs unpacked: every combination of
    layout, transposes and ld in {rows, rows + 7} up to 1024, four of them above."""
    from paper_2302_08417_amd import synth
    out = []
    for sdt in dtypes:
        for s in sizes:
            for layout, tA, tB, pad in (VARIANTS_ALL if s <= 1024 else VARIANTS_FEW):
                g = Gemm(F, torch, s, sdt, seed=synth.BASE_SEED + 17 * s, layout=layout, tA=tA,
                         tB=tB, ld_pad=pad)
                row = {"dtype": sdt, "m": s, "n": s, "k": s, "layout": "col" if layout == 0 else "row",
                       "trans": tA + tB, "ld_pad": pad}
                _time_row(F, torch, g, row, rounds=5, batch_s=0.003 if s <= 1024 else 0.01)
                row["fused_pct_peak"] = round(100 * row["fused_gflops"] / (PEAK_TFLOPS[sdt] * 1e3), 2)
                log(f"[sweep] {row}")
                out.append(row)
                g.release()
                del g
            torch.cuda.empty_cache()
    return out


def skinny_section(F, torch, dtypes):
    """Skinny shapes (HBM-bound): every layout / transpose / ld variant; algorithmic GB/s =
    elem (mk + kn + 2mn) / time."""
    from paper_2302_08417_amd import synth
    out = []
    for sdt in dtypes:
        es = 8 if sdt == "f64" else 4
        for (m, n, k) in ((4096, 4096, 32), (32, 4096, 4096), (4096, 32, 4096)):
            for layout, tA, tB, pad in VARIANTS_ALL:
                g = Gemm(F, torch, n, sdt, seed=synth.BASE_SEED + m + 3 * n + 7 * k, layout=layout,
                         tA=tA, tB=tB, m=m, k=k, ld_pad=pad)
                row = {"dtype": sdt, "m": m, "n": n, "k": k, "layout": "col" if layout == 0 else "row",
                       "trans": tA + tB, "ld_pad": pad}
                _time_row(F, torch, g, row, rounds=5, batch_s=0.003)
                nbytes = es * (m * k + k * n + 2 * m * n)
                row["fused_algorithmic_gbs"] = round(nbytes / (row["fused_us"] * 1e-6) / 1e9, 1)
                row["fused_pct_hbm_peak"] = round(100 * row["fused_algorithmic_gbs"] / 8000.0, 2)
                log(f"[skinny] {row}")
                out.append(row)
                g.release()
                del g
        torch.cuda.empty_cache()
    return out


LDIM_SIZES = [16, 32, 64, 128, 256, 512, 1024, 2000]


def ldim_section(F, torch):
    """The paper's second sweep (Sec. 4): m = n = k <= 2000 with every leading dimension 2000,
    column-major NN, binary64 and binary32; fused vs pack-then-compute vs unpacked."""
    from paper_2302_08417_amd import synth
    out = []
    for sdt in ("f64", "f32"):
        for s in LDIM_SIZES:
            g = Gemm(F, torch, s, sdt, seed=synth.BASE_SEED + 29 * s, ld_pad=2000 - s)
            row = {"dtype": sdt, "m": s, "n": s, "k": s, "ld": 2000}
            _time_row(F, torch, g, row, rounds=5, batch_s=0.003)
            row["fused_pct_peak"] = round(100 * row["fused_gflops"] / (PEAK_TFLOPS[sdt] * 1e3), 2)
            log(f"[ldim2000] {row}")
            out.append(row)
            g.release()
            del g
        torch.cuda.empty_cache()
    return out


def l3_section(F, torch, sizes=(4096, 8192)):
    """SYRK (C := 1.5 A A^T + 0.5 C, lower, column-major 'N', k = n), TRMM (C := 1.5 T B +
    0.5 C, side L, lower, no transpose, non-unit) and TRSM (T X = 1.5 C in place, side L,
    lower, no transpose) through the fused-pack tile kernel in FP64 and FP32: fused (AUTO)
    against unpacked (NONE) and fused with every panel packed (ALL).  flops: n^2 k for SYRK
    (one triangle), m^2 n for TRMM and TRSM (half the square)."""
    import statistics
    from paper_2302_08417_amd import synth
    out = []
    for dt in ("f64", "f32"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        for n in sizes:
            g = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + n)
            A = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            B = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            C = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            # TRSM's triangle: lower, off-diagonal U[-1, 1] / 2n, diagonal 1.5 (well
            # conditioned; with alpha = 1.5 the solution keeps B's magnitude call after call)
            T = (A.view(n, n) / (2 * n)).clone()
            T.diagonal().fill_(1.5)
            T = T.reshape(-1)
            for op in ("syrk", "trmm", "trsm"):
                hs = {key: F.Handle(policy=pol) for key, pol in
                      (("fused", F.FIP_PACK_AUTO), ("no_pack", F.FIP_PACK_NONE),
                       ("fused_all", F.FIP_PACK_ALL))}

                def mk(h):
                    if op == "syrk":
                        return lambda: h.syrk(0, "L", "N", n, n, 1.5, A, n, 0.5, C, n)
                    if op == "trsm":
                        return lambda: h.trsm(0, "L", "L", "N", "N", n, n, 1.5, T, n, C, n)
                    return lambda: h.trmm(0, "L", "L", "N", "N", n, n, 1.5, A, n, B, n, 0.5, C, n)
                calls = {key: mk(h) for key, h in hs.items()}
                for c in calls.values():
                    c()
                torch.cuda.synchronize()
                fl = float(n) ** 3
                est = fl / (60e12 if dt == "f64" else 120e12)
                med = _median_times(torch, calls, 5, max(1, min(20, int(0.02 / est))))
                row = {"op": op, "dtype": dt, "n": n, "k_or_m": n}
                for key in calls:
                    row[key + "_us"] = round(med[key] * 1e3, 1)
                row["fused_tflops"] = round(fl / (med["fused"] * 1e-3) / 1e12, 2)
                row["fused_pct_peak"] = round(100 * row["fused_tflops"] / PEAK_TFLOPS[dt], 2)
                p = hs["fused"].last_plan()
                row["fused_pack"] = [p.pack_a, p.a_pack_first]
                log(f"[l3] {row}")
                out.append(row)
                for h in hs.values():
                    h.close()
            del A, B, C
            torch.cuda.empty_cache()
    return out


def dma_section(F, torch, sizes=(2048, 4096, 8192)):
    """Direct global -> LDS loads (FIP_ATTR_DMA) against the register path, FP64 and FP32,
    square column-major NN, alpha = 1.5, beta = 0.5: unpacked (NONE) and pack-then-compute
    (fip_pack + a CONSUME_ONLY call that fetches the packed chunks), each with the attribute
    off and on; every launch here is eligible, so "on" runs the DMA variant."""
    from paper_2302_08417_amd import synth
    out = []
    for dt in ("f64", "f32"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        for n in sizes:
            g = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 5 * n)
            A = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            B = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            C = torch.rand(n * n, device="cuda", generator=g, dtype=tdt) * 2 - 1
            hs = {}
            for pol, pname in ((F.FIP_PACK_NONE, "no_pack"), (F.FIP_PACK_CONSUME_ONLY, "pack_then_compute")):
                for dma in (0, 1):
                    h = F.Handle(policy=pol)
                    h.set_attr(F.FIP_ATTR_DMA, dma)
                    hs[f"{pname}_{'dma' if dma else 'reg'}"] = (h, pol)

            def mk(h, pol):
                def f():
                    if pol == F.FIP_PACK_CONSUME_ONLY:
                        h.pack(F.FIP_COL_MAJOR, n, n, n, A, n, "N", B, n, "N")
                    h.gemm(F.FIP_COL_MAJOR, n, n, n, 1.5, A, n, "N", B, n, "N", 0.5, C, n)
                return f
            calls = {key: mk(h, pol) for key, (h, pol) in hs.items()}
            for c in calls.values():
                c()
            torch.cuda.synchronize()
            used = {key: h.get_attr(F.FIP_ATTR_LAST_DMA) for key, (h, _) in hs.items()}
            fl = 2.0 * float(n) ** 3
            est = fl / (60e12 if dt == "f64" else 120e12)
            med = _median_times(torch, calls, 5, max(1, min(50, int(0.02 / est))))
            row = {"dtype": dt, "n": n}
            for key in calls:
                row[key + "_us"] = round(med[key] * 1e3, 1)
            row["dma_speedup_no_pack"] = round(med["no_pack_reg"] / med["no_pack_dma"], 3)
            row["dma_speedup_pack_then_compute"] = round(
                med["pack_then_compute_reg"] / med["pack_then_compute_dma"], 3)
            row["dma_pct_peak_no_pack"] = round(100 * fl / (med["no_pack_dma"] * 1e-3) / 1e12 /
                                                PEAK_TFLOPS[dt], 2)
            row["ran_dma"] = [used[k] for k in sorted(used)]
            log(f"[dma] {row}")
            out.append(row)
            for h, _ in hs.values():
                h.close()
            del A, B, C
            torch.cuda.empty_cache()
    return out


def cx_section(F, torch, sizes=(1024, 2048, 4096)):
    """Complex GEMM through the 1m method (fip_zgemm, fip_cgemm): C := alpha A B + beta C,
    column-major NN, alpha = 1.5 - 0.5i, beta = 0.5 + 0.25i, re and im U[-1, 1]; fused
    (AUTO) vs pack-then-compute (fip_pack + CONSUME_ONLY) vs unpacked.  flops: 8 m n k (a
    complex multiply-add is 8 real flops; the 1m expansion multiplies 2m x 2k by 2k x n, the
    same count)."""
    from paper_2302_08417_amd import synth
    out = []
    al, be = 1.5 - 0.5j, 0.5 + 0.25j
    for dt in ("z", "c"):
        tdt = torch.complex128 if dt == "z" else torch.complex64
        rdt = torch.float64 if dt == "z" else torch.float32
        for n in sizes:
            g = torch.Generator(device="cuda").manual_seed(synth.BASE_SEED + 3 * n)

            def draw():
                return torch.complex(torch.rand(n * n, device="cuda", generator=g, dtype=rdt) * 2 - 1,
                                     torch.rand(n * n, device="cuda", generator=g, dtype=rdt) * 2 - 1)
            A, B, C = draw().to(tdt), draw().to(tdt), draw().to(tdt)
            hs = {key: F.Handle(policy=pol) for key, pol in
                  (("fused", F.FIP_PACK_AUTO), ("pack_then_compute", F.FIP_PACK_CONSUME_ONLY),
                   ("no_pack", F.FIP_PACK_NONE))}

            def mk(key, h):
                if key == "pack_then_compute":
                    def f():
                        h.pack(F.FIP_COL_MAJOR, n, n, n, A, n, "N", B, n, "N")
                        h.zgemm(F.FIP_COL_MAJOR, n, n, n, al, A, n, "N", B, n, "N", be, C, n)
                    return f
                return lambda: h.zgemm(F.FIP_COL_MAJOR, n, n, n, al, A, n, "N", B, n, "N", be, C, n)
            calls = {key: mk(key, h) for key, h in hs.items()}
            for c in calls.values():
                c()
            torch.cuda.synchronize()
            fl = 8.0 * float(n) ** 3
            est = fl / (60e12 if dt == "z" else 120e12)
            med = _median_times(torch, calls, 5, max(1, min(50, int(0.02 / est))))
            row = {"dtype": dt, "n": n}
            for key in calls:
                row[key + "_us"] = round(med[key] * 1e3, 1)
            row["fused_tflops"] = round(fl / (med["fused"] * 1e-3) / 1e12, 2)
            row["fused_pct_peak"] = round(100 * row["fused_tflops"] / PEAK_TFLOPS["f64" if dt == "z" else "f32"], 2)
            row["fused_vs_ptc"] = round(med["pack_then_compute"] / med["fused"], 3)
            p = hs["fused"].last_plan()
            row["fused_pack"] = [p.pack_a, p.pack_b]
            log(f"[cx] {row}")
            out.append(row)
            for h in hs.values():
                h.close()
            del A, B, C
            torch.cuda.empty_cache()
    return out


def plain_dgemm_section(F, torch):
    """C := A B + C, m = n = k = 256, column-major NN, alpha = beta = 1 (FP64)."""
    from paper_2302_08417_amd import synth
    g = Gemm(F, torch, 256, "f64", seed=synth.BASE_SEED + 1)
    g.case.alpha, g.case.beta = 1.0, 1.0
    row = {"dtype": "f64", "m": 256, "n": 256, "k": 256, "alpha": 1.0, "beta": 1.0}
    _time_row(F, torch, g, row, rounds=7, batch_s=0.003)
    row["fused_pct_peak"] = round(100 * row["fused_gflops"] / (PEAK_TFLOPS["f64"] * 1e3), 3)
    log(f"[plain] {row}")
    g.release()
    return row


def cpu_oracle_rate(n, target_s):
    """GFLOP/s of the oracle, as it stands, on a column sample of the m = n = k = n binary64
    workload grown until it takes about target_s; returns (GFLOP/s, columns, seconds, threads)."""
    import numpy as np
    import oracle
    from paper_2302_08417_amd import synth
    c = synth.make_case(0, n, n, n, "N", "N", alpha=1.5, beta=0.5, dtype=np.float64,
                        seed=synth.BASE_SEED + n)
    A = c.A

    def run(cols):
        B = c.B[: c.ldb * cols]
        C = c.C[: c.ldc * cols]
        t = time.perf_counter()
        oracle.gemm(0, n, cols, n, c.alpha, A, c.lda, "N", B, c.ldb, "N", c.beta, C, c.ldc)
        return time.perf_counter() - t

    cols = 1
    t = run(cols)
    while t < 0.5 * target_s and cols < n:  # grow the sample until it takes about target_s
        cols = int(max(cols + 1, min(n, cols * target_s / max(t, 1e-3))))
        t = run(cols)
    return 2.0 * n * cols * n / t / 1e9, cols, t, oracle.num_threads()


def cpu_oracle_sizes(sizes=(256, 512, 1024, 2048, 4096), batch=2000):
    """Context for the CPU baseline: the oracle on whole square binary64 problems (column-major
    NN, every entry of C) at each size, and on the first `batch` problems of the 10,000-problem
    batched workload (binary32 operands, the oracle computes in binary64), all threads.  Only
    timed here, never a reference for anything."""
    import numpy as np
    import oracle
    from paper_2302_08417_amd import synth
    out = {"threads": oracle.num_threads(), "square_gflops": {}}
    for n in sizes:
        c = synth.make_case(0, n, n, n, "N", "N", alpha=1.5, beta=0.5, dtype=np.float64,
                            seed=synth.BASE_SEED + n)
        t = time.perf_counter()
        oracle.gemm(0, n, n, n, c.alpha, c.A, c.lda, "N", c.B, c.ldb, "N", c.beta, c.C, c.ldc)
        dt = time.perf_counter() - t
        out["square_gflops"][str(n)] = round(2.0 * n ** 3 / dt / 1e9, 3)
    b = synth.make_batch(batch, synth.COL, lo=4, hi=512, seed=synth.BASE_SEED + 3)
    fl = 0.0
    t = time.perf_counter()
    for i in range(batch):
        m, n, k = int(b.m[i]), int(b.n[i]), int(b.k[i])
        oracle.gemm(0, m, n, k, b.alpha, b.A[i], int(b.lda[i]), chr(b.transA[i]), b.B[i],
                    int(b.ldb[i]), chr(b.transB[i]), b.beta, b.C[i], int(b.ldc[i]))
        fl += 2.0 * m * n * k
    dt = time.perf_counter() - t
    out["batched_sample"] = {"problems": batch, "gflops": round(fl / dt / 1e9, 3),
                             "seconds": round(dt, 2)}
    return out


def cpu_baseline(n, target_s=10.0, one_thread_s=6.0):
    """The oracle timed on the host: all the threads OpenMP gives it, and one thread (in a child
    process started with OMP_NUM_THREADS=1, so the setting cannot leak into this one)."""
    import subprocess
    gf, cols, t, threads = cpu_oracle_rate(n, target_s)
    res = {"value": round(gf, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"binary64 oracle (triple loop, ascending-k sums, plus the |A||B| bound) on "
                     f"C[:, :{cols}] of the m=n=k={n} workload ({t:.1f} s)",
           "host_cpus": len(os.sched_getaffinity(0))}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", str(n),
                        str(one_thread_s)], env=env, capture_output=True, text=True, timeout=300)
    if p.returncode == 0 and p.stdout.strip():
        leg = json.loads(p.stdout.strip().splitlines()[-1])
        res["one_thread"] = {"value": leg["gflops"], "cores": leg["threads"],
                             "sample": f"C[:, :{leg['cols']}] ({leg['seconds']:.1f} s)"}
    return res


def cache_section(F, torch):
    """FP64, fused vs pack-then-compute: "hot" per-call times (repeated calls) beside "cold" ones
    (a 512 MB write before every call evicts the XCD L2s and the 256 MB Infinity Cache; only the
    call is timed), and for tiny sizes the per-call time of 100 calls replayed from one captured
    graph beside the eager launch."""
    import statistics
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    cold = []
    for m, n, k in [(256, 256, 256), (1024, 1024, 1024), (4096, 4096, 4096), (32, 4096, 4096)]:
        g = Gemm(F, torch, n, "f64", seed=71 + n + k, m=m, k=k)
        row = {"m": m, "n": n, "k": k}
        for pol, name in ((F.FIP_PACK_AUTO, "fused"), (F.FIP_PACK_CONSUME_ONLY,
                                                         "pack_then_compute")):
            reps = 20 if m * n * k >= 4096 ** 3 else 50
            row[f"{name}_hot_us"] = round(1e3 * g.time(pol, reps, 3), 2)
            ts = []
            for r in range(reps):
                flush.fill_(r & 0xFF)
                a, b = ev(), ev()
                a.record()
                g.call(pol)
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            row[f"{name}_cold_us"] = round(1e3 * statistics.median(ts), 2)
        row["cold_fused_speedup_vs_pack_then_compute"] = round(
            row["pack_then_compute_cold_us"] / row["fused_cold_us"], 3)
        log(f"[cold] {row}")
        cold.append(row)
        g.release()
    graph = []
    for n in (16, 64, 256):
        g = Gemm(F, torch, n, "f64", seed=91 + n)
        eager_us = 1e3 * g.time(F.FIP_PACK_AUTO, 200, 10)
        h = g.handle(F.FIP_PACK_AUTO)
        c = g.case
        gr = torch.cuda.CUDAGraph()
        calls = 100
        with torch.cuda.graph(gr):
            h.bind_stream()
            for _ in range(calls):
                rc = g.fn(h.h, c.layout, c.m, c.n, c.k, c.alpha, g.A, c.lda, c.transA, g.B, c.ldb,
                          c.transB, c.beta, g.C, c.ldc)
                if rc:
                    raise F.FipError(g.fn.__name__, rc)
        h.bind_stream()
        gr.replay()
        torch.cuda.synchronize()
        ts = []
        for r in range(5):
            a, b = ev(), ev()
            a.record()
            gr.replay()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e3 / calls)
        row = {"n": n, "eager_us_per_call": round(eager_us, 2),
               "graph_us_per_call": round(statistics.median(ts), 2)}
        log(f"[graph] {row}")
        graph.append(row)
        g.release()
    del flush
    torch.cuda.empty_cache()
    return {"cold": cold, "graph_replay": graph}


SUMMARY_MAX_BYTES = 2000


def compact_summary(result, full):
    """Short per-section summaries for the final stdout line (the full rows go to the results
    file and to stderr)."""
    s = {}
    if "sweep" in full:
        rows = full["sweep"] + full["skinny"] + full.get("ldim2000", [])
        sp = [r["fused_speedup_vs_pack_then_compute"] for r in rows]
        s["sweep_summary"] = {
            "rows": len(rows),
            "rows_fused_faster_than_pack_then_compute": sum(x > 1.0 for x in sp),
            "min_fused_speedup": min(sp), "median_fused_speedup": sorted(sp)[len(sp) // 2],
            "fused_pct_peak_nn_col": {
                f"{r['dtype']}_{r['m']}": r["fused_pct_peak"] for r in full["sweep"]
                if r["m"] >= 4096 and r["layout"] == "col" and r["trans"] == "NN"
                and r["ld_pad"] == 0}}
    if "mixed_precision" in full:
        big = max(r["m"] for r in full["mixed_precision"])
        s["mixed_precision"] = {
            r["form"]: {"n": big, "pct_peak": r["fused_pct_mfma_peak"],
                        "vs_ptc": round(r["pack_then_compute_us"] / r["fused_us"], 3)}
            for r in full["mixed_precision"] if r["m"] == big and "tile256" not in r["form"]}
    if "level3" in full:
        s["l3_pct_peak"] = {f"{r['op']}_{r['dtype']}_{r['n']}": r["fused_pct_peak"]
                                   for r in full["level3"] if r["n"] == 8192}
    if "dma" in full:
        s["dma_speedup"] = {f"{r['dtype']}_{r['n']}": [r["dma_speedup_no_pack"],
                                                        r["dma_speedup_pack_then_compute"]]
                            for r in full["dma"] if r["n"] == 8192}
    if "complex_1m" in full:
        s["complex_1m"] = {f"{r['dtype']}gemm_{r['n']}": [r["fused_pct_peak"], r["fused_vs_ptc"]]
                           for r in full["complex_1m"] if r["n"] == 4096}
    if "autograd" in full:
        s["autograd"] = {k: full["autograd"][k] for k in ("ms_per_step", "pct_bf16_mfma_peak")}
    if "batched" in full:
        s["batched"] = {k: full["batched"][k] for k in ("eager_us", "graph_us",
                                                         "pct_hbm_peak_graph")}
    for key, val in s.items():
        trial = dict(result, **{key: val})
        if len(json.dumps(trial)) <= SUMMARY_MAX_BYTES:
            result = trial
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-sizes", default=None,
                    help="comma-separated sizes for the sweep (default: 16..8192 powers of two)")
    ap.add_argument("--sweep-dtypes", default="f64,f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mx", action="store_true", help="skip the mixed-precision section")
    ap.add_argument("--mx-sizes", default="1024,4096,16384")
    ap.add_argument("--mx-forms", default=None,
                    help="comma-separated subset of bf16,e4m3,bf16x3,bf16x3_fast (default: all)")
    ap.add_argument("--no-mx-deep", action="store_true", help="skip the mixed deep-k shapes")
    ap.add_argument("--no-autograd", action="store_true")
    ap.add_argument("--no-l3", action="store_true", help="skip the SYRK / TRMM section")
    ap.add_argument("--no-cx", action="store_true", help="skip the complex (1m) section")
    ap.add_argument("--no-dma", action="store_true", help="skip the LDS-DMA section")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--results", default=os.path.join("gpurun_out", "bench_full.json"),
                    help="file that receives every section's rows (the stdout line carries\n"
                         "only their summaries); empty string: do not write it")
    ap.add_argument("--cpu-leg", nargs=2, default=None, metavar=("N", "SECONDS"),
                    help="no GPU work: time the oracle on a column sample of the N^3 workload\n"
                         "for about SECONDS and print one JSON line (used for the one-thread leg)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times), to "
                         "calibrate HBM byte counters against a kernel of known traffic")
    ap.add_argument("--traffic-summary", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="no GPU work: read four rocprofv3 --pmc output folders (FETCH_SIZE and\n"
                         "WRITE_SIZE of the headline run, then of the --copy-probe run) and write\n"
                         "profiles/traffic_gemm_<dtype>_<size>.json for the roofline 'traffic'")
    args = ap.parse_args()

    if args.traffic_summary:
        write_traffic_summary(args, *args.traffic_summary)
        return
    if args.cpu_leg:
        gf, cols, t, threads = cpu_oracle_rate(int(args.cpu_leg[0]), float(args.cpu_leg[1]))
        print(json.dumps({"gflops": round(gf, 3), "cols": cols, "seconds": round(t, 2),
                          "threads": threads}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs a GEMM on a single MI355X, "
              "and sharding across GPUs is described as a design, not implemented; "
              "use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2302_08417_amd import fipgemm as F
    from paper_2302_08417_amd import synth

    if args.copy_probe:
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "reads": args.copy_probe,
                          "writes": args.copy_probe}), flush=True)
        return

    n, dt = args.size, args.dtype
    log(f"[bench] headline: fused-pack {dt} gemm m=n=k={n}")
    g = Gemm(F, torch, n, dt, seed=synth.BASE_SEED + n)
    ms = g.time(F.FIP_PACK_AUTO, args.steps, args.warmup)
    plan = g.handle(F.FIP_PACK_AUTO).last_plan()
    flops = g.flops()
    value = flops / (ms * 1e-3) / 1e9
    achieved_tf = value / 1e3
    log(f"[bench] {ms:.3f} ms/step, {value:.1f} GFLOP/s ({achieved_tf / PEAK_TFLOPS[dt]:.1%} of peak)")
    g.release()
    del g
    torch.cuda.empty_cache()

    traffic = load_traffic(f"traffic_gemm_{dt}_{n}.json")
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {
            "workload": f"fused-pack {'DGEMM' if dt == 'f64' else 'SGEMM'} m=n=k={n}, column-major, "
                        f"no transpose, ld=rows, alpha=1.5, beta=0.5, entries U[-1,1]",
            "m": n, "n": n, "k": n, "tile": f"{plan.MT}x{plan.NT}x{plan.KT}",
            "pack_a": plan.pack_a, "pack_b": plan.pack_b, "pack_copies": plan.copies,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved_tf, 3),
            "peak": PEAK_TFLOPS[dt],
            "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_TFLOPS[dt], 4),
            "traffic": traffic,
        },
    }

    full = {}
    if not args.no_sweep:
        full["plain_dgemm_256"] = plain_dgemm_section(F, torch)
        sizes = [int(x) for x in args.sweep_sizes.split(",")] if args.sweep_sizes else SWEEP_SIZES
        full["sweep"] = sweep_section(F, torch, sizes, args.sweep_dtypes.split(","))
        full["skinny"] = skinny_section(F, torch, args.sweep_dtypes.split(","))
        full["ldim2000"] = ldim_section(F, torch)
        full["cache_and_graph"] = cache_section(F, torch)
    if not args.no_mx:
        forms = args.mx_forms.split(",") if args.mx_forms else None
        full["mixed_precision"] = mx_section(F, torch, [int(x) for x in args.mx_sizes.split(",")],
                                             forms)
        if not args.no_mx_deep:
            full["mixed_precision_deep_k"] = mx_deep_k_section(F, torch)
    if not args.no_l3:
        full["level3"] = l3_section(F, torch)
    if not args.no_cx:
        full["complex_1m"] = cx_section(F, torch)
    if not args.no_dma:
        full["dma"] = dma_section(F, torch)
    if not args.no_autograd:
        full["autograd"] = autograd_section(F, torch)
    if not args.no_batched:
        full["batched"] = batched_section(F, torch)

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(n)
        full["cpu_oracle_sizes"] = cpu_oracle_sizes()
        log(f"[bench] cpu oracle sizes {full['cpu_oracle_sizes']}")
    if args.results:
        os.makedirs(os.path.dirname(os.path.abspath(args.results)), exist_ok=True)
        with open(args.results, "w") as f:
            json.dump(dict(result, sections=full), f, indent=1)
        log(f"[bench] every section's rows: {args.results}")
    result = compact_summary(result, full)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
