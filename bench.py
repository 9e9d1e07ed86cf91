"""Benchmark of the OK-operator hot path on one MI355X.

Workload: 20^3 x 64 lattice (512,000 sites), random SU(3) links U = exp(i eps H)
with eps tuned to an average plaquette of 0.6, tadpole u0 from the plaquette,
the stand-in coefficient set at m0 a = 0.5, and the 12 spin-colour point
sources at the origin.

One step = one application of M (ok_apply_M) to the 12-right-hand-side batch,
with the chosen storage of W (FP32 by default), which runs the MFMA kernel
(one launch for the 12 right-hand sides).  The metric is the HBM throughput of
that application in algorithmic bytes (the dense W streamed once + 12 spinors
read and 12 written, per site), timed with HIP events on the stream the
library launches on.  The second half of the metric, time to
||xi - M psi||/||xi|| <= 1e-10, is measured on the same batch: "plain" = FP64
BiCGStab with 27 dense FP64 blocks, one right-hand side after the other;
"chosen" = the fastest of the other solve forms (median of three solves each),
each reported with its solution's error against the plain FP64 solution and the
HBM roofline fraction of the whole solve (solve_bytes below).

Prints one JSON line.  --gpus N > 1 is refused (single-GPU build).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (20, 20, 20, 64)
V = 20 * 20 * 20 * 64
NRHS = 12
# algorithmic bytes per site of one single-right-hand-side application: dense
# 27 x 12x12 complex W + spinor in + spinor out
BYTES_SITE = {0: 27 * 144 * 16 + 2 * 192, 1: 27 * 144 * 8 + 2 * 96, 2: 27 * 144 * 4 + 2 * 96}
# the 14-block saved set (OK_LAYOUT_SAVED): each stored block read once from HBM
BYTES_SAVED = {0: 14 * 144 * 16 + 2 * 192, 1: 14 * 144 * 8 + 2 * 96, 2: 14 * 144 * 4 + 2 * 96}
# W as 46 Pauli-component colour matrices per site (OK_LAYOUT_SIGMA), each read once from HBM
BYTES_SIGMA = {0: 46 * 9 * 16 + 2 * 192, 1: 46 * 9 * 8 + 2 * 96}
# ... and the sigma layout on the 12-RHS batch (FP32): W once + 12 spinors in and out
BYTES_SIGMA_MR = {1: 46 * 9 * 8 + NRHS * 2 * 96}
# ... and of one application to the 12-RHS batch by the MFMA kernel: W streamed
# once for all right-hand sides + 12 spinors in and out (FP64 W: 12 single launches)
BYTES_STEP = {0: NRHS * BYTES_SITE[0], 1: 27 * 144 * 8 + NRHS * 2 * 96, 2: 27 * 144 * 4 + NRHS * 2 * 96}
PREC_NAME = {0: "f64", 1: "f32", 2: "bf16"}
KERNEL_NAME = "k_apply"
# reliable-update threshold of the chosen form (FP32 W): an FP64 update when the FP32 residual has
# dropped by this factor.  At 20^3x64 (12 point sources) 0.1 / 0.03 / 0.01 / 0.003 / 0.001 / 0.0003
# gave 0.82 / 0.76 / 0.75 / 0.72 / 0.72 / 0.74 s with 94-98 iterations (the BF16-W forms keep 0.1:
# their operator is only accurate to ~2^-8, so an FP32 cycle cannot go much deeper).
CHOSEN_DELTA = 0.003


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_hash(kernel="k_apply"):
    """Hash of the sources of a kernel (its file plus the shared layout headers)."""
    h = hashlib.sha256()
    main = {"k_apply": "stencil.hip", "k_apply_sigma": "stencil_sigma.hip",
            "k_apply_sigma_mr": "stencil_sigma.hip"}.get(kernel, "stencil_mrhs.hip")
    for f in (main, "wlayout.h", "common.h"):
        with open(os.path.join(ROOT, "paper_1311_5029_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_path(kernel, form):
    return os.path.join(ROOT, "profiles", "%s_%s_20x20x20x64_traffic.json" % (kernel, form))


def load_traffic(kernel, form):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 PMC
    summary, or None when the kernel source changed since the counters were taken."""
    path = traffic_path(kernel, form)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha") != source_hash(kernel):
        return None
    return d.get("bytes_per_launch")


COPY_BYTES = 1 << 30


def is_apply_kernel(name, form, kernel="k_apply"):
    """Whether a (mangled or demangled) kernel name is the apply kernel of this form:
    k_apply<prec, threads-per-site, 0> (single RHS, no reduction epilogue),
    k_apply_site<prec, 1> (the batched MFMA kernel, site-major W, RHS-inner spinors)
    or k_apply_mrhs<prec> (batched, plane-major W)."""
    p = {"f64": 0, "f32": 1, "bf16": 2}[form]
    if kernel == "k_apply_site":
        return ("k_apply_site<%d, 1>" % p) in name or ("k_apply_siteILi%dELi1E" % p) in name
    if kernel == "k_apply_mrhs":
        return ("k_apply_mrhs<%d>" % p) in name or ("k_apply_mrhsILi%dE" % p) in name
    if kernel == "k_apply_saved":   # <prec, no epilogue>
        return ("k_apply_saved<%d, 0>" % p) in name or ("k_apply_savedILi%dELi0E" % p) in name
    if kernel in ("k_apply_sigma", "k_apply_sigma_mr"):   # <prec, no epilogue, right-hand-side-inner>
        mr = 1 if kernel == "k_apply_sigma_mr" else 0
        head = "k_apply_sigma<%d, 0, %d" % (p, mr)   # followed by '>' or by the waves-per-SIMD argument
        return (head + ">") in name or (head + ",") in name or ("k_apply_sigmaILi%dELi0ELi%dE" % (p, mr)) in name
    return any(("k_apply<%d, %d, 0>" % (p, t)) in name or ("k_applyILi%dELi%dELi0E" % (p, t)) in name
               for t in (1, 2, 4))


def copy_probe():
    """A plain 1 GiB device-to-device copy (one kernel of known traffic) used to
    calibrate the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _read_counters(d):
    """{(kernel, dispatch): {counter: value}} from the counter_collection CSVs under d."""
    import csv
    out = {}
    for dirpath, _, files in os.walk(d):
        for f in files:
            if not f.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(dirpath, f)) as fh:
                for row in csv.DictReader(fh):
                    key = (row.get("Kernel_Name", ""), row.get("Dispatch_Id", row.get("Correlation_Id", "")))
                    cn = row.get("Counter_Name")
                    out.setdefault(key, {})
                    out[key][cn] = out[key].get(cn, 0.0) + float(row.get("Counter_Value", 0.0))
    return out


def parse_pmc(fetch_dir, write_dir, form):
    """Average FETCH_SIZE + WRITE_SIZE (KiB per dispatch) of each apply kernel of this
    form, each counter scaled by its reading for the 1 GiB copy; writes one traffic
    summary per kernel found (consumed by the benchmark's roofline entry)."""
    prec = {"f64": 0, "f32": 1, "bf16": 2}[form]
    algo = {"k_apply": BYTES_SITE[prec] * V, "k_apply_mrhs": BYTES_STEP[prec] * V,
            "k_apply_site": BYTES_STEP[prec] * V, "k_apply_sigma": BYTES_SIGMA.get(prec, 0) * V,
            "k_apply_sigma_mr": BYTES_SIGMA_MR.get(prec, 0) * V}
    rows = {c: _read_counters(d) for c, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir))}
    for kernel in ("k_apply", "k_apply_mrhs", "k_apply_site", "k_apply_sigma", "k_apply_sigma_mr"):
        res = {}
        for cname in ("FETCH_SIZE", "WRITE_SIZE"):
            ker = [v[cname] for (k, _), v in rows[cname].items() if cname in v and is_apply_kernel(k, form, kernel)]
            cop = [v[cname] for (k, _), v in rows[cname].items() if "copy" in k.lower() and cname in v]
            # the 1 GiB calibration copy (the counters read 0.5 and 1 GiB for it), not the 4 GiB
            # bandwidth copy the benchmark also runs
            cop = [x for x in cop if 0.25 * COPY_BYTES < x * 1024 < 1.5 * COPY_BYTES]
            if not ker or not cop:
                break
            scale = COPY_BYTES / (1024.0 * float(np.median(cop)))
            res[cname] = {"kib_per_dispatch": float(np.mean(ker)), "dispatches": len(ker),
                          "copy_kib": float(np.median(cop)), "scale": scale,
                          "bytes_per_launch": float(np.mean(ker)) * 1024.0 * scale}
        if len(res) < 2:
            continue
        total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
        out = {"kernel": "%s<%s>" % (kernel, form), "lattice": list(DIMS), "bytes_per_launch": total,
               "algorithmic_bytes_per_launch": algo[kernel], "ratio_to_algorithmic": total / algo[kernel],
               "counters": res, "source_sha": source_hash(kernel)}
        with open(traffic_path(kernel, form), "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out, indent=1))


def summarize_trace(d, out_path, command):
    """Short text summary of a rocprofv3 --kernel-trace --stats run (top kernels by time)."""
    import csv
    import re
    files = [os.path.join(dp, f) for dp, _, fs in os.walk(d) for f in fs if f.endswith("kernel_stats.csv")]
    rows = list(csv.DictReader(open(files[0])))
    lines = ["# rocprofv3 kernel statistics", "", "command: " + command, "",
             "%-44s %6s %14s %10s %8s" % ("kernel", "calls", "avg ns", "total ms", "% time")]
    for r in rows[:16]:
        name = r["Name"].replace("okinv::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
        name = re.sub(r"\(.*", "", name).replace("void ", "")[:44]
        lines.append("%-44s %6s %14.0f %10.2f %8.2f" % (name, r["Calls"], float(r["AverageNs"]),
                                                        float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    for kernel, per_site in (("k_apply", BYTES_SITE), ("k_apply_site", BYTES_STEP), ("k_apply_saved", BYTES_SAVED),
                             ("k_apply_sigma", BYTES_SIGMA), ("k_apply_sigma_mr", BYTES_SIGMA_MR)):
        for form, prec in (("f64", 0), ("f32", 1), ("bf16", 2)):
            if prec not in per_site:
                continue
            for r in rows:
                if is_apply_kernel(r["Name"], form, kernel):
                    ns = float(r["AverageNs"])
                    gbs = per_site[prec] * V / ns
                    lines.append("")
                    lines.append("%s<%s> (%s): average %.0f ns per launch -> %.1f GB/s algorithmic "
                                 "(%d B/site x %d sites), %.1f%% of 8 TB/s"
                                 % (kernel, form, "12 RHS" if kernel in ("k_apply_site", "k_apply_sigma_mr")
                                    else "1 RHS", ns, gbs,
                                    per_site[prec], V, gbs / HBM_PEAK_GBS * 100))
                    break
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# Algorithmic bytes per site of the operator forms a solve launches (W read once + spinor in and out)
W_SITE = {"f64": 27 * 144 * 16, "f64_sigma": 46 * 9 * 16, "f32": 27 * 144 * 8, "f32_sigma": 46 * 9 * 8,
          "bf16": 27 * 144 * 4}
FIELD_PASSES_PER_ITER = 20   # BLAS-1 and operator field reads/writes per BiCGStab iteration and RHS
UPDATE_FIELD_PASSES = 12     # FP64 field passes of one reliable update (accumulate, residual, cast, restart)


def solve_bytes(form, stats):
    """Algorithmic HBM bytes per site of a whole solve, from its kernel sequence (csrc/solver.cpp):
    per BiCGStab iteration two operator applications (W once each) and 20 field passes per
    right-hand side (p update 4, s update 3, x/r update with its dots 7, the two operators' input,
    output and epilogue-dot fields 6); per reliable update one FP64 application (the sigma-layout
    FP64 W is read once per four right-hand sides) and 12 FP64 field passes; plus the final FP64
    check.  Batched forms iterate all 12 right-hand sides until the last converges, so their
    iteration count is the largest per-column one."""
    f = form["kind"]
    nrhs = NRHS
    its = [s["iterations"] for s in stats]
    ups = sum(s["reliable_updates"] for s in stats)
    w64 = W_SITE["f64_sigma" if form["w64_sigma"] else "f64"]
    if f == "plain":
        return sum(its) * (2 * w64 + FIELD_PASSES_PER_ITER * 192) + nrhs * (w64 + 4 * 192)
    wlo = W_SITE[form["wlo"]]
    fb = 96   # FP32 fields
    upd = UPDATE_FIELD_PASSES * 192
    if f == "mixed":
        return sum(its) * (2 * wlo + FIELD_PASSES_PER_ITER * fb) + ups * (w64 + upd) + nrhs * (w64 + 4 * 192)
    # batched: one W read per operator application for the whole group
    groups_w64 = (ups + 3) // 4 if form["w64_sigma"] else ups
    return (max(its) * (2 * wlo + FIELD_PASSES_PER_ITER * fb * nrhs) + groups_w64 * w64 + ups * upd
            + nrhs * (w64 + 4 * 192))


def host_record():
    """nproc, usable cores, CPU model and RAM of the host this runs on."""
    rec = {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    rec["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    rec["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return rec


def cpu_baseline(plain_iterations=None):
    """The FP64 oracle (route B, the operator composed from the links) on the bench's own
    workload: one application of M to the 12 point-source-shaped right-hand sides at
    20^3 x 64, evaluated as time slabs in one worker process per usable core (at most 16),
    with NumPy's own threads limited to one per worker.  Also the full oracle BiCGStab solve
    of the 4^4 configuration, and the oracle's 16^3 x 32 time to solution extrapolated from
    its measured application time."""
    from threadpoolctl import threadpool_limits

    from oracle.bicgstab import bicgstab
    from oracle.local import apply_slabs
    from oracle.route_b import OKOperatorB
    from paper_1311_5029_amd import inputs as I
    host = host_record()
    nproc = max(1, min(16, host["usable_cores"]))
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    cfg = I.make_config("batched_20x20x20x64", with_sources=False)
    U, c = cfg["U"], cfg["coeffs"]
    psi = I.gaussian_sources(DIMS, NRHS, I.SEED_SOURCES + 3)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        apply_slabs(U, psi, c, nproc=nproc)
        t_apply = time.perf_counter() - t0
        # C1: the whole oracle solve at 4^4
        c1 = I.make_config("dense_4x4x4x4")
        op1 = OKOperatorB(c1["U"], c1["coeffs"])
        t0 = time.perf_counter()
        _, info = bicgstab(op1.apply, c1["xi"][0], tol=1e-10)
        t_c1 = time.perf_counter() - t0
        # C2: one oracle application at 16^3 x 32 (slab-parallel), times 2 per iteration
        c2 = I.make_config("mixed_16x16x16x32")
        t0 = time.perf_counter()
        apply_slabs(c2["U"], c2["xi"][0], c2["coeffs"], nproc=nproc)
        t_c2 = time.perf_counter() - t0
    sites = NRHS * V
    out = {
        "value": round(BYTES_STEP[1] * V / t_apply / 1e9, 4),
        "unit": "GB/s (the bench's algorithmic bytes for the same 12-RHS application / the oracle's time)",
        "cores": nproc,
        "kind": "oracle",
        "sample": "one M.psi on 12 right-hand sides at 20^3x64 (the whole bench workload, one application): "
                  "route-B FP64 NumPy in %d slab processes, %.2f s including process start and data transfer; "
                  "%.0f RHS-sites/s" % (nproc, t_apply, sites / t_apply),
        "rhs_sites_per_s": round(sites / t_apply, 1),
        "host": host,
        "c1_4x4x4x4_solve": {"seconds": round(t_c1, 3), "iterations": info["iters"],
                             "true_rel_resid": info["true_rel_resid"], "threads": 1, "measured": True},
        "c2_16x16x16x32_seconds_per_iteration": round(2 * t_c2, 3),
    }
    if plain_iterations:
        out["extrapolated_plain_solve_seconds"] = round(2 * plain_iterations * V / (sites / t_apply), 1)
        out["extrapolated_note"] = ("oracle rate x 2 applications x %d BiCGStab iterations (the GPU plain "
                                    "solve's count over the 12 sources), not run" % plain_iterations)
    return out


def learned(args):
    """The learned preconditioner, trained on the GPU on the same gauge field.

    learned_24x24x24x64: 256 training pairs, 64 fresh Gaussian evaluation sources; each solved
        plain (FP64, unpreconditioned), mixed (FP32 W + FP64 reliable updates) with and without
        the network, and in batches of 16 (BF16 site-major W on the matrix cores) with and
        without the network.
    learned_batched_32x32x32x64: 12 point sources: plain FP64 one after the other vs the network + batched BF16
        on the matrix cores (12 together); the network is trained on 64 Gaussian pairs.
    Training pairs come from the batched solver: FP64 solutions with true residual <= 1e-10,
    the same criterion the plain solver stops at."""
    import torch

    from paper_1311_5029_amd import inputs as I
    from paper_1311_5029_amd import okinv as ok
    from paper_1311_5029_amd import train as TR

    torch.cuda.set_device(0)
    gauss_eval = args.workload == "learned_24x24x24x64"
    dims = tuple(args.dims) if args.dims else ((24, 24, 24, 64) if gauss_eval else (32, 32, 32, 64))
    V = int(np.prod(dims))
    n_train = args.n_train or (256 if gauss_eval else 64)
    n_eval = args.n_eval or (64 if gauss_eval else 12)
    SITE, SIGMA, INNER = ok.OK_LAYOUT_SITE, ok.OK_LAYOUT_SIGMA, ok.OK_SPINOR_RHS_INNER
    log("%s: links %s" % (args.workload, dims))
    cfg = I.make_config(args.workload, dims=dims, with_sources=False)
    c = cfg["coeffs"]
    links = ok.to_device_complex(cfg["U"])
    del cfg["U"]
    Ws = {}
    pre = {}
    for prec in ([ok.OK_F64, ok.OK_F32, ok.OK_BF16 | SITE, ok.OK_F64 | SIGMA, ok.OK_F32 | SIGMA] if gauss_eval
                 else [ok.OK_F64, ok.OK_BF16 | SITE, ok.OK_F64 | SIGMA, ok.OK_F32 | SIGMA]):
        Ws[prec] = ok.empty_bytes(ok.ok_W_bytes(dims, prec))
        scr = ok.empty_bytes(ok.ok_precompute_scratch_bytes(dims))
        torch.cuda.synchronize()
        t = time.perf_counter()
        ok.ok_precompute_W(dims, c, links, prec, Ws[prec], scr)
        torch.cuda.synchronize()
        pre[PREC_NAME[prec & 3] + ("_site" if prec & SITE else "_sigma" if prec & SIGMA else "")] = \
            time.perf_counter() - t
        del scr
    T = ok.empty_bytes(ok.ok_net_transports_bytes(dims))
    ok.ok_net_transports(dims, links, T)
    del links
    log("precompute s %s" % {k: round(v, 3) for k, v in pre.items()})

    lowb = ok.OK_BF16 | SITE
    lows = ok.OK_F32 | SIGMA | INNER   # the fastest batched solve: FP32 sigma W, sigma FP64 reliable updates
    xi32, psi32, pinfo = TR.solve_pairs(dims, c, Ws[ok.OK_F64 | SIGMA], Ws[ok.OK_F32 | SIGMA], lows, n_train,
                                        I.SEED_TRAIN, log=log, w64_layout=SIGMA, delta=CHOSEN_DELTA)
    torch.cuda.synchronize()
    t = time.perf_counter()
    net, hist = TR.train(dims, T, xi32, psi32, n_train, 1.0 / c.mhat, n_layers=4, steps=args.train_steps,
                         batch=16 if gauss_eval else 8, lr=3e-3, log=log)
    train_s = time.perf_counter() - t
    del xi32, psi32
    torch.cuda.empty_cache()

    def run(xi_host, low, with_net, nrhs, w64=0):
        lp = -1 if low is None else low
        nn = net if with_net else None
        work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(dims, nrhs, lp, nn))
        d_xi = ok.to_device_complex(xi_host)
        psi = torch.zeros_like(d_xi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the FP32 sigma-layout batched forms run at the chosen form's reliable-update threshold
        delta = CHOSEN_DELTA if low == lows else 0.1
        rc, st = ok.ok_bicgstab(dims, c, ok.SolverParams(tol=1e-10, delta=delta, W64_layout=w64),
                                Ws[ok.OK_F64 | w64], None if low is None else Ws[low & ~INNER], lp, d_xi, psi, nrhs,
                                work, net=nn)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, rc, st, psi.view(nrhs, -1)

    forms = {}

    def add(name, sec, rc, st, psi, ref=None):
        """ref: the plain FP64 solutions of the same sources ([nrhs][...] device), for the error"""
        f = forms.setdefault(name, {"seconds": [], "iterations": [], "status": [], "resid": [], "fallbacks": 0,
                                    "err": []})
        f["seconds"].append(sec)
        f["iterations"].extend(s["iterations"] for s in st)
        f["status"].append(rc)
        f["resid"].extend(s["true_rel_resid"] for s in st)
        f["fallbacks"] += sum(s["fallbacks"] for s in st)
        if ref is not None:
            e = torch.linalg.vector_norm(psi - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)
            f["err"].extend(e.tolist())

    if gauss_eval:
        for j, xi in enumerate(I.gaussian_source_batches(dims, n_eval, I.SEED_EVAL, 16)):
            plain = []
            for k in range(xi.shape[0]):
                r = run(xi[k], None, False, 1)
                add("plain_f64", *r)
                plain.append(r[3])
                for name, low, wn in (("mixed_f32", ok.OK_F32, False), ("mixed_f32_net", ok.OK_F32, True)):
                    add(name, *run(xi[k], low, wn, 1), ref=plain[-1])
            ref = torch.cat(plain)
            for name, wn in (("batched_bf16", False), ("batched_bf16_net", True)):
                add(name, *run(xi, lowb, wn, xi.shape[0]), ref=ref)
            for name, wn in (("batched_f32_sigma", False), ("batched_f32_sigma_net", True)):
                add(name, *run(xi, lows, wn, xi.shape[0], SIGMA), ref=ref)
            del plain, ref
            log("evaluated %d/%d: %s" % (min(n_eval, 16 * (j + 1)), n_eval,
                                         {k: (round(float(np.mean(v["iterations"])), 1), round(sum(v["seconds"]), 2))
                                          for k, v in forms.items()}))
    else:
        xi = I.point_sources(dims)
        plain = []
        for k in range(12):
            r = run(xi[k], None, False, 1)
            add("plain_f64", *r)
            plain.append(r[3])
        ref = torch.cat(plain)
        add("batched_bf16", *run(xi, lowb, False, 12), ref=ref)
        add("batched_bf16_net", *run(xi, lowb, True, 12), ref=ref)
        add("batched_f32_sigma", *run(xi, lows, False, 12, SIGMA), ref=ref)
        add("batched_f32_sigma_net", *run(xi, lows, True, 12, SIGMA), ref=ref)
        del plain, ref
        log("evaluated: %s" % {k: (round(float(np.mean(v["iterations"])), 1), round(sum(v["seconds"]), 2))
                               for k, v in forms.items()})

    summary = {}
    for name, f in forms.items():
        summary[name] = {"seconds_total": round(sum(f["seconds"]), 3),
                         "seconds_per_source": round(sum(f["seconds"]) / len(f["iterations"]), 4),
                         "iterations_mean": round(float(np.mean(f["iterations"])), 2),
                         "iterations_median": float(np.median(f["iterations"])),
                         "all_converged": all(r == ok.OK_SUCCESS for r in f["status"]),
                         "max_true_rel_resid": max(f["resid"]), "fallbacks": f["fallbacks"]}
        if f["err"]:   # against the plain FP64 solution of the same source
            summary[name]["rel_error_vs_plain_f64"] = {"max": max(f["err"]), "median": float(np.median(f["err"]))}
    plain = summary["plain_f64"]["seconds_per_source"]
    out = {
        "metric": "time to 1e-10 residual per source, plain FP64 vs learned preconditioner",
        "workload": "%dx%dx%dx%d, plaquette 0.6 links, %d %s sources" % (
            *dims, n_eval if gauss_eval else 12, "Gaussian evaluation" if gauss_eval else "point"),
        "n_gpus": 1, "unit": "s/source", "higher_is_better": False,
        "value": min(summary[k]["seconds_per_source"] for k in ("batched_bf16_net", "batched_f32_sigma_net")),
        "value_form": min(("batched_bf16_net", "batched_f32_sigma_net"),
                          key=lambda k: summary[k]["seconds_per_source"]),
        "speedup_vs_plain": {k: round(plain / v["seconds_per_source"], 3) for k, v in summary.items()},
        # what the network adds to the same batched solver, and what it costs to get
        "learned_gain_vs_same_solver": learned_gain(summary, train_s, pinfo),
        "forms": summary,
        "network": {"layers": 4, "hops": 27, "params_real": ok.ok_net_param_count(4), "precision": "f32",
                    "training_pairs": n_train, "pair_solves": pinfo,
                    "train_steps": args.train_steps, "train_seconds": round(train_s, 3),
                    "loss_history": hist},
        "precompute_seconds": {k: round(v, 3) for k, v in pre.items()},
        "u0": round(cfg["u0"], 6), "eps": round(cfg["eps"], 6),
        "data": "synthetic: random SU(3) links at plaquette 0.6; stand-in OK coefficients",
    }
    print(json.dumps(out), flush=True)


def learned_gain(summary, train_s, pinfo):
    """Per-source time of the batched FP32 sigma solver without / with the network, the one-time
    cost of the network (pair solves + training) and the number of sources after which it has
    paid for itself."""
    a = summary["batched_f32_sigma"]["seconds_per_source"]
    b = summary["batched_f32_sigma_net"]["seconds_per_source"]
    pair_s = float(pinfo.get("seconds", 0.0)) if isinstance(pinfo, dict) else 0.0
    cost = pair_s + train_s
    return {"seconds_per_source_without": a, "seconds_per_source_with": b, "ratio": round(a / b, 3),
            "one_time_seconds": round(cost, 2), "pair_solve_seconds": round(pair_s, 2),
            "train_seconds": round(train_s, 2),
            "break_even_sources": (round(cost / (a - b), 1) if a > b else None)}


def mixed(args):
    """16^3x32, plaquette 0.6, one Gaussian source: plain FP64 BiCGStab vs FP32 (and BF16) W with
    FP64 reliable updates, all to 1e-10; each mixed solution's error against the plain FP64 one."""
    import torch

    from paper_1311_5029_amd import inputs as I
    from paper_1311_5029_amd import okinv as ok

    torch.cuda.set_device(0)
    dims = tuple(args.dims) if args.dims else (16, 16, 16, 32)
    cfg = I.make_config("mixed_16x16x16x32", dims=dims)
    c = cfg["coeffs"]
    links = ok.to_device_complex(cfg["U"])
    Ws = {}
    SIGMA = ok.OK_LAYOUT_SIGMA
    for prec in (ok.OK_F64, ok.OK_F32, ok.OK_BF16, ok.OK_F64 | SIGMA, ok.OK_F32 | SIGMA):
        Ws[prec] = ok.empty_bytes(ok.ok_W_bytes(dims, prec))
        scr = ok.empty_bytes(ok.ok_precompute_scratch_bytes(dims))
        ok.ok_precompute_W(dims, c, links, prec, Ws[prec], scr)
        del scr
    xi = ok.to_device_complex(cfg["xi"][0])
    out = {"metric": "time to 1e-10 residual, plain FP64 vs mixed precision with FP64 reliable updates",
           "workload": "%dx%dx%dx%d, plaquette 0.6 links, one Gaussian source" % dims, "n_gpus": 1,
           "unit": "s", "forms": {}}
    sol = {}
    for name, low, w64 in (("plain_f64", None, 0), ("mixed_f32", ok.OK_F32, 0), ("mixed_bf16", ok.OK_BF16, 0),
                           ("plain_f64_sigma", None, SIGMA), ("mixed_f32_sigma", ok.OK_F32 | SIGMA, SIGMA),
                           ("mixed_f32_sigma_delta0.003", ok.OK_F32 | SIGMA, SIGMA)):
        delta = CHOSEN_DELTA if name.endswith("_delta0.003") else 0.1
        lp = -1 if low is None else low
        work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(dims, 1, lp))
        best = None
        for _ in range(3):   # median of three solves
            psi = torch.zeros_like(xi)
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, st = ok.ok_bicgstab(dims, c, ok.SolverParams(tol=1e-10, delta=delta, W64_layout=w64),
                                    Ws[ok.OK_F64 | w64], None if low is None else Ws[low], lp, xi, psi, 1, work)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            best = sorted((best or []) + [sec])
        sol[name] = psi
        out["forms"][name] = {"seconds_median": round(best[1], 4), "status": rc, "iterations": st[0]["iterations"],
                              "reliable_updates": st[0]["reliable_updates"],
                              "true_rel_resid": st[0]["true_rel_resid"]}
        log("%s %s" % (name, out["forms"][name]))
    for name in ("mixed_f32", "mixed_bf16", "plain_f64_sigma", "mixed_f32_sigma", "mixed_f32_sigma_delta0.003"):
        err = float(torch.linalg.vector_norm(sol[name] - sol["plain_f64"]) /
                    torch.linalg.vector_norm(sol["plain_f64"]))
        out["forms"][name]["rel_error_vs_plain_f64"] = err
        out["forms"][name]["speedup"] = round(out["forms"]["plain_f64"]["seconds_median"] /
                                              out["forms"][name]["seconds_median"], 3)
    print(json.dumps(out), flush=True)


def net_kernels(args):
    """The network kernels alone at 24^3x64: one layer on 1 field ([V][12]) and on 16 fields
    (right-hand side fastest), its adjoint, and the weight gradient; HIP events on the
    library's stream.  Bytes: 936 B of transports per site (13 forward 3x3 FP32 complex;
    the backward hops reread them at the neighbour) + 96 B in and 96 B out per field;
    flops: 26 hops x (36 + 48) + 48 complex multiply-adds = 17,856 per site and field."""
    import torch

    from paper_1311_5029_amd import inputs as I
    from paper_1311_5029_amd import okinv as ok

    torch.cuda.set_device(0)
    dims = tuple(args.dims) if args.dims else (24, 24, 24, 64)
    V = int(np.prod(dims))
    log("net kernels at %s" % (dims,))
    U = I.random_su3_links(dims, I.config_epsilon("plaq0.6"), I.SEED_LINKS + 4)
    links = ok.to_device_complex(U)
    del U
    T = ok.empty_bytes(ok.ok_net_transports_bytes(dims))
    ok.ok_net_transports(dims, links, T)
    del links
    A = ok.to_device_complex(I.net_init_params(1, 1.0, I.SEED_NET, noise=0.1)[0], dtype="float32")
    stream = torch.cuda.current_stream()
    out = {"metric": "network layer throughput", "lattice": list(dims), "kernels": {}}
    flops_site = 26 * (36 + 48) * 8 + 48 * 8

    def timed(fn, n=10):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    for nf, inner in ((1, False), (16, True)):
        x = torch.randn(nf * V * 24, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        fl = ok.OK_SPINOR_RHS_INNER if inner else 0
        gA = torch.empty(27 * 32, dtype=torch.float32, device="cuda")
        work = ok.empty_bytes(ok.ok_net_workspace_bytes(dims, 1, nf, 2))
        for name, fn in (("layer", lambda: ok.ok_net_layer(dims, A, T, x, y, nf, fl, stream)),
                         ("adjoint", lambda: ok.ok_net_layer(dims, A, T, x, y, nf, fl | ok.OK_NET_ADJOINT, stream)),
                         ("wgrad", lambda: ok.ok_net_layer_wgrad(dims, T, x, y, gA, nf, fl, work, stream))):
            ms = timed(fn)
            by = V * (936 + nf * 192)
            fl_ = V * nf * flops_site
            key = "%s_nf%d_%s" % (name, nf, "inner" if inner else "outer")
            out["kernels"][key] = {"ms": round(ms, 4), "GB/s": round(by / ms / 1e6, 1),
                                   "TFLOP/s": round(fl_ / ms / 1e9, 2),
                                   "frac_hbm": round(by / ms / 1e6 / HBM_PEAK_GBS, 4),
                                   "frac_fp32_valu": round(fl_ / ms / 1e9 / 157.3, 4),
                                   # without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
                                   "frac_fp32_valu_unpacked": round(fl_ / ms / 1e9 / 78.6, 4)}
            log("%s %s" % (key, out["kernels"][key]))
        del x, y, work
    print(json.dumps(out), flush=True)


def chosen_solve(args):
    """The chosen form alone: the 12 point sources at 20^3 x 64 solved together with FP32
    sigma-layout W and FP64 reliable updates (sigma FP64 W), three times; one JSON line.  Run
    under rocprofv3 --kernel-trace --stats it gives the solve's time per kernel."""
    import torch

    from paper_1311_5029_amd import inputs as I
    from paper_1311_5029_amd import okinv as ok

    torch.cuda.set_device(0)
    cfg = I.make_config("batched_20x20x20x64")
    c = cfg["coeffs"]
    links = ok.to_device_complex(cfg["U"])
    S, INNER = ok.OK_LAYOUT_SIGMA, ok.OK_SPINOR_RHS_INNER
    Ws = {}
    for prec in (ok.OK_F64 | S, ok.OK_F32 | S):
        Ws[prec] = ok.empty_bytes(ok.ok_W_bytes(DIMS, prec))
        scr = ok.empty_bytes(ok.ok_precompute_scratch_bytes(DIMS))
        ok.ok_precompute_W(DIMS, c, links, prec, Ws[prec], scr)
        del scr
    xi = ok.to_device_complex(cfg["xi"])
    lp = ok.OK_F32 | S | INNER
    work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(DIMS, NRHS, lp))
    secs = []
    for _ in range(3):
        psi = torch.zeros_like(xi)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = ok.ok_bicgstab(DIMS, c, ok.SolverParams(tol=1e-10, delta=CHOSEN_DELTA, W64_layout=S),
                                Ws[ok.OK_F64 | S], Ws[ok.OK_F32 | S], lp, xi, psi, NRHS, work)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t)
        log("chosen solve %.3f s, status %d" % (secs[-1], rc))
    print(json.dumps({"metric": "time to 1e-10 residual, 12 point sources at 20^3x64, chosen form",
                      "seconds": [round(x, 4) for x in secs], "status": rc,
                      "iterations_largest": max(s["iterations"] for s in st),
                      "reliable_updates": sum(s["reliable_updates"] for s in st),
                      "max_true_rel_resid": max(s["true_rel_resid"] for s in st)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB copy (counter calibration)")
    ap.add_argument("--parse-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into the traffic file and exit")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "OUT", "COMMAND"),
                    help="write a text summary of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--workload", default="batched_20x20x20x64",
                    choices=["batched_20x20x20x64", "mixed_16x16x16x32", "learned_24x24x24x64",
                             "learned_batched_32x32x32x64", "net", "chosen_solve_20x20x20x64"],
                    help="batched_20x20x20x64 (default): the M.psi bench line and its solves; "
                         "mixed_16x16x16x32: plain vs mixed precision; learned_*: learned-preconditioner "
                         "solves; net: the network kernels alone")
    ap.add_argument("--dims", type=int, nargs=4, help="override the c4/c5 lattice (Lx Ly Lz Lt)")
    ap.add_argument("--n-train", type=int, default=0)
    ap.add_argument("--n-eval", type=int, default=0)
    ap.add_argument("--train-steps", type=int, default=400)
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.parse_pmc:
        parse_pmc(args.parse_pmc[0], args.parse_pmc[1], args.form)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "net":
        net_kernels(args)
        return
    if args.workload == "chosen_solve_20x20x20x64":
        chosen_solve(args)
        return
    if args.workload == "mixed_16x16x16x32":
        mixed(args)
        return
    if args.workload.startswith("learned"):
        learned(args)
        return

    import torch

    from paper_1311_5029_amd import inputs as I
    from paper_1311_5029_amd import okinv as ok

    torch.cuda.set_device(0)
    form = {"f64": ok.OK_F64, "f32": ok.OK_F32, "bf16": ok.OK_BF16}[args.form]
    log("generating links 20^3x64")
    t0 = time.time()
    cfg = I.make_config("batched_20x20x20x64")
    c = cfg["coeffs"]
    log("links in %.1fs, plaquette^(1/4) = u0 = %.5f, eps = %.5f" % (time.time() - t0, cfg["u0"], cfg["eps"]))
    links = ok.to_device_complex(cfg["U"])
    SITE, INNER = ok.OK_LAYOUT_SITE, ok.OK_SPINOR_RHS_INNER
    Ws = {}
    pre_ms = {}
    SAVED, SIGMA = ok.OK_LAYOUT_SAVED, ok.OK_LAYOUT_SIGMA
    # (the 14-block saved set, OK_LAYOUT_SAVED, is parity-tested but not timed here: it reads as many
    # lines through L2 as the 27 dense blocks and is no faster)
    wforms = [ok.OK_F64, ok.OK_F32, ok.OK_BF16, ok.OK_F32 | SITE, ok.OK_BF16 | SITE, ok.OK_F64 | SIGMA,
              ok.OK_F32 | SIGMA]
    for prec in wforms:
        Ws[prec] = ok.empty_bytes(ok.ok_W_bytes(DIMS, prec))
        scr = ok.empty_bytes(ok.ok_precompute_scratch_bytes(DIMS))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ok.ok_precompute_W(DIMS, c, links, prec, Ws[prec], scr)
        e1.record()
        torch.cuda.synchronize()
        pre_ms[PREC_NAME[prec & 3] + ("_site" if prec & SITE else "_saved" if prec & SAVED else
                                      "_sigma" if prec & SIGMA else "")] = \
            round(e0.elapsed_time(e1), 3)
        del scr
    log("precompute ms %s" % pre_ms)

    # ---- timed region: M applied to the 12-RHS batch --------------------------------
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda").manual_seed(I.SEED_SOURCES + 3)
    if form == ok.OK_F64:    # no FP64 matrix-core kernel: 12 single-RHS launches (plane W)
        wprec, sprec, launches, kname = ok.OK_F64, ok.OK_F64, NRHS, "k_apply"
        x = torch.randn(NRHS * V * 24, dtype=torch.float64, device="cuda", generator=gen)
    else:
        wprec, sprec, launches, kname = form | SITE, ok.OK_F32 | INNER, 1, "k_apply_site"
        x = torch.randn(NRHS * V * 24, dtype=torch.float32, device="cuda", generator=gen)
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        ok.ok_apply_M(DIMS, c, Ws[wprec], wprec, x, y, sprec, NRHS, stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_wall0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        ok.ok_apply_M(DIMS, c, Ws[wprec], wprec, x, y, sprec, NRHS, stream)
        b.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    step_ms = [a.elapsed_time(b) for a, b in evs]
    ms_per_step = float(np.mean(step_ms))
    launch_ms = ms_per_step / launches
    bytes_launch = BYTES_STEP[form] * V / launches
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    value = BYTES_STEP[form] * V / (ms_per_step * 1e-3) / 1e9
    log("M.psi %s: %.3f ms/step (%d RHS), %.1f GB/s, %.1f%% of peak; wall %.3fs"
        % (args.form, ms_per_step, NRHS, value, 100 * value / HBM_PEAK_GBS, t_wall))

    def time_apply(wp, sp, nrhs, n=10):
        dt = torch.float64 if sp == ok.OK_F64 else torch.float32
        xx = x[: nrhs * V * 24].to(dt)
        yy = torch.empty_like(xx)
        for _ in range(2):
            ok.ok_apply_M(DIMS, c, Ws[wp], wp, xx, yy, sp, nrhs, stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n):
            ok.ok_apply_M(DIMS, c, Ws[wp], wp, xx, yy, sp, nrhs, stream)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    # context: one right-hand side (plane W), and the batched forms
    apply_forms = {}
    for prec in (ok.OK_F64, ok.OK_F32, ok.OK_BF16):
        for lay in (0, SIGMA):
            if lay == SIGMA and prec == ok.OK_BF16:
                continue
            ms = time_apply(prec | lay, ok.OK_F64 if prec == ok.OK_F64 else ok.OK_F32, 1)
            # the saved and sigma layouts stream their stored set once per site (the backward
            # blocks are reread from neighbours); their GB/s counts the bytes of that set
            by = BYTES_SAVED[prec] if lay == SAVED else BYTES_SIGMA[prec] if lay == SIGMA else BYTES_SITE[prec]
            gbs = by * V / (ms * 1e-3) / 1e9
            apply_forms["1rhs_" + PREC_NAME[prec] + ("_saved" if lay == SAVED else "_sigma" if lay else "")] = {
                "ms": round(ms, 4), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                "rhs_sites_per_s": round(V / (ms * 1e-3), 0)}
    # 12 right-hand sides with FP32 sigma-layout W (one W read for all of them, no matrix cores)
    ms = time_apply(ok.OK_F32 | SIGMA, ok.OK_F32 | INNER, NRHS)
    gbs = (BYTES_SIGMA[1] - 2 * 96 + NRHS * 2 * 96) * V / (ms * 1e-3) / 1e9
    apply_forms["12rhs_sigma_f32"] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                      "rhs_sites_per_s": round(NRHS * V / (ms * 1e-3), 0)}
    for prec in (ok.OK_F32, ok.OK_BF16):
        ms = time_apply(prec | SITE, ok.OK_F32 | INNER, NRHS)
        gbs = BYTES_STEP[prec] * V / (ms * 1e-3) / 1e9
        apply_forms["12rhs_mfma_" + PREC_NAME[prec]] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                                                        "frac": round(gbs / HBM_PEAK_GBS, 4),
                                                        "rhs_sites_per_s": round(NRHS * V / (ms * 1e-3), 0)}
    log("apply forms %s" % apply_forms)

    if args.copy_probe:
        copy_probe()

    # context: a plain 4 GiB device copy (read + write) as a practical bandwidth ceiling
    a4 = torch.empty((4 << 30) // 4, dtype=torch.float32, device="cuda")
    b4 = torch.empty_like(a4)
    b4.copy_(a4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b4.copy_(a4)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (4 << 30) / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    del a4, b4
    log("4 GiB device copy: %.1f GB/s" % copy_gbs)

    # ---- time to solution: plain vs chosen, the 12 point sources --------------------
    # plain: FP64 W (27 dense blocks), FP64 fields, one source after the other.  The other forms
    # change only the storage of W and the arithmetic of the inner solve; every one stops on
    # the FP64 true residual.  chosen = the fastest of them (median of three solves each).
    solve = None
    if not args.no_solve:
        xi = ok.to_device_complex(cfg["xi"])
        res = {}
        forms = (("plain", None, 0, 1, "FP64 W (27 dense blocks), FP64 fields, one RHS after the other"),
                 ("plain_sigma", None, SIGMA, 1, "FP64 W as 46 Pauli-component colour matrices per site, FP64 "
                                                 "fields, one RHS after the other"),
                 ("batched_bf16", ok.OK_BF16 | SITE, 0, 3, "12 RHS together: BF16 W on the matrix cores, FP32 "
                                                           "fields, FP64 reliable updates (dense FP64 W)"),
                 ("batched_bf16_sigma64", ok.OK_BF16 | SITE, SIGMA, 3, "as batched_bf16, FP64 reliable updates "
                                                                       "with the sigma-layout FP64 W"),
                 ("mixed_f32_sigma", ok.OK_F32 | SIGMA, SIGMA, 3, "one RHS after the other: FP32 sigma-layout W, "
                                                                  "FP32 fields, FP64 reliable updates (sigma W)"),
                 ("batched_f32_sigma_delta0.1", ok.OK_F32 | SIGMA | INNER, SIGMA, 1,
                  "12 RHS together: FP32 sigma-layout W read once for all of them, FP32 fields, FP64 reliable "
                  "updates (sigma W) at the default threshold delta = 0.1"),
                 ("batched_f32_sigma", ok.OK_F32 | SIGMA | INNER, SIGMA, 3,
                  "12 RHS together: FP32 sigma-layout W read once for all of them, FP32 fields, FP64 reliable "
                  "updates (sigma W) when the FP32 residual has dropped by delta = %g" % CHOSEN_DELTA))
        kinds = {"plain": dict(kind="plain", w64_sigma=False), "plain_sigma": dict(kind="plain", w64_sigma=True),
                 "batched_bf16": dict(kind="batched", wlo="bf16", w64_sigma=False),
                 "batched_bf16_sigma64": dict(kind="batched", wlo="bf16", w64_sigma=True),
                 "mixed_f32_sigma": dict(kind="mixed", wlo="f32_sigma", w64_sigma=True),
                 "batched_f32_sigma": dict(kind="batched", wlo="f32_sigma", w64_sigma=True),
                 "batched_f32_sigma_delta0.1": dict(kind="batched", wlo="f32_sigma", w64_sigma=True)}
        psi_plain = None
        for name, low, w64, reps, desc in forms:
            lp = -1 if low is None else low
            work = ok.empty_bytes(ok.ok_bicgstab_workspace_bytes(DIMS, NRHS, lp))
            params = ok.SolverParams(tol=1e-10, W64_layout=w64,
                                     delta=CHOSEN_DELTA if name == "batched_f32_sigma" else 0.1)
            secs = []
            for _ in range(reps):
                psi = torch.zeros_like(xi)
                torch.cuda.synchronize()
                t = time.perf_counter()
                rc, st = ok.ok_bicgstab(DIMS, c, params, Ws[ok.OK_F64 | w64],
                                        None if low is None else Ws[low & ~INNER], lp, xi, psi, NRHS, work, stream)
                torch.cuda.synchronize()
                secs.append(time.perf_counter() - t)
            sec = float(np.median(secs))
            nbytes = solve_bytes(kinds[name], st) * V
            res[name] = {
                "form": desc, "seconds": round(sec, 3), "status": rc, "repeats": reps,
                "iterations": int(sum(s["iterations"] for s in st)),
                "iterations_max_rhs": int(max(s["iterations"] for s in st)),
                "matvec_f64": int(sum(s["matvec_hi"] for s in st)),
                "matvec_low": int(sum(s["matvec_lo"] for s in st)),
                "reliable_updates": int(sum(s["reliable_updates"] for s in st)),
                "max_true_rel_resid": max(s["true_rel_resid"] for s in st),
                "roofline": {"algorithmic_bytes": nbytes, "GB/s": round(nbytes / sec / 1e9, 1),
                             "frac": round(nbytes / sec / 1e9 / HBM_PEAK_GBS, 4)},
            }
            # error of this form's solution against the plain FP64 one (whose residual the oracle
            # checks in the full-size tests), per right-hand side
            if psi_plain is None:
                psi_plain = psi.clone()
            else:
                d = (psi - psi_plain).view(NRHS, -1)
                errs = (torch.linalg.vector_norm(d, dim=1) /
                        torch.linalg.vector_norm(psi_plain.view(NRHS, -1), dim=1)).tolist()
                res[name]["rel_error_vs_plain_f64"] = {"max": max(errs), "median": float(np.median(errs))}
            log("solve %s: %s" % (name, res[name]))
            del work, psi
        # CG on the normal equations (ok_cgnr, sigma-layout FP64 W) on the first two sources, per source,
        # next to BiCGStab with the same operator
        work = ok.empty_bytes(ok.ok_cgnr_workspace_bytes(DIMS, 2))
        xi2 = xi.reshape(-1)[: 2 * V * 24]
        psi = torch.zeros_like(xi2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, st = ok.ok_cgnr(DIMS, c, ok.SolverParams(tol=1e-10, max_iter=20000, W64_layout=SIGMA), Ws[ok.OK_F64 | SIGMA],
                            xi2, psi, 2, work, stream)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        cg = {"form": "CG on M^dag M (M^dag = gamma5 M gamma5), FP64, sigma-layout W, first 2 of the 12 sources",
              "status": rc, "seconds_per_source": round(sec / 2, 3),
              "iterations_per_source": sum(s["iterations"] for s in st) / 2,
              "applications_per_source": sum(s["matvec_hi"] for s in st) / 2,
              "max_true_rel_resid": max(s["true_rel_resid"] for s in st),
              "bicgstab_same_operator_seconds_per_source": round(res["plain_sigma"]["seconds"] / NRHS, 3),
              "bicgstab_same_operator_applications_per_source": res["plain_sigma"]["matvec_f64"] / NRHS}
        log("cgnr: %s" % cg)
        del work, psi
        best = min((k for k in res if k != "plain"), key=lambda k: res[k]["seconds"])
        solve = {"workload": "12 point sources to ||xi-M psi||/||xi|| <= 1e-10 (FP64 true residual)",
                 "plain": res["plain"], "chosen": dict(name=best, **res[best]),
                 "speedup": round(res["plain"]["seconds"] / res[best]["seconds"], 3),
                 # the best unpreconditioned FP64 form (sigma-layout W), for scale
                 "speedup_vs_plain_sigma": round(res["plain_sigma"]["seconds"] / res[best]["seconds"], 3),
                 "forms": res, "cgnr": cg}

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(solve["plain"]["iterations"] if solve is not None else None)
        log("cpu baseline %s" % cpu)

    out = {
        "metric": "M.psi HBM GB/s (% peak) at 20^3x64; time to 1e-10 residual, plain vs chosen",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16 W, f32 spinors, f32 accumulate"}[args.form],
        "data": "synthetic: random SU(3) links at plaquette 0.6, 12 point sources; stand-in OK coefficients",
        "config": {"workload": "OK operator M.psi, 20^3x64 lattice, 12 RHS batched on the matrix cores, %s W "
                               "(dense 27x12x12 per site, site-major)" % args.form, "lattice": list(DIMS), "nrhs": NRHS, "W_storage": args.form,
                   "u0": round(cfg["u0"], 6), "eps": round(cfg["eps"], 6)},
        "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
        "copy_GBs": round(copy_gbs, 1),
        "frac_of_copy": round(value / copy_gbs, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(kname, args.form),
                     "kernel": "%s<%s>, %d sites, %d B/site" % (kname, args.form, V, BYTES_STEP[form] // launches),
                     "launch_ms": round(launch_ms, 4)},
        "apply_forms": apply_forms,
        "precompute_ms": pre_ms,
        "time_to_solution": solve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
