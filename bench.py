#!/usr/bin/env python3
"""Benchmark: approximate fPEPS contraction on a random 3-regular graph.

Workload (one GPU): a Z2 fermionic PEPS on a seeded random 3-regular graph
with 40 sites, physical dim 4 (2 even / 2 odd), bond D = 4 (2 / 2), entries
N(0, 1/32); approximate contraction with bond compression to chi = 64 along
a seeded greedy path, FP64 throughout. One step = the norm <psi|psi> plus
the hopping term <psi|h|psi> on the first edge: two network contractions
(metric unit: contractions per second). The timed steps run on two streams,
each driven by its own host thread and alternating the two kinds of
contraction (--serial: one stream, norm then hopping term).

Prints one JSON line with the throughput of the timed steps, a roofline
entry for the dominant kernel (timed with two HIP events on each of its
dispatches, on the stream it runs on, over an instrumented repeat of the
timed steps: the events cost host time per launch, about 12% of the step,
so they stay out of the steps that give the throughput), and the CPU oracle
timed on a bounded sample on rank 0.
"""

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# per profiler class: (peak, unit, bound). The factorisation kernels (Cholesky,
# Jacobi) run FP64 vector arithmetic, priced against the FP64 vector peak
# (256 CUs x 2.4 GHz x 128 FP64 flops per CU per clock = 78.6 TFLOP/s).
PEAK = {"gemm_f64": (78.6, "TFLOP/s", "mfma"), "gemm_f32": (157.3, "TFLOP/s", "mfma"),
        "gemm_bf16x3": (2500.0, "TFLOP/s", "mfma"), "permute": (8000.0, "GB/s", "hbm"),
        "factor": (78.6, "TFLOP/s", "alu"), "k_splitk_reduce_f64": (8000.0, "GB/s", "hbm")}
for _k in ("64x64", "128x128", "256x16", "256x32", "16x256", "32x256"):
    PEAK["k_gemm_f64_" + _k] = (78.6, "TFLOP/s", "mfma")
for _k in ("k_orth_factor", "k_jacobi_sweep", "k_jacobi_sweep_la", "k_jacobi_vectors", "k_svd_cols"):
    PEAK[_k] = (78.6, "TFLOP/s", "alu")
PEAK["k_skinny_f64"] = (8000.0, "GB/s", "hbm")  # tall-skinny A^T B reads A and B once
PEAK["k_gemm_f64_tall"] = (8000.0, "GB/s", "hbm")  # tall A (N <= 16, K <= 256) streamed once
# single kernels (the classes gemm_f64 and factor are families of kernels)
KERNELS = ["gemm_f32", "gemm_bf16x3", "permute", "k_splitk_reduce_f64", "k_gemm_f64_64x64", "k_gemm_f64_128x128",
           "k_gemm_f64_256x16", "k_gemm_f64_256x32", "k_gemm_f64_16x256", "k_gemm_f64_32x256", "k_orth_factor",
           "k_jacobi_sweep", "k_jacobi_sweep_la", "k_jacobi_vectors", "k_svd_cols", "k_skinny_f64", "k_gemm_f64_tall"]
PROFILES = os.path.join(ROOT, "profiles")


def source_hash():
    """SHA-256 over the library sources (kernels, plans, launch code)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2410_02215_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(cls, workload):
    """HBM bytes per launch of a class from the committed PMC summary, or None.

    The summary of a workload records the source hash it was measured at;
    any change of the library sources since then makes the figure stale.
    """
    try:
        with open(os.path.join(PROFILES, "hbm_traffic_%s.md" % workload)) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"^source-hash: ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(1) != source_hash():
        return None
    m = re.search(r"^traffic-per-launch %s ([0-9.eE+]+)$" % re.escape(cls), text, re.M)
    return float(m.group(1)) if m else None


def load_paths():
    with open(os.path.join(ROOT, "synth", "data", "paths.json")) as f:
        return json.load(f)


def gpu_setup(cfg, paths):
    import torch
    from paper_2410_02215_amd import peps as GP
    from synth import workloads as W
    from synth.operators import operator_dense
    spec = cfg["spec"]
    vals = W.all_site_values(spec, cfg["seed"])
    kets = GP.ket_tensors(spec, vals)
    op = GP.operator_tensor(spec, operator_dense("hop", "Z2"))
    nn = GP.norm_network(spec, kets)
    nh = GP.norm_network(spec, kets, op=op, op_sites=cfg["op_sites"])
    # a second network object of each kind (same site tensors) for the second
    # host thread of the alternating schedule (gpu_steps)
    nn2 = GP.norm_network(spec, kets)
    nh2 = GP.norm_network(spec, kets, op=op, op_sites=cfg["op_sites"])
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]  # default priority
    return dict(nn=nn, nh=nh, nn2=nn2, nh2=nh2, kets=kets, op=op, pn=paths["c2_norm"]["path"],
                ph=paths["c2_hop"]["path"], streams=streams)


def gpu_step(g, chi, concurrent=True, gemm=None):
    """One step: the norm and the hopping-term contraction.

    The two contractions are independent. By default they run at the same
    time, each on its own HIP stream from its own host thread (the library
    call releases the GIL), so that the latency-bound factorisation kernels
    of one overlap the bandwidth- and MFMA-bound kernels of the other.
    """
    import threading
    import torch
    jobs = [(g["nn"], g["pn"]), (g["nh"], g["ph"])]
    out = [None, None]
    err = [None, None]

    def run(k):
        try:
            with torch.cuda.stream(g["streams"][k]):
                if gemm is None:
                    out[k] = jobs[k][0].contract(jobs[k][1], chi=chi)
                else:
                    out[k] = jobs[k][0].contract(jobs[k][1], chi=chi, gemm=gemm)
        except Exception as ex:  # re-raised in the caller
            err[k] = ex

    if concurrent:
        th = threading.Thread(target=run, args=(1,))
        th.start()
        run(0)
        th.join()
    else:
        run(0)
        run(1)
    for ex in err:
        if ex is not None:
            raise ex
    (m1, e1, s1), (m2, e2, s2) = out
    return (m1, e1, m2, e2), (s1, s2)


def gpu_steps(g, chi, steps, concurrent=True, gemm=None, label=None):
    """`steps` steps, each one norm and one hopping-term contraction.

    Concurrent: two host threads, each driving its own stream, run `steps`
    contractions each, alternating the two kinds (stream 0: norm, hop,
    norm, ...; stream 1: hop, norm, hop, ...) with no join between steps, so
    that both streams carry the same mix of work (alone the hopping term
    takes longer than the norm, and a per-step join leaves one stream idle).
    Every step's pair is computed; the results are those of the last norm
    and the last hopping term. Not concurrent: norm then hopping term per
    step on one stream.
    """
    import threading
    import torch
    nets = [[(g["nn"], g["pn"]), (g["nh"], g["ph"])], [(g["nn2"], g["pn"]), (g["nh2"], g["ph"])]]
    last = [[None, None], [None, None]]  # per thread: last norm, last hop
    stats = [[], []]
    err = [None, None]

    def contract(k, kind):
        net, path = nets[k][kind]
        if gemm is None:
            return net.contract(path, chi=chi)
        return net.contract(path, chi=chi, gemm=gemm)

    def run(k):
        try:
            with torch.cuda.stream(g["streams"][k]):
                for i in range(steps):
                    kind = (i + k) % 2
                    m, e, st = contract(k, kind)
                    last[k][kind] = (i, m, e)
                    stats[k].append(st)
                    if label and k == 0:
                        print("[bench] %s %d done (stream 0)" % (label, i), file=sys.stderr, flush=True)
        except Exception as ex:  # re-raised in the caller
            err[k] = ex

    if concurrent:
        th = threading.Thread(target=run, args=(1,))
        th.start()
        run(0)
        th.join()
        for ex in err:
            if ex is not None:
                raise ex
        pick = lambda kind: max((x for x in (last[0][kind], last[1][kind]) if x is not None))[1:]
        (m1, e1), (m2, e2) = pick(0), pick(1)
        return (m1, e1, m2, e2), stats[0] + stats[1]
    res, st = None, []
    for i in range(steps):
        res, s2 = gpu_step(g, chi, False, gemm)
        st += list(s2)
        if label:
            print("[bench] %s %d done" % (label, i), file=sys.stderr, flush=True)
    return res, st


def to_f32(P, t):
    """FP32 copy of a library tensor (entries rounded to nearest)."""
    inf = t.info()
    return P.Tensor.create(inf["sym"], t.legs(), inf["total"], P.F32, data=t.data().float())


def to_f64(P, t):
    """FP64 copy of a library tensor."""
    inf = t.info()
    return P.Tensor.create(inf["sym"], t.legs(), inf["total"], P.F64, data=t.data().double())


def c2_forms(P, cfg, g, chi, steps, golden):
    """The same workload with FP32 tensors and FP32 or split-BF16 block GEMMs
    (compression and the final reduction in FP64), measured after the timed
    FP64 region: contractions/s and error against the oracle."""
    import torch
    from paper_2410_02215_amd import peps as GP
    spec = cfg["spec"]
    k32 = [to_f32(P, k) for k in g["kets"]]
    op32 = to_f32(P, g["op"])
    g32 = dict(g, nn=GP.norm_network(spec, k32), nh=GP.norm_network(spec, k32, op=op32, op_sites=cfg["op_sites"]),
               nn2=GP.norm_network(spec, k32), nh2=GP.norm_network(spec, k32, op=op32, op_sites=cfg["op_sites"]))
    # the FP64 path on the FP32-rounded inputs: the reference that isolates
    # the error of the FP32 arithmetic from the rounding of the inputs
    k64r = [to_f64(P, k) for k in k32]
    g64r = dict(g, nn=GP.norm_network(spec, k64r),
                nh=GP.norm_network(spec, k64r, op=to_f64(P, op32), op_sites=cfg["op_sites"]))
    r64, _ = gpu_step(g64r, chi, True)
    n64 = r64[0] * 2.0 ** r64[1]
    h64 = (r64[2] / r64[0]) * 2.0 ** (r64[3] - r64[1])
    out = {}
    for name, gemm in (("f32", P.GEMM_F32), ("bf16x3", P.GEMM_BF16X3)):
        gpu_steps(g32, chi, 2, True, gemm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = gpu_steps(g32, chi, steps, True, gemm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        norm = res[0] * 2.0 ** res[1]
        hop = (res[2] / res[0]) * 2.0 ** (res[3] - res[1])
        out[name] = {"value": 2.0 * steps / el, "ms_per_step": 1000.0 * el / steps, "steps": steps,
                     "rel_err_vs_oracle": golden(norm, hop),
                     "rel_err_vs_f64_same_inputs": {"norm": abs(norm - n64) / abs(n64),
                                                    "hop_term": abs(hop - h64) / abs(h64)}}
        print("[bench] form %s: %.3f contractions/s" % (name, out[name]["value"]), file=sys.stderr, flush=True)
    return out


def cpu_baseline(cfg, paths, runs=3):
    """The oracle on the host cores: full <psi|psi> contractions, timed.

    One untimed warm-up contraction, then ``runs`` timed ones; the rate is
    that of the median. The hopping term costs about six times a norm
    contraction on the CPU, so it is left out of the bounded sample: the rate
    of norm contractions alone is an upper bound on the oracle's rate for the
    benchmark's mix of contractions.
    """
    import torch
    from oracle import physics as OP
    from oracle.network import network_value
    from synth import workloads as W
    spec = cfg["spec"]
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    net = OP.norm_network(spec, kets, conv="local")
    m, e = network_value(net, paths["c2_norm"]["path"], chi=cfg["chi"])
    ts = []
    for _ in range(runs):
        t0 = time.time()
        network_value(net, paths["c2_norm"]["path"], chi=cfg["chi"])
        ts.append(time.time() - t0)
    el = sorted(ts)[len(ts) // 2]
    return dict(value=1.0 / el, unit="contractions/s", cores=cores, kind="oracle",
                sample="full <psi|psi> contractions of the same workload: one warm-up, then the median of %d "
                       "(%s s; FP64, torch CPU with %d threads); the hopping-term contraction is not included"
                       % (runs, ", ".join("%.1f" % t for t in ts), cores),
                log2_norm=math.log2(abs(m)) + e if m else None)


def golden_errors(norm, hop):
    """Relative errors of the step's results against the stored oracle values.

    tests/golden/values.json is written by tests/golden/make_golden.py, which
    calls only the oracle, with the same seeded inputs, paths and chi.
    """
    try:
        with open(os.path.join(ROOT, "tests", "golden", "values.json")) as f:
            gold = json.load(f)
        rn = gold["c2_norm"]["mantissa"] * 2.0 ** gold["c2_norm"]["exp2"]
        rh = gold["c2_hop"]["mantissa"] * 2.0 ** gold["c2_hop"]["exp2"]
    except (OSError, KeyError, ValueError):
        return None
    return {"norm": abs(norm / rn - 1.0), "hop_term": abs(hop * norm / rh - 1.0)}


TUNING = os.path.join(ROOT, "paper_2410_02215_amd", "tuning", "gfx950.json")


def autotune_setup(P, args):
    """GEMM tile autotuner: stored choices, unseen shapes tuned during warm-up."""
    if args.no_autotune:
        P.ftn.autotune(0)
        return
    if os.path.exists(TUNING):
        P.ftn.autotune_load(TUNING)
    P.ftn.autotune(2)


def amplitude_setup(cfg):
    import torch
    from paper_2410_02215_amd import peps as GP
    from synth import workloads as W
    from synth.peps import occupation_samples
    spec = cfg["spec"]
    kets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    torch.cuda.synchronize()
    return dict(kets=kets, bonds=W.amplitude_bonds(spec), path=W.boundary_path(cfg["lx"], cfg["ly"]),
                samples=occupation_samples(spec.n_sites, cfg["n_samples"], cfg["seed"] + 1))


def amplitude_cpu_baseline(cfg, g, n):
    """The oracle on the host cores: n amplitudes of the same workload, timed."""
    import torch
    from oracle import physics as OP
    from oracle.amplitude import amplitude
    from synth import workloads as W
    spec = cfg["spec"]
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"]))
    t0 = time.time()
    for c in g["samples"][:n]:
        amplitude(kets, g["bonds"], c, g["path"], chi=cfg["chi"])
    el = time.time() - t0
    return dict(value=n / el, unit="contractions/s", cores=cores, kind="oracle",
                sample="%d amplitudes <n|psi> of the same workload, one after the other (%.1f s, FP64, torch "
                       "CPU with %d threads)" % (n, el, cores))


def main_amplitudes(args):
    """Amplitude workload: a step is one batch of sampled configurations."""
    import torch
    import paper_2410_02215_amd as P
    from synth import workloads as W
    cfg = W.c4()
    g = amplitude_setup(cfg)
    B = args.batch
    need = B * (args.warmup + args.steps)
    if need > len(g["samples"]):
        raise SystemExit("batch x (warmup + steps) exceeds the %d samples" % len(g["samples"]))
    print("[bench] workload %s: batch %d, workers %d" % (cfg["name"], B, args.workers), file=sys.stderr, flush=True)
    k = 0
    for _ in range(args.warmup):
        P.amplitudes(g["kets"], g["bonds"], g["path"], g["samples"][k:k + B], chi=cfg["chi"], nworkers=args.workers)
        k += B
        print("[bench] warmup batch done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    P.ftn.profile_collect()
    P.ftn.profile_enable(True)
    t0 = time.perf_counter()
    for st in range(args.steps):
        m, e = P.amplitudes(g["kets"], g["bonds"], g["path"], g["samples"][k:k + B], chi=cfg["chi"],
                            nworkers=args.workers)
        k += B
        print("[bench] batch %d done" % st, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.ftn.profile_enable(False)
    prof = P.ftn.profile_collect()
    el = t1 - t0
    out = {
        "metric": "ftensordot useful TFLOP/s + fPEPS contractions/sec on 1 GPU at stated err vs FP64",
        "value": B * args.steps / el, "unit": "contractions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "sites": cfg["spec"].n_sites, "chi": cfg["chi"],
                   "amplitudes_per_step": B, "workers": args.workers},
        "kernel_time_ms": {c: prof[c][0] / args.steps for c in prof if prof[c][0] > 0},
        "kernel_launches": {c: prof[c][1] / args.steps for c in prof if prof[c][0] > 0},
        # algorithmic work (flops or bytes, as the class's peak is priced) and
        # algorithmic bytes per launch of every class
        "kernel_work_per_launch": {c: prof[c][2] / prof[c][1] for c in prof if prof[c][1] > 0},
        "kernel_bytes_per_launch": {c: prof[c][3] / prof[c][1] for c in prof if prof[c][1] > 0},
        # launches of the library's worker threads are not instrumented: with
        # more than one worker the line carries wall-clock rates only
        "roofline": roofline(prof, cfg["name"]) if any(prof[c][0] > 0 for c in prof) else None,
    }
    if not args.no_forms:
        out["forms"] = amplitude_forms(P, cfg, g, g["samples"][k - B:k], args.workers, m, e)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, %d amplitudes)" % args.cpu_samples, file=sys.stderr, flush=True)
        out["cpu_baseline"] = amplitude_cpu_baseline(cfg, g, args.cpu_samples)
    print(json.dumps(out), flush=True)


def amplitude_forms(P, cfg, g, samples, workers, m64, e64):
    """After the timed batches: the last batch again as the plain FP64 loop
    (one worker, one sample after the other; a subset of 16) and with FP32 site
    tensors and FP32 block GEMMs (compression in FP64) over the same workers,
    with the error of every amplitude against the FP64 result."""
    import numpy as np
    import torch
    out = {}
    sub = samples[:16]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.amplitudes(g["kets"], g["bonds"], g["path"], sub, chi=cfg["chi"], nworkers=1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["plain_f64"] = {"value": len(sub) / el, "samples": len(sub), "workers": 1}
    k32 = [to_f32(P, k) for k in g["kets"]]
    P.amplitudes(k32, g["bonds"], g["path"], samples[:4], chi=cfg["chi"], gemm=P.GEMM_F32, nworkers=workers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m32, e32 = P.amplitudes(k32, g["bonds"], g["path"], samples, chi=cfg["chi"], gemm=P.GEMM_F32, nworkers=workers)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m64, e64 = np.asarray(m64, dtype=np.float64), np.asarray(e64, dtype=np.int64)
    ok = m64 != 0
    rel = np.abs(np.asarray(m32)[ok] * np.exp2((np.asarray(e32)[ok] - e64[ok]).astype(np.float64)) - m64[ok]) \
        / np.abs(m64[ok])
    out["f32"] = {"value": len(samples) / el, "samples": len(samples), "workers": workers,
                  "rel_err_vs_f64": {"max": float(rel.max()) if rel.size else None,
                                     "median": float(np.median(rel)) if rel.size else None}}
    out["note"] = ("plain_f64: the same amplitudes one after the other on one worker; f32: FP32 site tensors and "
                   "block GEMMs, compression in FP64, error against the FP64 amplitudes of the timed batch")
    print("[bench] forms: plain %.2f/s, f32 %.2f/s" % (out["plain_f64"]["value"], out["f32"]["value"]),
          file=sys.stderr, flush=True)
    return out


def main_gradient(args):
    """Energy-gradient workload: a step is one gradient of
    E = sum_t <psi|h_t|psi> / <psi|psi> (Hubbard, t = 1, U = 8) with respect
    to every ket tensor, every network compressed as early as possible."""
    import torch
    import paper_2410_02215_amd as P
    from paper_2410_02215_amd import autograd as AG, peps as GP
    from synth import workloads as W
    from synth.operators import operator_dense
    cfg = W.c5()
    spec = cfg["spec"]
    chi = args.chi or cfg["chi"]
    lx, ly = cfg["lx"], cfg["ly"]
    kets = [AG.DTensor.from_tensor(k, requires_grad=True)
            for k in GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))]
    terms = W.hubbard_terms(spec)
    paths = {None: W.norm_layer_path(spec, lx, ly)}
    for _, sites in terms:
        paths[tuple(sites)] = W.norm_layer_path(spec, lx, ly, tuple(sites))
    gterms = [(AG.DTensor.from_tensor(GP.operator_tensor(spec, operator_dense(kind, "Z2"))), sites)
              for kind, sites in terms]
    nnet = len(terms) + 1
    wname = cfg["name"].replace("chi%d" % cfg["chi"], "chi%d" % chi)
    print("[bench] workload %s: %d networks per gradient" % (wname, nnet), file=sys.stderr, flush=True)

    # recomputation checkpoints: by default one absorbed layer of the boundary
    # contraction per segment, so the stored tensors are the boundaries
    # between layers (the environments)
    ck = ly if args.checkpoint is None else (args.checkpoint or None)

    gkets = GP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    gops = [(GP.operator_tensor(spec, operator_dense(kind, "Z2")), sites) for kind, sites in terms]

    def step():
        if args.autograd:
            E = AG.expectation_ratio(spec, kets, gterms, paths, chi=chi, checkpoint=ck)
            gs = torch.autograd.grad(E, [k.data for k in kets])
            return float(E.detach()), gs
        # the library's backward pass per network (ftn_contract_network_grad)
        E, gt = GP.energy_gradient(spec, gkets, gops, paths, chi=chi, checkpoint=ck or 0)
        return E, [g.data() for g in gt]

    for _ in range(args.warmup):
        E, _ = step()
        print("[bench] warmup gradient done: E = %.10f" % E, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    P.ftn.memory_stats(torch.cuda.current_device(), reset_peak=True)
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    for k in range(args.steps):
        E, gs = step()
        print("[bench] gradient %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    peak = {"library": P.ftn.memory_stats(torch.cuda.current_device())["peak"] / 1e9,
            "torch": torch.cuda.max_memory_allocated() / 1e9}
    # an instrumented repeat (two HIP events on every dispatch) for the
    # per-kernel durations and the roofline, timed apart from `value`
    P.ftn.profile_collect()
    P.ftn.profile_enable(True)
    tp0 = time.perf_counter()
    for k in range(args.steps):
        step()
        print("[bench] profiled gradient %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    P.ftn.profile_enable(False)
    prof = P.ftn.profile_collect()
    el = t1 - t0
    gnorm = math.sqrt(sum(float((g.double() ** 2).sum()) for g in gs))
    out = {
        "metric": "ftensordot useful TFLOP/s + fPEPS contractions/sec on 1 GPU at stated err vs FP64",
        "value": nnet * args.steps / el, "unit": "contractions/s (forward + backward)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wname, "sites": spec.n_sites,
                   "chi": chi, "networks_per_gradient": nnet, "gradients_per_s": args.steps / el,
                   "checkpoint_steps": ck or 0,
                   "backward": "torch.autograd over the library's adjoints" if args.autograd
                   else "library network backward (ftn_contract_network_grad)"},
        "peak_memory_gb": peak,
        "profiled_ms_per_step": 1000.0 * (tp1 - tp0) / args.steps,
        "kernel_time_ms": {c: prof[c][0] / args.steps for c in prof if prof[c][0] > 0},
        "kernel_launches": {c: prof[c][1] / args.steps for c in prof if prof[c][0] > 0},
        # algorithmic work (flops or bytes, as the class's peak is priced) and
        # algorithmic bytes per launch of every class
        "kernel_work_per_launch": {c: prof[c][2] / prof[c][1] for c in prof if prof[c][1] > 0},
        "kernel_bytes_per_launch": {c: prof[c][3] / prof[c][1] for c in prof if prof[c][1] > 0},
        "result": {"energy": E, "grad_norm": gnorm},
        "roofline": roofline(prof, cfg["name"]),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, gradient of the norm network)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = gradient_cpu_baseline(cfg, chi, paths)
    print(json.dumps(out), flush=True)


def gradient_cpu_baseline(cfg, chi, paths):
    """The oracle on the host cores: value and gradient of <psi|psi> alone."""
    import torch
    from oracle import physics as OP
    from oracle.adjoint import network_grad
    from synth import workloads as W
    spec = cfg["spec"]
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    kets = OP.ket_tensors(spec, W.all_site_values(spec, cfg["seed"], std=cfg["std"]))
    net = OP.norm_network(spec, kets, conv="local")
    t0 = time.time()
    network_grad(net, paths[None], chi=chi)
    el = time.time() - t0
    return dict(value=1.0 / el, unit="contractions/s (forward + backward)", cores=cores, kind="oracle",
                sample="value and gradient of <psi|psi> (one of the %d networks of a gradient) on the same "
                       "lattice and chi (%.1f s, FP64, torch CPU with %d threads)" % (len(W.hubbard_terms(spec)) + 1,
                                                                                      el, cores))


def roofline(prof, workload):
    """Roofline entry of the dominant kernel (the single kernel with the most
    time; the permute class is one kernel template, the GEMM and factor
    classes are split into their kernels)."""
    dom = max((c for c in prof if c in KERNELS), key=lambda c: prof[c][0])
    ms, cnt, work = prof[dom][:3]
    peak, unit, bound = PEAK[dom]
    if unit == "GB/s":  # memory-bound classes are priced on their algorithmic bytes
        work = prof[dom][3]
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    achieved = work / (ms * 1e-3) / scale if ms > 0 else 0.0
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": measured_traffic(dom, workload), "kernel": dom, "launches": cnt,
            "avg_launch_ms": ms / max(cnt, 1), "work_per_launch": work / max(cnt, 1),
            "algorithmic_bytes_per_launch": prof[dom][3] / max(cnt, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32 / split-BF16 forms measured after the FP64 timed region")
    ap.add_argument("--serial", action="store_true", help="run the two contractions of a step one after the other")
    ap.add_argument("--workload", choices=["c2", "amplitudes", "gradient"], default="c2",
                    help="c2: the 40-site norm and hopping contractions (default); amplitudes: <n|psi> of the "
                         "8x8 lattice at chi = 36; gradient: Hubbard energy gradient on the 6x6 lattice")
    ap.add_argument("--batch", type=int, default=64, help="amplitudes per step (amplitude workload)")
    ap.add_argument("--workers", type=int, default=8, help="host worker threads (amplitude workload)")
    ap.add_argument("--checkpoint", type=int, default=None,
                    help="path steps per recomputation segment (gradient workload; default: one lattice "
                         "layer, 0: keep every intermediate)")
    ap.add_argument("--chi", type=int, default=0, help="bond dimension of the gradient workload (default: 32)")
    ap.add_argument("--cpu-samples", type=int, default=12, help="oracle amplitudes timed (amplitude workload)")
    ap.add_argument("--no-autotune", action="store_true", help="tile shapes from the built-in heuristic only")
    ap.add_argument("--autograd", action="store_true",
                    help="gradient workload: torch.autograd over the library's adjoints instead of the library's "
                         "network backward pass")
    ap.add_argument("--save-tuning", default=None, help="write the autotuner's table to this JSON file")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a single approximate contraction does not shard "
              "(see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2410_02215_amd as P
    from synth import workloads as W
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    P.load_library()
    if args.workload == "amplitudes":
        return main_amplitudes(args)
    if args.workload == "gradient":
        return main_gradient(args)
    cfg = W.c2()
    chi = cfg["chi"]
    paths = load_paths()
    g = gpu_setup(cfg, paths)
    autotune_setup(P, args)
    print("[bench] workload %s: warmup %d" % (cfg["name"], args.warmup), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        res, st = gpu_step(g, chi, not args.serial)
        print("[bench] warmup step done: norm mantissa %.6g exp %d" % (res[0], res[1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if not args.no_autotune:
        P.ftn.autotune(1)  # the timed steps use the stored choices only
        if args.save_tuning:
            P.ftn.autotune_save(args.save_tuning)
    tune_stats = P.ftn.autotune_stats()
    # timed steps, uninstrumented: `value`
    w0 = time.monotonic_ns()
    t0 = time.perf_counter()
    flops = 0.0
    tb_flops = 0.0
    res, st = gpu_steps(g, chi, args.steps, not args.serial, label="step")
    for x in st:
        flops += x["flops"]
        tb_flops += x["compress_textbook_flops"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w1 = time.monotonic_ns()
    # the same steps again with the library's kernel timer on (two HIP events
    # on every dispatch): per-kernel durations and the roofline. The events
    # cost host time per launch, so these steps are timed apart from `value`.
    P.ftn.profile_collect()
    P.ftn.profile_enable(True)
    p0 = time.monotonic_ns()
    tp0 = time.perf_counter()
    gpu_steps(g, chi, args.steps, not args.serial)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    p1 = time.monotonic_ns()
    P.ftn.profile_enable(False)
    prof = P.ftn.profile_collect()
    print("[bench] profiled steps done", file=sys.stderr, flush=True)
    el = t1 - t0
    ms_step = 1000.0 * el / args.steps
    value = 2.0 * args.steps / el
    norm = res[0] * 2.0 ** res[1]
    hop = (res[2] / res[0]) * 2.0 ** (res[3] - res[1])
    # dominant kernel class by time (HIP events on the library's streams)
    roof = roofline(prof, cfg["name"])
    out = {
        "metric": "ftensordot useful TFLOP/s + fPEPS contractions/sec on 1 GPU at stated err vs FP64",
        "value": value, "unit": "contractions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "sites": cfg["spec"].n_sites, "chi": chi,
                   "contractions_per_step": 2, "terms": ["norm", "hopping(first edge)"],
                   "streams": 1 if args.serial else 2,
                   "schedule": ("one stream: norm then hopping term per step" if args.serial else
                                "two streams, each running one contraction per step, alternating norm and "
                                "hopping term, no join between steps")},
        "ftensordot_useful_tflops": flops / el / 1e12,
        "textbook_tflops": {"ftensordot": flops / el / 1e12, "compression": tb_flops / el / 1e12,
                            "note": "useful block-pair GEMM flops plus the textbook QR/LQ/SVD/absorb counts of "
                                    "the compressions, per second of the timed steps"},
        "autotune": dict(tune_stats, enabled=not args.no_autotune),
        "kernel_time_ms": {c: prof[c][0] / args.steps for c in prof if prof[c][0] > 0},
        "kernel_launches": {c: prof[c][1] / args.steps for c in prof if prof[c][0] > 0},
        # algorithmic work (flops or bytes, as the class's peak is priced) and
        # algorithmic bytes per launch of every class
        "kernel_work_per_launch": {c: prof[c][2] / prof[c][1] for c in prof if prof[c][1] > 0},
        "kernel_bytes_per_launch": {c: prof[c][3] / prof[c][1] for c in prof if prof[c][1] > 0},
        "kernel_rate": {c: "%.4g %s" % (prof[c][2 if PEAK[c][1] == "TFLOP/s" else 3] / (prof[c][0] * 1e-3) /
                                        (1e12 if PEAK[c][1] == "TFLOP/s" else 1e9),
                                        PEAK[c][1])
                        for c in prof if c in PEAK and prof[c][0] > 0},
        "result": {"log2_norm": math.log2(abs(norm)) if norm else None, "hop_expectation": hop},
        "rel_err_vs_oracle": golden_errors(norm, hop),
        # CLOCK_MONOTONIC bounds of the timed steps and of their instrumented
        # repeat (kernel_* and roofline): a rocprofv3 kernel trace of the same
        # run can be cut to the latter (rocprof_summary stats <dir> <this line>)
        "timed_window_ns": [w0, w1],
        "profiled_window_ns": [p0, p1],
        "profiled_ms_per_step": 1000.0 * (tp1 - tp0) / args.steps,
        "roofline": roof,
    }
    if not args.no_forms:
        out["forms"] = c2_forms(P, cfg, g, chi, min(args.steps, 3), golden_errors)
        out["forms"]["f64"] = {"value": value, "ms_per_step": ms_step, "steps": args.steps,
                               "rel_err_vs_oracle": out["rel_err_vs_oracle"]}
        out["forms"]["note"] = ("FP32 tensors with FP32 or split-BF16 (three BF16 products, FP32 accumulation) "
                                "block GEMMs, compression and final reduction in FP64; measured after the FP64 "
                                "timed region on the same workload and streams. rel_err_vs_oracle includes the "
                                "rounding of the inputs to FP32; rel_err_vs_f64_same_inputs compares with the FP64 "
                                "path run on the rounded inputs (the error of the reduced-precision arithmetic)")
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, norm contractions: warm-up + 3)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, paths)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
