"""Summaries of rocprofv3 runs of the library, by kernel and by kernel class.

Usage (CSV output of rocprofv3, ``--output-format csv``):

    python3 -m paper_2410_02215_amd.rocprof_summary stats <dir> [<bench output>]
        per-kernel table from the ``*_kernel_stats.csv`` of a
        ``--kernel-trace --stats`` run, plus the library's profiler classes;
        with the JSON line that bench.py printed in that run, also the same
        tables over its instrumented steps only (dispatches of
        ``*_kernel_trace.csv`` inside its ``profiled_window_ns``, else its
        ``timed_window_ns``; CLOCK_MONOTONIC nanoseconds as the trace's
        timestamps), which is what the line's roofline averages over
    python3 -m paper_2410_02215_amd.rocprof_summary pmc <dir>
        per-class sums and per-launch means of every counter in the
        ``*_counter_collection.csv`` files of a ``--pmc`` run
    python3 -m paper_2410_02215_amd.rocprof_summary copy <MiB>
        one device-to-device copy of the given size (calibration target for
        the FETCH_SIZE / WRITE_SIZE counters: it reads and writes exactly
        that many bytes)

Classes match the library's own profiler (families, and single kernels
under the keys bench.py uses for its roofline): one "launch" of a class is one
timed call (a grouped GEMM is its GEMM kernel plus, when the plan splits K,
its reduction kernel; a permute is one block-permute kernel; a factor
launch is one Cholesky kernel, or one Jacobi eigensolve: its sweep kernel
plus the kernel that accumulates its eigenvectors).
"""

import csv
import glob
import os
import re
import sys

CLASSES = [
    ("gemm_f64", re.compile(r"k_gemm<double"), True),
    ("gemm_f64", re.compile(r"k_splitk_reduce<double"), False),
    ("gemm_f64", re.compile(r"k_skinny_atb<double|k_gemm_tall<"), True),
    ("gemm_f64", re.compile(r"k_skinny_reduce<double"), False),
    ("gemm_f32", re.compile(r"k_gemm<float"), True),
    ("gemm_f32", re.compile(r"k_splitk_reduce<float"), False),
    ("gemm_bf16x3", re.compile(r"k_gemm_bf16x3"), True),
    ("permute", re.compile(r"k_block_perm<"), True),
    ("factor", re.compile(r"k_jacobi_sweep|k_orth_factor|k_svd_cols"), True),
    ("factor", re.compile(r"k_jacobi_vectors"), False),
    ("copy", re.compile(r"__amd_rocclr_copyBuffer"), True),
]


def kernel_key(name):
    """The name of a kernel in the library's per-kernel profiler classes (the
    keys of bench.py's roofline), or None."""
    m = re.search(r"k_gemm<double, (\d+), (\d+),", name)
    if m:
        return "k_gemm_f64_%sx%s" % (m.group(1), m.group(2))
    if re.search(r"k_splitk_reduce<double", name):
        return "k_splitk_reduce_f64"
    if re.search(r"k_skinny_(atb|reduce)<double", name):
        return "k_skinny_f64"
    if re.search(r"k_gemm_tall<", name):
        return "k_gemm_f64_tall"
    if re.search(r"k_block_perm<", name):
        return "permute"
    for k in ("k_jacobi_sweep_la", "k_jacobi_sweep", "k_jacobi_vectors", "k_orth_factor", "k_svd_cols"):
        if re.search(r"\b%s\b" % k, name):
            return k
    return None


def kernel_class(name):
    """(class, counts_as_launch) of a kernel name, or (None, False)."""
    for cls, rx, launch in CLASSES:
        if rx.search(name):
            return cls, launch
    return None, False


def short(name):
    return re.sub(r"\(.*", "", name).strip()


def _find(d, suffix):
    out = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not out:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return out


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def stats(d, bench_out=None, top=30):
    rows = []
    for f in _find(d, "kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((short(_col(r, "Name", "KernelName")), int(_col(r, "Calls")),
                             float(_col(r, "TotalDurationNs")) / 1e6))
    _tables(rows, top)
    if bench_out:
        import json
        line = [l for l in open(bench_out).read().splitlines() if l.startswith("{")][-1]
        bl = json.loads(line)
        w0, w1 = bl.get("profiled_window_ns", bl["timed_window_ns"])
        rows = []
        for f in _find(d, "kernel_trace.csv"):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                    if a >= w0 and b <= w1:
                        rows.append((short(r["Kernel_Name"]), 1, (b - a) / 1e6))
        print("\n## Timed steps only (%.1f ms window)\n" % ((w1 - w0) / 1e6))
        _tables(rows, top)


def _tables(rows, top):
    agg = {}
    for n, c, ms in rows:
        a = agg.setdefault(n, [0, 0.0])
        a[0] += c
        a[1] += ms
    tot = sum(v[1] for v in agg.values())
    print("Kernel time %.3f ms over %d dispatches.\n" % (tot, sum(v[0] for v in agg.values())))
    print("| kernel | calls | total ms | avg us | share |")
    print("|---|---|---|---|---|")
    for n, (c, ms) in sorted(agg.items(), key=lambda x: -x[1][1])[:top]:
        print("| `%s` | %d | %.3f | %.1f | %.1f%% |" % (n, c, ms, 1000 * ms / c, 100 * ms / max(tot, 1e-30)))
    cls = {}
    for n, (c, ms) in agg.items():
        k, launch = kernel_class(n)
        if k is None:
            continue
        a = cls.setdefault(k, [0, 0.0])
        a[0] += c if launch else 0
        a[1] += ms
    keys = {}
    for n, (c, ms) in agg.items():
        k = kernel_key(n)
        if k is None:
            continue
        a = keys.setdefault(k, [0, 0.0])
        a[0] += c
        a[1] += ms
    print("\n| kernel (profiler key) | launches | total ms | avg ms per launch |")
    print("|---|---|---|---|")
    for k, (c, ms) in sorted(keys.items(), key=lambda x: -x[1][1]):
        print("| %s | %d | %.3f | %.4f |" % (k, c, ms, ms / max(c, 1)))
    print("\n| class | launches | total ms | avg ms per launch |")
    print("|---|---|---|---|")
    for k, (c, ms) in sorted(cls.items(), key=lambda x: -x[1][1]):
        print("| %s | %d | %.3f | %.4f |" % (k, c, ms, ms / max(c, 1)))


def pmc(d):
    per = {}
    launches = {}
    seen = set()
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                n = short(_col(r, "Kernel_Name", "Kernel-Name", "KernelName"))
                k, launch = kernel_class(n)
                if k is None:
                    k = "other"
                cn = _col(r, "Counter_Name", "Counter-Name", "CounterName")
                v = float(_col(r, "Counter_Value", "Counter-Value", "CounterValue"))
                did = (f, _col(r, "Dispatch_Id", "Dispatch-Id", "DispatchId"))
                per.setdefault(k, {}).setdefault(cn, 0.0)
                per[k][cn] += v
                kk = kernel_key(n)
                if kk is not None and kk != k:
                    per.setdefault(kk, {}).setdefault(cn, 0.0)
                    per[kk][cn] += v
                if did not in seen:
                    seen.add(did)
                    if launch:
                        launches[k] = launches.get(k, 0) + 1
                    if kk is not None and kk != k:
                        launches[kk] = launches.get(kk, 0) + 1
    print("| class | launches | counter | sum | per launch |")
    print("|---|---|---|---|---|")
    for k in sorted(per):
        for cn in sorted(per[k]):
            nl = launches.get(k, 0)
            print("| %s | %d | %s | %.6g | %.6g |" % (k, nl, cn, per[k][cn], per[k][cn] / max(nl, 1)))


def copy(mib):
    import torch
    n = int(mib) * (1 << 20) // 8
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes (read %d, written %d)" % (8 * n, 8 * n, 8 * n))


def main(argv):
    if len(argv) < 3 or argv[1] not in ("stats", "pmc", "copy"):
        raise SystemExit(__doc__)
    {"stats": stats, "pmc": pmc, "copy": copy}[argv[1]](*argv[2:4])


if __name__ == "__main__":
    main(sys.argv)
