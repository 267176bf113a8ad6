"""HBM traffic of the gradient kernel from rocprofv3 hardware counters.

Each counter is read in its own profiled run (FETCH_SIZE, then WRITE_SIZE),
for the benchmark and for a plain device copy of known size; the copy gives
the scale of each counter (KiB it reports per KiB really moved), which turns
the kernel's counts into bytes ($R: the repository root, $OUT: a directory for
the profiler's output):

    cd /tmp && export TMPDIR=/tmp
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_copy_f -o c -- \\
        python3 -m paper_1611_01652_amd.traffic copy
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_copy_w -o c -- \\
        python3 -m paper_1611_01652_amd.traffic copy
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_arms_f -o b -- \\
        python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-check
    rocprofv3 --pmc WRITE_SIZE ... (same, pmc_arms_w)
    python3 -m paper_1611_01652_amd.traffic summarize --workload arms --dir $OUT

The summary (profiles/traffic_<workload>.json) holds the bytes per launch of
k_rollout_grad (or, with --kernel, another kernel: the camera's workload
`camera` takes k_render_grad) and a hash of the kernel sources it was
measured with; the
benchmark reports it only while the sources are unchanged.  With --buckets n
(a workload whose envs run in n size buckets, one reverse kernel launch each
per call, launched in bucket order) it also holds the bytes of each bucket's
launch.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ["csrc/sim_kernels.hip", "csrc/step_core.h", "csrc/drivers.h"]
# the sources of a workload's kernels where they are not the step's
WORKLOAD_SOURCES = {"camera": ["csrc/render_kernels.hip"]}
COPY_MIB = 1024


def source_hash(workload=None):
    h = hashlib.sha256()
    for f in WORKLOAD_SOURCES.get(workload, KERNEL_SOURCES):
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_main(mib=COPY_MIB, reps=4):
    """A plain device-to-device copy of `mib` MiB, `reps` times (nothing else
    runs on the device in this process)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "reps": reps}))


def read_counters(d, counter):
    """{kernel name: [per-dispatch values]} from the counter CSVs under d."""
    out = {}
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    for f in files:
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def read_dispatches(d, counter):
    """[(dispatch id, kernel name, value)] in dispatch order."""
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") == counter:
                    out.append((int(row["Dispatch_Id"]), row["Kernel_Name"], float(row["Counter_Value"])))
    return sorted(out)


def by_bucket(d, counter, kernel, n_b):
    """Mean value of each bucket's launches of `kernel` (launch j is bucket j mod n_b)."""
    v = [x for _, k, x in read_dispatches(d, counter) if kernel in k]
    if not v or len(v) % n_b:
        raise ValueError(f"{len(v)} dispatches of {kernel} do not split into {n_b} buckets")
    return [sum(v[i::n_b]) / len(v[i::n_b]) for i in range(n_b)]


def per_dispatch(vals, match):
    ks = [k for k in vals if match(k)]
    if not ks:
        raise KeyError("kernel not found among " + ", ".join(sorted(vals)[:10]))
    v = [x for k in ks for x in vals[k]]
    return sum(v) / len(v), len(v), ks


def summarize(workload, d, kernel="k_rollout_grad", buckets=None):
    expect_kib = COPY_MIB * 1024.0
    is_copy = lambda k: "copy" in k.lower() or "elementwise" in k.lower()   # noqa: E731
    cf, ncf, _ = per_dispatch(read_counters(os.path.join(d, "pmc_copy_f"), "FETCH_SIZE"), is_copy)
    cw, ncw, _ = per_dispatch(read_counters(os.path.join(d, "pmc_copy_w"), "WRITE_SIZE"), is_copy)
    kf, nkf, names = per_dispatch(read_counters(os.path.join(d, f"pmc_{workload}_f"), "FETCH_SIZE"),
                                  lambda k: kernel in k)
    kw, nkw, _ = per_dispatch(read_counters(os.path.join(d, f"pmc_{workload}_w"), "WRITE_SIZE"),
                              lambda k: kernel in k)
    sf, sw = cf / expect_kib, cw / expect_kib
    out = dict(workload=workload, kernel=kernel, kernel_names=names,
               fetch_kib_per_dispatch=kf, write_kib_per_dispatch=kw, dispatches=[nkf, nkw],
               copy_kib_expected=expect_kib, copy_fetch_kib=cf, copy_write_kib=cw,
               fetch_scale=sf, write_scale=sw,
               bytes_per_launch=(kf / sf + kw / sw) * 1024.0,
               fetch_bytes_per_launch=kf / sf * 1024.0, write_bytes_per_launch=kw / sw * 1024.0,
               kernel_source_hash=source_hash(workload))
    if buckets:
        bf = by_bucket(os.path.join(d, f"pmc_{workload}_f"), "FETCH_SIZE", kernel, buckets)
        bw = by_bucket(os.path.join(d, f"pmc_{workload}_w"), "WRITE_SIZE", kernel, buckets)
        out["bytes_per_launch_by_bucket"] = [(f / sf + w / sw) * 1024.0 for f, w in zip(bf, bw)]
    # the other kernels of the gradient and the forward, when the run has them
    for other in ("k_recompute", "k_rollout<", "k_rollout_keep", "k_render("):
        try:
            of, _, _ = per_dispatch(read_counters(os.path.join(d, f"pmc_{workload}_f"), "FETCH_SIZE"),
                                    lambda k: other in k)
            ow, _, _ = per_dispatch(read_counters(os.path.join(d, f"pmc_{workload}_w"), "WRITE_SIZE"),
                                    lambda k: other in k)
            out["other_kernels"] = out.get("other_kernels", {})
            out["other_kernels"][other.rstrip("<(")] = dict(fetch_bytes_per_launch=of / sf * 1024.0,
                                                           write_bytes_per_launch=ow / sw * 1024.0)
        except KeyError:
            pass
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return out


def load(workload, bucket=None, all_buckets=False):
    """Bytes per launch (of `bucket`'s launch, or with all_buckets the sum
    over the buckets' launches of one call, where measured by bucket), or
    None when missing or measured on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("kernel_source_hash") != source_hash(workload):
        return None
    b = t.get("bytes_per_launch_by_bucket")
    if b and all_buckets:
        return float(sum(b))
    if b and bucket is not None:
        return b[bucket] if 0 <= bucket < len(b) else None
    return t.get("bytes_per_launch")


def load_other(workload, kernel, launches):
    """Bytes of `launches` launches of another kernel of the same run (the
    mean per launch times the count), or None as load()."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    o = (t.get("other_kernels") or {}).get(kernel)
    if t.get("kernel_source_hash") != source_hash(workload) or not o:
        return None
    return float(launches * (o["fetch_bytes_per_launch"] + o["write_bytes_per_launch"]))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["copy", "summarize", "hash"])
    ap.add_argument("--workload", default="arms")
    ap.add_argument("--dir", help="directory holding the profiler's pmc_* output folders")
    ap.add_argument("--buckets", type=int, default=None, help="size buckets of the workload (one launch each per call)")
    ap.add_argument("--kernel", default="k_rollout_grad", help="the kernel whose launches are summarized")
    a = ap.parse_args()
    if a.cmd == "copy":
        copy_main()
    elif a.cmd == "summarize":
        if not a.dir:
            ap.error("summarize needs --dir")
        summarize(a.workload, a.dir, kernel=a.kernel, buckets=a.buckets)
    else:
        print(source_hash(a.workload))
    sys.exit(0)
