"""HBM traffic of a workload's likelihood kernel from rocprofv3 counters.

Turns two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of bench.py and of its
1 GiB copy calibration into the workload's record under profiles/ (JSON):

    python -m paper_2503_08586_amd.profiling <workload> <pmc_copy_fetch dir> <pmc_copy_write dir> \\
        <pmc_kernel_fetch dir> <pmc_kernel_write dir>

with <workload> one of RECORDS (plain: the one-lens survey-scale launch;
batched: the persistent multi-lens launch of the default bench line).

The counters are read per dispatch (KiB); each is scaled by what the same
counter reads for a plain 1 GiB device copy (bytes_known / counter_reading), so
that the reported traffic is in calibrated bytes.  The record carries the
SHA-256 of the kernel sources it was measured on; bench.py reports the traffic
only while the sources still hash to that value.
"""
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# workload -> (record file, kernel-name part, the bench command the counters were taken on)
RECORDS = {
    "plain": ("traffic_plain_128px_s4_k21.txt", "k_loglike_fp32",
              "python3 bench.py --workload plain --steps 2 --warmup 1 --no-cpu-baseline"),
    "batched": ("traffic_batched_c4.txt", "k_loglike_batch",
                "python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-serving --no-plain"),
}
WORKLOAD_TEXT = {
    "plain": "plain 128x128 s=4, 21x21 PSF as given, 65,536 proposals/launch",
    "batched": "64 lenses 200x200 s=4, 41x41 Moffat PSF, FP16 split, 1,048,576 proposals/launch",
}


def record_path(workload):
    return os.path.join(ROOT, "profiles", RECORDS[workload][0])


# everything that decides what the launch does: the kernels, and the runtime
# that picks the PSF crop and the tile shape
KERNEL_SOURCES = ["paper_2503_08586_amd/csrc/lens_kernels.hip", "paper_2503_08586_amd/csrc/lens_device.h",
                  "paper_2503_08586_amd/csrc/lens_approx.h", "paper_2503_08586_amd/csrc/lens_internal.h",
                  "paper_2503_08586_amd/csrc/lens_prep.h", "paper_2503_08586_amd/csrc/lens_runtime.cpp"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_counter(d, counter, name_part):
    """Mean per-dispatch value of `counter` over dispatches whose kernel name contains
    name_part, and the (last) full kernel name matched."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals, name = [], ""
    for f in files:
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") == counter and name_part in row.get("Kernel_Name", ""):
                vals.append(float(row["Counter_Value"]))
                name = row["Kernel_Name"]
    if not vals:
        raise SystemExit("no %s rows for %s in %s" % (counter, name_part, d))
    return sum(vals) / len(vals), len(vals), name


def rel(d):
    """A counter directory as given on the command line, relative to the repository root."""
    return os.path.relpath(os.path.abspath(d), ROOT)


def main():
    workload, cf, cw, pf, pw = sys.argv[1:6]
    fname, kpart, bench_cmd = RECORDS[workload]
    copy_f, _, _ = read_counter(cf, "FETCH_SIZE", "")
    copy_w, _, _ = read_counter(cw, "WRITE_SIZE", "")
    # a 1 GiB copy reads and writes 1 GiB (2^20 KiB)
    sf, sw = 2.0 ** 20 / copy_f, 2.0 ** 20 / copy_w
    kf, nf, kname = read_counter(pf, "FETCH_SIZE", kpart)
    kw, nw, _ = read_counter(pw, "WRITE_SIZE", kpart)
    rec = {"kernel": kname.split("(")[0].replace("void lensk::", ""),
           "workload": WORKLOAD_TEXT[workload],
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
           "copy_fetch_kib": copy_f, "copy_write_kib": copy_w, "scale_fetch": sf, "scale_write": sw,
           "traffic_bytes_per_launch": (kf * sf + kw * sw) * 1024.0, "kernel_src_sha256": kernel_hash(),
           # the commands that wrote the four counter directories given here
           "commands": [
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o p -- python3 bench.py --copy-calibration"
               % rel(cf),
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o p -- python3 bench.py --copy-calibration"
               % rel(cw),
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o p -- %s" % (rel(pf), bench_cmd),
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o p -- %s" % (rel(pw), bench_cmd),
               "python -m paper_2503_08586_amd.profiling %s %s %s %s %s"
               % ((workload,) + tuple(rel(x) for x in (cf, cw, pf, pw)))]}
    with open(record_path(workload), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
