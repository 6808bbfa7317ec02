"""HBM traffic of the likelihood kernel from rocprofv3 counters.

Turns two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of bench.py and of its
1 GiB copy calibration into profiles/traffic_plain_128px_s4_k21.txt (JSON):

    python -m paper_2503_08586_amd.profiling <pmc_copy_fetch dir> <pmc_copy_write dir> \\
        <pmc_plain_fetch dir> <pmc_plain_write dir>

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
RECORD = os.path.join(ROOT, "profiles", "traffic_plain_128px_s4_k21.txt")
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
    cf, cw, pf, pw = sys.argv[1:5]
    copy_f, _, _ = read_counter(cf, "FETCH_SIZE", "")
    copy_w, _, _ = read_counter(cw, "WRITE_SIZE", "")
    # a 1 GiB copy reads and writes 1 GiB (2^20 KiB)
    sf, sw = 2.0 ** 20 / copy_f, 2.0 ** 20 / copy_w
    kf, nf, kname = read_counter(pf, "FETCH_SIZE", "k_loglike_fp32")
    kw, nw, _ = read_counter(pw, "WRITE_SIZE", "k_loglike_fp32")
    rec = {"kernel": kname.split("(")[0].replace("void lensk::", ""),
           "workload": "plain 128x128 s=4, 21x21 PSF as given, 65,536 proposals/launch",
           "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
           "copy_fetch_kib": copy_f, "copy_write_kib": copy_w, "scale_fetch": sf, "scale_write": sw,
           "traffic_bytes_per_launch": (kf * sf + kw * sw) * 1024.0, "kernel_src_sha256": kernel_hash(),
           # the commands that wrote the four counter directories given here
           "commands": [
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o p -- python3 bench.py --copy-calibration"
               % rel(cf),
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o p -- python3 bench.py --copy-calibration"
               % rel(cw),
               "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o p -- "
               "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline" % rel(pf),
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o p -- "
               "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline" % rel(pw),
               "python -m paper_2503_08586_amd.profiling %s %s %s %s" % tuple(rel(x) for x in (cf, cw, pf, pw))]}
    with open(RECORD, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
