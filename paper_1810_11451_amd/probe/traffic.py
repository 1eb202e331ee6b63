"""HBM traffic per launch from rocprofv3 counter runs.

    python -m paper_1810_11451_amd.probe.traffic --key full-width-fp32 \\
        --kernel apply_fp32 --fetch K_FETCH.csv --write K_WRITE.csv \\
        --copy-fetch C_FETCH.csv --copy-write C_WRITE.csv --copy-bytes 1073741824 \\
        --algorithmic-bytes 786432000 --command "..."

FETCH_SIZE and WRITE_SIZE (KiB per dispatch, from `rocprofv3 --pmc ...
--output-format csv`) are averaged over the dispatches whose name contains
--kernel, then each is scaled by the factor that makes the same counter
read the known traffic of the plain copy probe (`probe/hbm.py`, which
reads and writes --copy-bytes per dispatch).  The result is stored in
profiles/traffic.json under --key, with the hash of the kernel sources and
the launch variant (--variant), so that bench.py reports it only while the
kernels and the variant it launches are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[2]
KERNEL_SOURCES = ["paper_1810_11451_amd/csrc/bf_kernels.hip",
                  "paper_1810_11451_amd/csrc/bf_internal.h"]
FILTER_SOURCES = ["paper_1810_11451_amd/csrc/bf_filter.hip",
                  "paper_1810_11451_amd/csrc/bf_fft.h"]
TRAFFIC_JSON = ROOT / "profiles" / "traffic.json"


def _code_only(text: str) -> str:
    """Source text without comments and blank lines, each line stripped, so
    that edits to comments alone do not change a kernel's hash.  (Only line
    comments are used in these sources; a "//" inside a string literal would
    be cut too, which only makes the hash stricter.)"""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].strip()
        if code:
            out.append(code)
    return "\n".join(out)


def kernel_sha(key: str = "") -> str:
    """Hash of the code (comments left out) of the kernel sources a traffic
    entry depends on: the filter stage's for keys naming it, else the
    beamforming kernels'."""
    h = hashlib.sha256()
    for p in (FILTER_SOURCES if "filter" in key else KERNEL_SOURCES):
        h.update(_code_only((ROOT / p).read_text()).encode())
    return h.hexdigest()[:16]


def _col(header, *names):
    low = [h.lower() for h in header]
    for n in names:
        if n.lower() in low:
            return low.index(n.lower())
    raise KeyError(f"none of {names} in {header}")


def counter_mean_kib(path: str, counter: str, kernel_substr: str) -> tuple[float, int]:
    """Mean value (KiB) of `counter` over dispatches of kernels matching."""
    with open(path, newline="") as fh:
        rows = list(csv.reader(fh))
    hdr = rows[0]
    kn = _col(hdr, "Kernel_Name", "kernel_name")
    cn = _col(hdr, "Counter_Name", "counter_name")
    cv = _col(hdr, "Counter_Value", "value")
    vals = [float(r[cv]) for r in rows[1:] if kernel_substr in r[kn] and r[cn] == counter]
    if not vals:
        raise ValueError(f"no {counter} rows for '{kernel_substr}' in {path}")
    return sum(vals) / len(vals), len(vals)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--key", required=True)
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--algorithmic-bytes", type=int, required=True)
    ap.add_argument("--variant", default=None,
                    help="launch variant the counters were taken on, schedule:wg_per_cu:order:store")
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)

    f_kib, nf = counter_mean_kib(a.fetch, "FETCH_SIZE", a.kernel)
    w_kib, nw = counter_mean_kib(a.write, "WRITE_SIZE", a.kernel)
    cf_kib, _ = counter_mean_kib(a.copy_fetch, "FETCH_SIZE", "copy_kernel")
    cw_kib, _ = counter_mean_kib(a.copy_write, "WRITE_SIZE", "copy_kernel")
    k_fetch = a.copy_bytes / (cf_kib * 1024.0)
    k_write = a.copy_bytes / (cw_kib * 1024.0)
    fetch_b = f_kib * 1024.0 * k_fetch
    write_b = w_kib * 1024.0 * k_write
    entry = {
        "kernel_sha": kernel_sha(a.key),
        "kernel": a.kernel,
        "fetch_kib_per_dispatch": round(f_kib, 1), "write_kib_per_dispatch": round(w_kib, 1),
        "dispatches": [nf, nw],
        "copy_probe_bytes": a.copy_bytes,
        "scale_fetch": round(k_fetch, 4), "scale_write": round(k_write, 4),
        "fetch_bytes_per_launch": int(fetch_b), "write_bytes_per_launch": int(write_b),
        "traffic_bytes_per_launch": int(fetch_b + write_b),
        "algorithmic_bytes_per_launch": a.algorithmic_bytes,
        "traffic_over_algorithmic": round((fetch_b + write_b) / a.algorithmic_bytes, 4),
        "command": a.command,
    }
    if a.variant is not None:
        entry["variant"] = a.variant
    data = json.loads(TRAFFIC_JSON.read_text()) if TRAFFIC_JSON.exists() else {}
    data[a.key] = entry
    TRAFFIC_JSON.parent.mkdir(exist_ok=True)
    TRAFFIC_JSON.write_text(json.dumps(data, indent=1, sort_keys=True) + "\n")
    print(json.dumps({a.key: entry}, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
