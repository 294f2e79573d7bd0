"""HBM traffic per kernel launch from rocprofv3 counter runs.

Reads the counter_collection CSVs of four `rocprofv3 --pmc ... --output-format csv`
runs: FETCH_SIZE and WRITE_SIZE of the benchmark, and the same two counters of a
device-to-device copy of known size (`bench.py --copy-probe MiB`).  The copy
gives the factor between each counter (KiB per dispatch) and the bytes actually
moved; the benchmark's per-kernel averages over its one-item dispatches (the
kernel's smallest grid) are scaled by it.  Writes a JSON
summary keyed by the stages of one CG iteration, with a hash of the sources of
the measured kernels, so that a reader can tell when they have changed since.

Usage (plain script, does not load the library):
  python paper_2307_14437_amd/pmc.py FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR COPY_MIB OUT.json
"""

from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# stage of a CG iteration -> kernel symbol fragment (single-precision grid, 2D, L = 2048)
STAGE_SYMBOLS = {   # fragments that together name the kernel of each stage
    "passA": ("k_passA<float, 2048", "SrcPairSegRows"),
    "passA_rows": ("k_passA<float, 2048", "SrcPairGatherRows"),     # the form of IC(1)-preconditioned items
    "passB": ("k_passB<float, 2048", "true>"),
    "passC": ("k_passC<float, float, 2048", "true"),
    "scatter": ("k_vertex_cg",),
}


# the sources of the measured kernels (the FFT passes, the vertex CG kernel) and the headers they include
KERNEL_SOURCES = ("conv.hip", "conv_common.h", "fft.h", "solver.hip", "cg_state.h", "cg_items.h", "bary.h",
                  "internal.h")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.path.join(HERE, "csrc", n) for n in KERNEL_SOURCES):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _load(d):
    """Counter values per kernel, of the dispatches with the kernel's smallest grid: the launches that cover
    one item (batched launches cover several items along the grid's y axis)."""
    rows = collections.defaultdict(list)
    for path in glob.glob(os.path.join(d, "*counter_collection.csv")):
        for r in csv.DictReader(open(path)):
            rows[r["Kernel_Name"]].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    out = {}
    for k, v in rows.items():
        g = min(x[0] for x in v)
        out[k] = [x[1] for x in v if x[0] == g]
    return out


def main(argv):
    fdir, wdir, fcdir, wcdir, mib, out = argv
    copy_bytes = int(mib) * (1 << 20)
    F, Wr, Fc, Wc = _load(fdir), _load(wdir), _load(fcdir), _load(wcdir)
    copy = [k for k in Fc if "copyBuffer" in k][0]
    kf = copy_bytes / (sum(Fc[copy]) / len(Fc[copy]) * 1024)      # bytes per counted byte, FETCH_SIZE
    kw = copy_bytes / (sum(Wc[copy]) / len(Wc[copy]) * 1024)      # the same for WRITE_SIZE
    stages = {}
    for st, frag in STAGE_SYMBOLS.items():
        names = [k for k in F if all(f in k for f in frag)]
        if not names:
            continue
        k = max(names, key=lambda n: len(F[n]))      # the launch the iterations used most
        f = sum(F[k]) / len(F[k]) * 1024 * kf
        w = sum(Wr[k]) / len(Wr[k]) * 1024 * kw if k in Wr else 0.0
        name = k.replace("(anonymous namespace)::", "").split("(")[0]
        stages[st] = {"kernel": name, "dispatches": len(F[k]), "fetch_bytes": f, "write_bytes": w,
                      "bytes": f + w}
    res = {"source_hash": source_hash(), "fetch_factor": kf, "write_factor": kw, "copy_bytes": copy_bytes,
           "stages": stages}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(f"FETCH_SIZE factor {kf:.4f}, WRITE_SIZE factor {kw:.4f} (copy of {copy_bytes} bytes)")
    print("| stage | kernel | dispatches | fetched MB | written MB |")
    print("|---|---|---|---|---|")
    for st, v in stages.items():
        print(f"| {st} | `{v['kernel']}` | {v['dispatches']} | {v['fetch_bytes'] / 1e6:.2f} | {v['write_bytes'] / 1e6:.2f} |")


if __name__ == "__main__":
    main(sys.argv[1:])
