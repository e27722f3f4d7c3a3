"""Summaries of rocprofv3 counter databases for the step kernels: HBM bytes per launch from
FETCH_SIZE / WRITE_SIZE (scaled by what the same counters read for a device copy of known size)
and VALU, LDS and memory instructions per lattice update from the SQ counters.  Host code only
(sqlite): it reads databases a profiled `bench.py` run wrote and writes the JSON tables
`bench.py` reads back (`profiles/traffic.json`, `profiles/valu.json`), each entry tagged with
the digest of the kernel sources it was measured on.

    python3 -m paper_1812_05401_amd.counters traffic --out profiles/traffic.json \\
        --copy FETCH_DIR,WRITE_DIR --copy-bytes 1073741824 WORKLOAD:STORAGE=FETCH_DIR,WRITE_DIR ...
    python3 -m paper_1812_05401_amd.counters valu --out profiles/valu.json \\
        WORKLOAD:STORAGE=DIR ...
    python3 -m paper_1812_05401_amd.counters trace DIR

Each DIR is a `rocprofv3 --pmc ... -d DIR` output folder of one run (its .db files are found
below it).  The step kernels of a run are `vplbm::step3_kernel` (three lattice updates per
launch), `vplbm::step2_kernel` (two) and `vplbm::step_kernel` (one); per kernel the median over
its dispatches is taken.
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sqlite3
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("kernels.hip", "lattice.hpp", "kernels.hpp", "runtime.hip")


def source_digest(csrc=None):
    """Digest of the code the step kernels are built from (the sources in csrc, by default the
    package's): a counter summary taken on other code is not used.  Comments and the layout of
    whitespace are left out, so that an edit of a comment does not discard a summary."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc or os.path.join(HERE, "csrc"), f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def element_bytes(storage):
    return {"f64": 8, "f32": 4, "f32d": 4}.get(storage, 2)


def bytes_per_update(storage):
    """One load and one store of the nine populations and the 1-byte mask of a node."""
    return 18 * element_bytes(storage) + 1


def kernel_short_name(name):
    """A kernel's name without its argument list and a leading return type (an anonymous
    namespace is kept as `(anonymous namespace)::`)."""
    n = name.replace("(anonymous namespace)::", "\0")
    n = re.sub(r"\(.*", "", n).strip().replace("\0", "(anonymous namespace)::")
    return n[5:] if n.startswith("void ") else n


def dispatch_values(folder):
    """{(kernel name without its argument list, counter): [value per dispatch]} from every
    rocprofv3 database below `folder`."""
    dbs = sorted(glob.glob(os.path.join(folder, "**", "*.db"), recursive=True))
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database below {folder}")
    out = {}
    for db in dbs:
        con = sqlite3.connect(db)
        try:
            for k, c, v in con.execute("select kernel_name, counter_name, value "
                                       "from counters_collection"):
                out.setdefault((kernel_short_name(k), c), []).append(float(v))
        finally:
            con.close()
    return out


def step_kernels(vals, counter):
    """{updates per launch: (kernel name, dispatches, median value)} for the step kernels that
    carry `counter`; where a run has several instantiations of one kernel, the one with the most
    dispatches."""
    best = {}
    for (k, c), vs in vals.items():
        if c != counter:
            continue
        if k.startswith("vplbm::step3_kernel"):
            spl = 3
        elif k.startswith("vplbm::step2_kernel"):
            spl = 2
        elif k.startswith("vplbm::step_kernel"):
            spl = 1
        else:
            continue
        if spl not in best or len(vs) > best[spl][1]:
            best[spl] = (k, len(vs), statistics.median(vs))
    return best


def copy_scale(folder, counter, copy_bytes):
    """Bytes per counted KiB: the copy kernel's known bytes over what `counter` reads for it."""
    vals = dispatch_values(folder)
    cands = [(statistics.median(vs), k, len(vs)) for (k, c), vs in vals.items()
             if c == counter and "copyBuffer" in k]
    if not cands:
        raise ValueError(f"no copy kernel with {counter} in {folder}")
    med, k, n = max(cands)
    return copy_bytes / 1024.0 / med, {"kernel": k, "dispatches": n, "median_kib": med}


def workload_case(name):
    from . import inputs as I
    mk = {"cylinder_wake_2048x512": I.cylinder_wake_2048x512,
          "cylinder_wake_8192x2048": lambda: I.cylinder_wake_8192x2048("f32"),
          "oscillating_cylinder_8192x2048": I.oscillating_cylinder_8192x2048,
          "paper_cylinder_re500": I.paper_cylinder_re500,
          "taylor_couette_128": I.taylor_couette_128}
    return mk[name]()


def moving(case):
    return any(b["freq"] != 0 and (b["ax"] != 0 or b["ay"] != 0) for b in case.bodies)


def parse_spec(spec):
    head, dirs = spec.split("=", 1)
    workload, storage = head.split(":")
    return workload, storage, dirs.split(",")


def traffic(specs, copy_dirs, copy_bytes, profile="profiles/step_kernel_hbm_traffic.md"):
    fs, fcal = copy_scale(copy_dirs[0], "FETCH_SIZE", copy_bytes)
    ws, wcal = copy_scale(copy_dirs[1], "WRITE_SIZE", copy_bytes)
    digest = source_digest()
    table, rows = {}, []
    for spec in specs:
        workload, storage, (fdir, wdir) = parse_spec(spec)
        case = workload_case(workload)
        fk = step_kernels(dispatch_values(fdir), "FETCH_SIZE")
        wk = step_kernels(dispatch_values(wdir), "WRITE_SIZE")
        for spl in sorted(fk, reverse=True):
            if spl not in wk:
                continue
            kname, n, fkib = fk[spl]
            wkib = wk[spl][2]
            rd, wr = fkib * 1024 * fs, wkib * 1024 * ws
            # moving bodies: a launch of several steps reads the mask of each of its steps
            alg = (bytes_per_update(storage) + (spl - 1 if moving(case) else 0)) * case.nodes
            ent = {"kernel": kname, "dispatches": n, "lattice_updates_per_launch": spl,
                   "fetch_kib_raw": fkib, "write_kib_raw": wkib,
                   "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                   "bytes_per_launch": int(round(rd + wr)), "algorithmic_bytes_per_launch": alg,
                   "ratio_to_algorithmic": round((rd + wr) / alg, 4),
                   "bytes_per_lattice_update": round((rd + wr) / (case.nodes * spl), 2),
                   "source_digest": digest, "profile": profile}
            table[f"{workload}/{storage}/{spl}"] = ent
            rows.append(f"| `{kname}` | {spl} | {workload} ({case.nodes:,} nodes, {storage}) | {n} | "
                        f"{fkib:,.0f} | {wkib:,.0f} | {rd / 1e6:.1f} MB | {wr / 1e6:.1f} MB | "
                        f"{(rd + wr) / 1e6:.1f} MB | {alg / 1e6:.1f} MB | "
                        f"{ent['ratio_to_algorithmic']:.3f} | {ent['bytes_per_lattice_update']:.1f} |")
    head = [f"Kernel source digest: `{digest}`.",
            f"Calibration: `{fcal['kernel']}` ({fcal['dispatches']} dispatches) reads "
            f"{fcal['median_kib']:,.0f} KiB FETCH_SIZE and {wcal['median_kib']:,.0f} KiB WRITE_SIZE "
            f"for {copy_bytes / 1024:,.0f} KiB each way: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f}.",
            "",
            "| kernel | updates per launch | workload | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB "
            "| read | write | per launch | algorithmic | ratio | bytes per lattice update |",
            "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    return table, head + rows


SQ = ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
      "SQ_INSTS_LDS")


def valu(specs, profile="profiles/step_kernels_valu.md"):
    digest = source_digest()
    table, rows = {}, []
    for spec in specs:
        workload, storage, (folder,) = parse_spec(spec)
        case = workload_case(workload)
        vals = dispatch_values(folder)
        per = {c: step_kernels(vals, c) for c in SQ}
        for spl in sorted(per["SQ_INSTS_VALU"], reverse=True):
            kname, n, v = per["SQ_INSTS_VALU"][spl]
            get = lambda c: per[c][spl][2] if spl in per[c] else float("nan")
            upd = case.nodes * spl
            ent = {"kernel": kname, "dispatches": n, "lattice_updates_per_launch": spl,
                   "valu_lane_instr_per_launch": int(round(v * 64)),
                   "valu_per_lattice_update": round(v * 64 / upd, 1),
                   "lds_per_lattice_update": round(get("SQ_INSTS_LDS") * 64 / upd, 1),
                   "vmem_rd_per_lattice_update": round(get("SQ_INSTS_VMEM_RD") * 64 / upd, 2),
                   "salu_per_wave": round(get("SQ_INSTS_SALU") / get("SQ_WAVES"), 1),
                   "waves": int(get("SQ_WAVES")), "source_digest": digest, "profile": profile}
            table[f"{workload}/{storage}/{spl}"] = ent
            rows.append(f"| {workload} | {storage} | `{kname}` | {spl} | "
                        f"{ent['valu_per_lattice_update']:.1f} | {ent['lds_per_lattice_update']:.1f} | "
                        f"{ent['vmem_rd_per_lattice_update']:.2f} | {ent['salu_per_wave']:.1f} |")
    head = [f"Kernel source digest: `{digest}`.", "",
            "| workload | storage | kernel | updates per launch | VALU / update | LDS / update "
            "| VMEM reads / update | SALU / wave |",
            "|---|---|---|---|---|---|---|---|"]
    return table, head + rows


def trace(folder):
    """Kernel-trace summary of a `rocprofv3 --kernel-trace` run: per kernel and grid size the
    calls and their mean, min and max duration; then the step kernels' dispatches in launch
    order, cut into segments of consecutive launches of one kernel and grid (a workload's warmup
    and timed launches form their own segments), so that the launches a bench.py measurement
    timed can be read apart from other workloads that run the same kernel."""
    dbs = sorted(glob.glob(os.path.join(folder, "**", "*.db"), recursive=True))
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database below {folder}")
    disp = []
    for db in dbs:
        con = sqlite3.connect(db)
        try:
            disp += con.execute("select name, start, duration, grid_x * grid_y * grid_z, "
                                "workgroup_x, vgpr_count, lds_size from kernels").fetchall()
        finally:
            con.close()
    disp.sort(key=lambda r: r[1])
    short = kernel_short_name
    groups = {}
    for name, _, dur, grid, wg, vg, lds in disp:
        groups.setdefault((short(name), grid, wg, vg, lds), []).append(dur / 1e3)
    lines = ["| kernel | grid | workgroup | calls | avg µs | min µs | max µs | VGPRs | LDS bytes |",
             "|---|---|---|---|---|---|---|---|---|"]
    for (k, grid, wg, vg, lds), ds in sorted(groups.items(), key=lambda x: -sum(x[1])):
        lines.append(f"| `{k}` | {grid} | {wg} | {len(ds)} | {statistics.mean(ds):.2f} | "
                     f"{min(ds):.2f} | {max(ds):.2f} | {vg} | {lds} |")
    segs = []
    for name, _, dur, grid, *_ in disp:
        k = short(name)
        if not k.startswith(("vplbm::step3_kernel", "vplbm::step2_kernel", "vplbm::step_kernel")):
            continue
        if segs and segs[-1][0] == (k, grid):
            segs[-1][1].append(dur / 1e3)
        else:
            segs.append(((k, grid), [dur / 1e3]))
    lines += ["", "Step-kernel launches in order, in segments of one kernel and grid:", "",
              "| segment | kernel | grid | launches | avg µs | min µs | max µs |",
              "|---|---|---|---|---|---|---|"]
    for i, ((k, grid), ds) in enumerate(segs):
        lines.append(f"| {i} | `{k}` | {grid} | {len(ds)} | {statistics.mean(ds):.2f} | "
                     f"{min(ds):.2f} | {max(ds):.2f} |")
    return groups, segs, lines


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("kind", choices=["traffic", "valu", "trace"])
    ap.add_argument("specs", nargs="+", metavar="WORKLOAD:STORAGE=DIR[,DIR] (trace: DIR)")
    ap.add_argument("--out", default="", help="traffic, valu: JSON table to write")
    ap.add_argument("--copy", default="", help="traffic: FETCH_DIR,WRITE_DIR of the copy run")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    a = ap.parse_args(argv)
    if a.kind == "trace":
        print("\n".join(trace(a.specs[0])[2]))
        return 0
    if not a.out:
        ap.error(f"{a.kind} needs --out")
    if a.kind == "traffic":
        if not a.copy:
            ap.error("traffic needs --copy FETCH_DIR,WRITE_DIR")
        table, lines = traffic(a.specs, a.copy.split(","), a.copy_bytes)
    else:
        table, lines = valu(a.specs)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
