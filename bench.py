"""Benchmark: H-matrix DD-BEM products and solves on one MI355X.

Workload (the primary throughput configuration): planar fault of 256 x 256
square elements, h = 1 m (65,536 elements, 196,608 DOF), E = 30 GPa,
nu = 0.25; H-matrix with leaf 64, eta 2, ACA tolerance 1e-6; a batch of 16
seeded N(0,1) right-hand sides.  One step = one batched H-matrix product
(all 16 columns) in the FP32 form (FP32 dense leaves and low-rank factors,
FP32 accumulation); inputs and outputs resident in HBM.

Prints one JSON line on stdout.  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

YOUNG, NU = 30e9, 0.25
HBM_PEAK_GBS = 8000.0
NRHS = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("hm_apply.hip", "hm_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2605_14397_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof/trace -o primary -- "
             "python3 bench.py --only fp32 --steps 20 --warmup 3 --no-gmres --no-cpu-baseline --no-forms",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \"k_phase|k_reduceT|k_gather|k_scatter\" "
             "--output-format csv -d gpurun_out/prof/fetch -o primary -- "
             "python3 bench.py --only fp32 --steps 3 --warmup 1 --no-gmres --no-cpu-baseline --no-forms",
    "write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex \"k_phase|k_reduceT|k_gather|k_scatter\" "
             "--output-format csv -d gpurun_out/prof/write -o primary -- "
             "python3 bench.py --only fp32 --steps 3 --warmup 1 --no-gmres --no-cpu-baseline --no-forms",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \"copy|Copy\" --output-format csv "
                  "-d gpurun_out/prof/copy_fetch -o copy -- python3 bench.py --form copy --steps 3",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex \"copy|Copy\" --output-format csv "
                  "-d gpurun_out/prof/copy_write -o copy -- python3 bench.py --form copy --steps 3",
}
IF_PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_if/trace -o interface -- "
             "python3 bench.py --form interface --if-states mixed --steps 20 --warmup 3 --no-cpu-baseline",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex interface --output-format csv "
             "-d gpurun_out/prof_if/fetch -o interface -- "
             "python3 bench.py --form interface --if-states mixed --steps 3 --warmup 1 --no-cpu-baseline",
    "write": "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex interface --output-format csv "
             "-d gpurun_out/prof_if/write -o interface -- "
             "python3 bench.py --form interface --if-states mixed --steps 3 --warmup 1 --no-cpu-baseline",
}
# MFMA activity and L2 hits of the phase kernels (one counter group per run)
COUNTER_COMMANDS = {
    "mfma": "rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --kernel-include-regex "
            "\"k_phase\" --output-format csv -d gpurun_out/prof/mfma -o primary -- "
            "python3 bench.py --only fp32 --steps 3 --warmup 1 --no-gmres --no-cpu-baseline --no-forms",
    "l2": "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --kernel-include-regex \"k_phase\" --output-format csv "
          "-d gpurun_out/prof/l2 -o primary -- "
          "python3 bench.py --only fp32 --steps 3 --warmup 1 --no-gmres --no-cpu-baseline --no-forms",
}
PHASE_KERNELS = ("k_gather", "k_phaseA", "k_reduceT", "k_phaseB", "k_scatter")


def _kernel_base(name: str) -> str:
    s = name.split("(")[0].replace("void ", "").replace("hm::", "").strip()
    return s.split("<")[0]


def summarize_profiles(prof_dir: str):
    """Write profiles/traffic.json, profiles/traffic_primary_fp32.md and
    profiles/kernel_stats_primary_fp32.md from the CSV output of
    PROFILE_COMMANDS (run from the repository root with TMPDIR=/tmp)."""
    import csv
    import glob

    def counters(sub):
        f = glob.glob(os.path.join(prof_dir, sub, "*counter_collection.csv"))[0]
        rows = list(csv.DictReader(open(f)))
        per = {}
        for r in rows:
            k = _kernel_base(r["Kernel_Name"])
            per.setdefault(k, []).append(float(r["Counter_Value"]))
        return per

    fetch, write = counters("fetch"), counters("write")
    cf, cw = counters("copy_fetch"), counters("copy_write")
    copy_kib = 2 * 1024 * 1024  # 2 GiB read and 2 GiB written per copy dispatch
    ck = [k for k in cf if "opy" in k][0]
    fetch_scale = copy_kib / (sum(cf[ck]) / len(cf[ck]))
    write_scale = copy_kib / (sum(cw[ck]) / len(cw[ck]))
    products = len(fetch["k_gather1"])  # one gather per product
    kern = {}
    for k in PHASE_KERNELS:
        names = [n for n in fetch if n.startswith(k)]
        fk = sum(sum(fetch[n]) for n in names) / products
        wk = sum(sum(write.get(n, [])) for n in names) / products
        kern[k] = {"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                   "hbm_bytes_per_launch": int(1024 * (fk * fetch_scale + wk * write_scale))}
    d = {"source_hash": source_hash(), "fetch_scale": round(fetch_scale, 5), "write_scale": round(write_scale, 5),
         "workload": "256x256 planar fault, 16 RHS, FP32 form (leaf 64, eta 2, ACA 1e-6)",
         "per": "one product (all launches of the kernel in one product)", "kernels": kern}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(d, fh, indent=1)
    lines = ["# HBM traffic per product: 256x256 planar fault, 16 RHS, FP32 form", "",
             "Commands (one counter per run, from the repository root, `TMPDIR=/tmp`):", "", "```"]
    lines += [PROFILE_COMMANDS[k] for k in ("fetch", "write", "copy_fetch", "copy_write")]
    lines += ["```", "", f"Calibration: a plain device copy of 2 GiB (torch `copy_`, 2,097,152 KiB read and written) "
              f"gives FETCH_SIZE scale {fetch_scale:.4f} and WRITE_SIZE scale {write_scale:.4f}.", "",
              f"Counters summed over every launch of a kernel in one product ({products} products profiled).", "",
              "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | scaled HBM bytes per product |", "|---|---|---|---|"]
    for k, v in kern.items():
        lines.append(f"| `{k}` | {v['fetch_kib']:,.1f} | {v['write_kib']:,.1f} | {v['hbm_bytes_per_launch']:,} |")
    lines += ["", f"Apply source hash `{d['source_hash']}` (`profiles/traffic.json`); `bench.py` reports "
              "`roofline.traffic` only while the apply source matches it."]
    with open(os.path.join(ROOT, "profiles", "traffic_primary_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    f = glob.glob(os.path.join(prof_dir, "trace", "*kernel_stats.csv"))[0]
    rows = list(csv.DictReader(open(f)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel statistics: 256x256 planar fault, 16 RHS, FP32 form", "", "Command (from the repository root, "
             "`TMPDIR=/tmp`):", "", "```", PROFILE_COMMANDS["trace"], "```", "",
             "| kernel | calls | average us | min us | max us | share of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows[:16]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} % |")
    per_product = {}
    for r in rows:
        k = _kernel_base(r["Name"])
        for p in PHASE_KERNELS:
            if k.startswith(p):
                per_product[p] = per_product.get(p, 0.0) + float(r["TotalDurationNs"])
    calls = sum(int(r["Calls"]) for r in rows if _kernel_base(r["Name"]).startswith("k_gather"))
    lines += ["", f"Per product ({calls} products; phase kernels summed over their launches of one product):", ""]
    for p, ns in per_product.items():
        lines.append(f"* `{p}`: {ns / calls / 1e3:.1f} us")
    with open(os.path.join(ROOT, "profiles", "kernel_stats_primary_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(d))


MIXED_PROFILE_COMMAND = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_mixed/trace "
                         "-o mixed -- python3 bench.py --only mixed --steps 20 --warmup 3 --no-gmres "
                         "--no-cpu-baseline --no-forms")


def summarize_mixed_profile(prof_dir: str):
    """profiles/ kernel statistics of the precision form's product (FP32 near,
    BF16 far) on the primary workload."""
    import csv

    rows = list(csv.DictReader(open(os.path.join(prof_dir, "trace", "mixed_kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel statistics: 256x256 planar fault, 16 RHS, FP32 near / BF16 far form", "",
             "Command (from the repository root, `TMPDIR=/tmp`):", "", "```", MIXED_PROFILE_COMMAND, "```", "",
             "| kernel | calls | average us | min us | max us | share of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows[:16]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} % |")
    per_product = {}
    for r in rows:
        k = _kernel_base(r["Name"])
        for p in PHASE_KERNELS:
            if k.startswith(p):
                per_product[p] = per_product.get(p, 0.0) + float(r["TotalDurationNs"])
    calls = sum(int(r["Calls"]) for r in rows if _kernel_base(r["Name"]).startswith("k_gather"))
    lines += ["", f"Per product ({calls} products; phase kernels summed over their launches of one product):", ""]
    lines += [f"* `{p}`: {ns / calls / 1e3:.1f} us" for p, ns in per_product.items()]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_primary_mixed_bf16.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


BATCH_PROFILE_COMMAND = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_batch/trace "
                         "-o batched -- python3 bench.py --form batched --steps 10 --warmup 3")
BATCH_KERNELS = ("k_gatherN", "k_phaseA_q", "k_reduceT", "k_phaseB_q", "k_scatterN")
# HBM reads and L2 hits of the batched form's phase kernels (one counter group per run)
BATCH_COUNTER_COMMANDS = {
    "fetch": "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \"k_phaseA_q|k_phaseB_q\" --output-format csv "
             "-d gpurun_out/prof_batch/fetch -o batched -- python3 bench.py --form batched --steps 2 --warmup 1",
    "l2": "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --kernel-include-regex \"k_phaseA_q|k_phaseB_q\" "
          "--output-format csv -d gpurun_out/prof_batch/l2 -o batched -- python3 bench.py --form batched --steps 2 "
          "--warmup 1",
}


def summarize_batch_profile(prof_dir: str):
    """profiles/ kernel times of the batched form's merged product (64 planar
    faults, FP32, 16 columns): the last 10 merged products of BATCH_PROFILE_
    COMMAND (its 16-column timed loop), found in the kernel trace as the
    five-kernel sequence gather, phase A, reduction, phase B, scatter."""
    import csv

    rows = list(csv.DictReader(open(os.path.join(prof_dir, "trace", "batched_kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [_kernel_base(r["Kernel_Name"]) for r in rows]
    seqs = [rows[i:i + 5] for i in range(len(rows) - 4) if tuple(names[i:i + 5]) == BATCH_KERNELS]
    last = seqs[-10:]
    lines = ["# Kernel times: batched form, 64 planar faults (1,349,505 elements), FP32, 16 RHS", "",
             "Command (from the repository root, `TMPDIR=/tmp`):", "", "```", BATCH_PROFILE_COMMAND, "```", "",
             f"The last {len(last)} merged products of the run (its 16-column timed loop; one graph replay each), "
             "from the kernel trace:", "", "| kernel | workgroups | average us | min us | max us |",
             "|---|---|---|---|---|"]
    for j, k in enumerate(BATCH_KERNELS):
        d = [(int(q[j]["End_Timestamp"]) - int(q[j]["Start_Timestamp"])) / 1e3 for q in last]
        wg = int(last[-1][j]["Grid_Size_X"]) // int(last[-1][j]["Workgroup_Size_X"])
        lines.append(f"| `{k}` | {wg:,} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
    span = [(int(q[4]["End_Timestamp"]) - int(q[0]["Start_Timestamp"])) / 1e3 for q in last]
    lines += ["", f"Gather start to scatter end: {sum(span) / len(span):.1f} us on average."]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_batched_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if os.path.exists(os.path.join(prof_dir, "fetch")) and os.path.exists(os.path.join(prof_dir, "l2")):
        summarize_batch_counters(prof_dir)


def summarize_batch_counters(prof_dir: str):
    """profiles/traffic_batched_fp32.md: FETCH_SIZE (scaled by the copy
    calibration in profiles/traffic.json) and L2 hits of the merged
    product's phase kernels, the last dispatch of each (16 columns)."""
    import csv
    import glob

    def last(sub):
        f = glob.glob(os.path.join(prof_dir, sub, "*counter_collection.csv"))[0]
        out = {}
        for r in sorted(csv.DictReader(open(f)), key=lambda r: int(r.get("Dispatch_Id", 0) or 0)):
            out[(_kernel_base(r["Kernel_Name"]), r["Counter_Name"])] = float(r["Counter_Value"])
        return out

    scale = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["fetch_scale"]
    fe, l2 = last("fetch"), last("l2")
    lines = ["# HBM reads and L2 hits: batched form, 64 planar faults, FP32, 16 RHS", "",
             "Commands (one counter group per run, from the repository root, `TMPDIR=/tmp`):", "", "```",
             BATCH_COUNTER_COMMANDS["fetch"], BATCH_COUNTER_COMMANDS["l2"], "```", "",
             f"FETCH_SIZE scaled by {scale:.4f} (plain-copy calibration, `profiles/traffic.json`); the last "
             "dispatch of each kernel (the 16-column timed loop).", "",
             "| kernel | HBM bytes read | TCC_HIT | TCC_MISS | L2 hit rate |", "|---|---|---|---|---|"]
    for k in ("k_phaseA_q", "k_phaseB_q"):
        h, m = l2.get((k, "TCC_HIT_sum"), 0.0), l2.get((k, "TCC_MISS_sum"), 0.0)
        lines.append(f"| `{k}` | {fe.get((k, 'FETCH_SIZE'), 0.0) * 1024 * scale:,.0f} | {h:.4g} | {m:.4g} | "
                     f"{100 * h / max(1.0, h + m):.1f} % |")
    with open(os.path.join(ROOT, "profiles", "traffic_batched_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


NEWTON_PROFILE_COMMAND = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_newton/trace "
                          "-o newton -- python3 bench.py --form newton")


def summarize_newton_profile(prof_dir: str):
    """profiles/ summary of the kernels behind one implicit mechanical step
    (all four forms of bench.py --form newton, operator builds included)."""
    import csv

    rows = list(csv.DictReader(open(os.path.join(prof_dir, "trace", "newton_kernel_stats.csv"))))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# Kernel statistics: one implicit mechanical step, HF x fault (599,640 DOF), four forms", "",
             "Command (from the repository root, `TMPDIR=/tmp`):", "", "```", NEWTON_PROFILE_COMMAND, "```", "",
             "| kernel | calls | average us | total ms | share of GPU time |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {100 * float(r['TotalDurationNs']) / total:.1f} % |")
    lines += ["", f"All kernels: {total / 1e9:.2f} s of GPU time (builds of four operators included)."]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_newton_hf_fault.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_counters(prof_dir: str):
    """profiles/mfma_busy_primary_fp32.md and profiles/l2_hits_primary_fp32.md
    from the CSV output of COUNTER_COMMANDS (MFMA busy cycles and L2 hits of
    the phase kernels)."""
    import csv

    def load(sub):
        rows = list(csv.DictReader(open(os.path.join(prof_dir, sub, "primary_counter_collection.csv"))))
        agg, disp = {}, {}
        for r in rows:
            k = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hm::", "").strip()
            agg.setdefault(k, {}).setdefault(r["Counter_Name"], 0.0)
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp.setdefault(k, {})[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        return agg, {k: (len(v), sum(v.values())) for k, v in disp.items()}

    xcds, simds = 8, 1024   # MI355X: 8 XCDs, 256 CUs x 4 SIMDs
    agg, disp = load("mfma")
    lines = ["# MFMA activity of the product kernels: 256x256 planar fault, 16 RHS, FP32 form", "",
             "Command (from the repository root, `TMPDIR=/tmp`):", "", "```", COUNTER_COMMANDS["mfma"], "```", "",
             "MFMA utilisation as rocprofv3 defines it (`MfmaUtil`): SQ_VALU_MFMA_BUSY_CYCLES summed over the",
             f"SIMDs / (GRBM_GUI_ACTIVE of one XCD x {simds} SIMDs); the CSV's GRBM_GUI_ACTIVE is the sum over the",
             f"{xcds} XCDs, so one XCD's value is that sum / {xcds}.  Summed over every profiled dispatch.", "",
             "| kernel | dispatches | kernel time (us) | MFMA busy cycles | GRBM_GUI_ACTIVE (sum of XCDs) | MFMA util |",
             "|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items()):
        util = 100.0 * v["SQ_VALU_MFMA_BUSY_CYCLES"] / (v["GRBM_GUI_ACTIVE"] / xcds * simds)
        lines.append(f"| `{k}` | {disp[k][0]} | {disp[k][1] / 1e3:.0f} | {v['SQ_VALU_MFMA_BUSY_CYCLES']:.3e} | "
                     f"{v['GRBM_GUI_ACTIVE']:.3e} | {util:.1f} % |")
    lines += ["", "At 16 right-hand sides an FP32 panel entry meets 16 multiply-adds (8 flop per byte), so streaming",
              "at 5.3 TB/s needs about 42 TFLOP/s of FP32 MFMA, 27 % of its 157.3 TFLOP/s peak: the MFMA units",
              "are about a third busy, the kernels are bound by HBM, not by the matrix cores."]
    with open(os.path.join(ROOT, "profiles", "mfma_busy_primary_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    agg, disp = load("l2")
    lines = ["# L2 (TCC) hits of the product kernels: 256x256 planar fault, 16 RHS, FP32 form", "",
             "Command (from the repository root, `TMPDIR=/tmp`):", "", "```", COUNTER_COMMANDS["l2"], "```", "",
             "Summed over every profiled dispatch; a request is one 128-byte line.", "",
             "| kernel | dispatches | TCC_HIT | TCC_MISS | hit rate | miss bytes per dispatch |",
             "|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items()):
        h, m_ = v["TCC_HIT_sum"], v["TCC_MISS_sum"]
        lines.append(f"| `{k}` | {disp[k][0]} | {h:.3e} | {m_:.3e} | {100 * h / (h + m_):.1f} % | "
                     f"{128 * m_ / disp[k][0] / 1e6:.1f} MB |")
    lines += ["", "Phase B streams its panels once (misses) and re-reads X and T chunks from L2 (hits); phase A",
              "re-reads the X chunks of its source leaves across tasks (more hits)."]
    with open(os.path.join(ROOT, "profiles", "l2_hits_primary_fp32.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def interface_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2605_14397_amd", "csrc", "hm_interface.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def interface_traffic():
    """HBM bytes per interface-law launch from the committed counter summary,
    if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic_interface.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    return d.get("hbm_bytes_per_launch") if d.get("source_hash") == interface_source_hash() else None


def summarize_interface_profiles(prof_dir: str):
    """profiles/ summaries of the interface-law kernel from rocprofv3 CSVs
    (IF_PROFILE_COMMANDS run with prof_dir as gpurun_out/prof_if)."""
    import csv

    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        cal = json.load(fh)
    fs, ws = cal["fetch_scale"], cal["write_scale"]
    stats = list(csv.DictReader(open(os.path.join(prof_dir, "trace", "interface_kernel_stats.csv"))))
    k = [r for r in stats if "k_interface_update" in r["Name"]][0]

    def counter(sub, name):
        rows = list(csv.DictReader(open(os.path.join(prof_dir, sub, "interface_counter_collection.csv"))))
        v = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == name]
        return sum(v) / len(v), rows[0]

    fetch, row = counter("fetch", "FETCH_SIZE")
    write, _ = counter("write", "WRITE_SIZE")
    n = 199_880
    traffic = int(round((fetch * fs + write * ws) * 1024))
    alg = n * IF_BYTES_PER_ELEMENT
    d = {"source_hash": interface_source_hash(), "fetch_scale": fs, "write_scale": ws,
         "workload": "199,880 interface elements, every regime mixed (bench.py --form interface --if-states mixed)",
         "fetch_kib": round(fetch, 1), "write_kib": round(write, 1), "hbm_bytes_per_launch": traffic,
         "alg_bytes_per_launch": alg}
    with open(os.path.join(ROOT, "profiles", "traffic_interface.json"), "w") as fh:
        json.dump(d, fh, indent=1)
    lines = ["# Interface-law kernel: 199,880 elements, every regime mixed", "",
             "Commands (from the repository root, `TMPDIR=/tmp`):", "", "```"]
    lines += [IF_PROFILE_COMMANDS[c] for c in ("trace", "fetch", "write")]
    lines += ["```", "",
              f"`k_interface_update`: {k['Calls']} launches, average {float(k['AverageNs']) / 1e3:.1f} us "
              f"(min {float(k['MinNs']) / 1e3:.1f}, max {float(k['MaxNs']) / 1e3:.1f}); "
              f"scratch {row['Scratch_Size']} B per lane.", "",
              f"HBM counters per launch: FETCH_SIZE {fetch:.1f} KiB x {fs} + WRITE_SIZE {write:.1f} KiB x {ws} "
              f"(scales from the 2 GiB copy calibration in traffic.json) = {traffic / 1e6:.2f} MB, against "
              f"{alg / 1e6:.2f} MB algorithmic ({IF_BYTES_PER_ELEMENT} B per element: increment, traction, "
              "inelastic DD, internal variables, material index and eta/dt read; traction, inelastic DD, internal "
              f"variables, tangent, mode and D written): {traffic / alg:.3f}x.", ""]
    with open(os.path.join(ROOT, "profiles", "interface_update_hf_fault.md"), "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps(d))


def traffic_from_profile(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current apply source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the three-disk and 64-mesh sub-records")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", choices=["fp32", "fp64", "mixed"], default=None,
                    help="time one form only (profiling runs)")
    ap.add_argument("--form", choices=["primary", "batched", "precision", "learned", "interface", "newton", "precond",
                                       "coupled",
                                       "injection", "copy"],
                    default="primary",
                    help="batched: 64 independent faults in merged, graph-captured launches; "
                         "learned: trained preconditioner correction on the HF x fault tangent solves; "
                         "interface: interface-law update and consistent tangent of 199,880 elements; "
                         "newton: one implicit mechanical step (Newton) of the HF x fault under a pressure rise; "
                         "injection: adaptive implicit run of the HF x fault injection (paper's step controller); "
                         "copy: plain device copy of 2 GiB (calibrates HBM byte counters)")
    ap.add_argument("--meshes", type=int, default=64)
    ap.add_argument("--hf-h", type=float, default=None,
                    help="element leg of the HF x fault mesh (m); default 0.46 (199,880 triangles), "
                         "1.0 for the coupled form (42,400 triangles)")
    ap.add_argument("--train-epochs", type=int, default=8, help="learned form: passes over the 16 training states")
    ap.add_argument("--neighbors", type=int, default=16, help="learned form: neighbours per element")
    ap.add_argument("--train-extra-law", type=int, default=8,
                    help="learned form with --tangents newton: also train on this many states of the "
                         "prescribed-increment law path (steps 0-15, evenly spread), a second loading scenario")
    ap.add_argument("--tangents", choices=["newton", "law", "closed-form"], default="newton",
                    help="learned form: tangent states at the converged Newton steps of a rising-pressure "
                         "injection (newton), from the interface law driven along prescribed increments (law), "
                         "or the closed-form synthetic states")
    ap.add_argument("--if-states", choices=["both", "mixed", "elastic"], default="both",
                    help="interface form: which seeded state sets to time (profiling runs use one)")
    ap.add_argument("--summarize-profiles", default=None, metavar="DIR",
                    help="write the profiles/ summaries from rocprofv3 CSV output in DIR (no GPU)")
    args = ap.parse_args()
    if args.hf_h is None:
        args.hf_h = 1.0 if args.form == "coupled" else 0.46
    if args.summarize_profiles:
        d = args.summarize_profiles
        # every summary whose raw output is under d
        if os.path.exists(os.path.join(d, "mfma")) and os.path.exists(os.path.join(d, "l2")):
            summarize_counters(d)
        if os.path.exists(os.path.join(d, "trace", "mixed_kernel_stats.csv")):
            summarize_mixed_profile(d)
        if os.path.exists(os.path.join(d, "trace", "newton_kernel_stats.csv")):
            summarize_newton_profile(d)
        if os.path.exists(os.path.join(d, "trace", "batched_kernel_trace.csv")):
            summarize_batch_profile(d)
        if os.path.exists(os.path.join(d, "trace", "interface_kernel_stats.csv")):
            summarize_interface_profiles(d)
        if os.path.exists(os.path.join(d, "trace", "primary_kernel_stats.csv")) and os.path.exists(
                os.path.join(d, "fetch")):
            summarize_profiles(d)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the H-matrix path here is built and timed on a single MI355X "
              "(multi-GPU sharding is a design note only); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import penny_active_mask, rhs_columns, square_fault

    torch.cuda.set_device(0)
    if args.form == "batched":
        bench_batched(args)
        return
    if args.form == "precision":
        bench_precision(args)
        return
    if args.form == "learned":
        bench_learned(args)
        return
    if args.form == "interface":
        bench_interface(args)
        return
    if args.form == "newton":
        bench_newton(args)
        return
    if args.form == "injection":
        bench_injection(args)
        return
    if args.form == "precond":
        bench_precond(args)
        return
    if args.form == "coupled":
        bench_coupled(args)
        return
    if args.form == "copy":
        src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4,
                          "ms": round(ms, 4), "gbs_read_plus_write": round(2 * src.numel() * 4 / ms / 1e6, 1)}))
        return
    m = square_fault(256)
    n = m.ndof
    X = torch.as_tensor(rhs_columns(n, NRHS, 2001), device="cuda")
    Y = torch.empty_like(X)
    mesh = hm.Mesh.from_workload(m)

    def time_form(op, reference=False, steps=args.steps, warmup=args.warmup):
        for _ in range(warmup):
            op.apply(X, Y, reference=reference)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            op.apply(X, Y, reference=reference)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / steps
        # per-stage durations: HIP events recorded by the library on this stream
        st = {k: 0.0 for k in hm.Operator.STAGES}
        reps = max(5, steps // 5)
        for _ in range(reps):
            for k, v in op.apply_timed(X, Y, reference=reference).items():
                st[k] += v / reps
        return ms, wall, st

    out = {}
    forms = [("fp32", dict(near_prec=hm.HM_F32, far_prec=hm.HM_F32, keep_f64_reference=1))]
    if args.only in ("fp64",):
        forms = [("fp64", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64))]
    if args.only in ("mixed",):
        forms = [("mixed", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16))]
    res = {}
    for name, kw in forms:
        log(f"building {name} operator ...")
        t0 = time.perf_counter()
        op = hm.Operator(mesh, YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        st = op.stats()
        ms, wall, stages = time_form(op)
        log(f"{name}: {ms:.3f} ms/step, stages {stages}")
        res[name] = dict(op=op, stats=st, ms=ms, wall=wall, stages=stages, build_s=build_s, Y=Y.cpu().numpy())
        if name == "fp32" and args.only is None:
            ms64, wall64, st64 = time_form(op, reference=True)
            log(f"fp64 (reference copy): {ms64:.3f} ms/step, stages {st64}")
            res["fp64"] = dict(op=op, stats=st, ms=ms64, wall=wall64, stages=st64, build_s=None, ref=True,
                               Y=Y.cpu().numpy())

    head = res[forms[0][0]]
    st = head["stats"]
    ms = head["ms"]
    snear = {hm.HM_F64: 8, hm.HM_F32: 4, hm.HM_BF16: 2}[st["near_prec"]]
    sfar = {hm.HM_F64: 8, hm.HM_F32: 4, hm.HM_BF16: 2}[st["far_prec"]]
    sacc = 8 if st["near_prec"] == hm.HM_F64 else 4
    alg = product_bytes(st, n, snear, sfar, sacc)
    phaseB_ms = head["stages"]["phaseB"]
    achieved = alg["phaseB"] / (phaseB_ms * 1e-3) / 1e9
    value = NRHS * 1000.0 / ms
    product_gbs = alg["product"] / (ms * 1e-3) / 1e9
    out.update({
        "metric": "H-matvecs/s at 196,608 DOF (16-RHS batched H-matrix product)",
        "value": round(value, 2),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if forms[0][0] == "fp32" else ("f64" if forms[0][0] == "fp64" else "bf16/f32"),
        "data": "synthetic",
        "config": {
            "workload": "planar fault 256x256 square elements (65,536 elements, 196,608 DOF), 16 N(0,1) RHS; "
                        "H-matrix leaf 64, eta 2, ACA 1e-6; FP32 near and far field, FP32 accumulation",
            "n_dof": n, "nrhs": NRHS, "leaf_size": 64, "eta": 2.0, "aca_tol": 1e-6,
        },
        # whole product: stored entries without padding + FP64 vectors in and out
        "hbm_gbs": round(product_gbs, 1),
        "alg_bytes_per_step": alg["product"],
        "product_roofline_frac": round(product_gbs / HBM_PEAK_GBS, 4),
        "wall_s_timed": round(head["wall"], 4),
        "stage_ms": {k: round(v, 4) for k, v in head["stages"].items()},
        "roofline": {
            "kernel": "k_phaseB (dense pieces + U T; one workgroup per leaf section and 8-tile window; "
                      "all launches of one product)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile("k_phaseB"),
            "alg_bytes_per_launch": alg["phaseB"],
            "alg_bytes_formula": "stored dense entries x s_near + U entries (sum k c m) x s_far + X chunks "
                                 "(16 x 3N x s_near) + Y rows (16 x 3N x s_acc); no padding",
            "t_chunk_bytes_per_launch": alg["t_chunks"],
            "padding_bytes_per_launch": alg["phaseB_padding"],
            "launch_ms": round(phaseB_ms, 4),
        },
        "phaseA": {"ms": round(head["stages"]["phaseA"], 4), "alg_bytes": alg["phaseA"],
                   "gbs": round(alg["phaseA"] / (head["stages"]["phaseA"] * 1e-3) / 1e9, 1),
                   "frac": round(alg["phaseA"] / (head["stages"]["phaseA"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "formula": "V entries (sum k c n) x s_far + X chunks (16 x 3N x s_far); no padding"},
        "operator": {k: st[k] for k in ("n_dense_blocks", "n_lowrank_blocks", "dense_entries", "dense_entries_stored",
                                        "lowrank_entries",
                                        "lowrank_entries_u", "bytes_near", "bytes_far", "min_rank", "max_rank",
                                        "mean_rank", "apply_workspace_bytes")},
        "build_s": round(head["build_s"], 3) if head["build_s"] else None,
        "build_ms_split": {k: round(st[k], 1) for k in ("coef_ms", "aca_ms", "recompress_ms", "pack_ms")},
        # FP64 influence coefficients of the dense leaves (ALU-bound, not a roofline item)
        "coef_element_pairs_per_s": round(st["dense_entries"] / 9 / (st["coef_ms"] * 1e-3), 0)
        if st["coef_ms"] > 0 else None,
    })
    outputs = {forms[0][0]: head["Y"]}
    if "fp64" in res and forms[0][0] != "fp64":
        r64 = res["fp64"]
        a64 = product_bytes(st, n, 8, 8, 8, reference=True)
        out["fp64_form"] = {"value": round(NRHS * 1000.0 / r64["ms"], 2), "unit": "matvecs/s",
                            "ms_per_step": round(r64["ms"], 4),
                            "hbm_gbs": round(a64["product"] / (r64["ms"] * 1e-3) / 1e9, 1),
                            "product_roofline_frac": round(a64["product"] / (r64["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "stage_ms": {k: round(v, 4) for k, v in r64["stages"].items()}}
        outputs["fp64"] = r64["Y"]
    if args.only is None:
        # the precision form's operator: FP32 near field, BF16 far field, FP32 accumulation
        opm = hm.Operator(mesh, YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, near_prec=hm.HM_F32,
                          far_prec=hm.HM_BF16)
        stm = opm.stats()
        msm, _, stgm = time_form(opm)
        am = product_bytes(stm, n, 4, 2, 4)
        out["mixed_bf16_form"] = {
            "value": round(NRHS * 1000.0 / msm, 2), "unit": "matvecs/s", "ms_per_step": round(msm, 4),
            "hbm_gbs": round(am["product"] / (msm * 1e-3) / 1e9, 1),
            "product_roofline_frac": round(am["product"] / (msm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phaseA_frac": round(am["phaseA"] / (stgm["phaseA"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phaseB_frac": round(am["phaseB"] / (stgm["phaseB"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_far": stm["bytes_far"], "stage_ms": {k: round(v, 4) for k, v in stgm.items()}}
        outputs["mixed_bf16"] = Y.cpu().numpy()
        log(f"mixed (FP32 near / BF16 far): {msm:.3f} ms/step, stages {stgm}")
        del opm
        # the same with single BF16 in-vectors (no lo half)
        ops1 = hm.Operator(mesh, YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, near_prec=hm.HM_F32,
                           far_prec=hm.HM_BF16_1)
        sts1 = ops1.stats()
        mss1, _, stgs1 = time_form(ops1)
        as1 = product_bytes(sts1, n, 4, 2, 4)
        out["mixed_bf16_single_form"] = {
            "value": round(NRHS * 1000.0 / mss1, 2), "unit": "matvecs/s", "ms_per_step": round(mss1, 4),
            "hbm_gbs": round(as1["product"] / (mss1 * 1e-3) / 1e9, 1),
            "product_roofline_frac": round(as1["product"] / (mss1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phaseA_frac": round(as1["phaseA"] / (stgs1["phaseA"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phaseB_frac": round(as1["phaseB"] / (stgs1["phaseB"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_far": sts1["bytes_far"], "stage_ms": {k: round(v, 4) for k, v in stgs1.items()},
            "form": "FP32 near field, BF16 far factors, X and T rounded to one BF16 each (HM_BF16_1)"}
        outputs["mixed_bf16_single"] = Y.cpu().numpy()
        log(f"mixed (FP32 near / BF16 far, single in-vectors): {mss1:.3f} ms/step, stages {stgs1}")
        del ops1

    # ---------------------------------------------------------- GMRES time to 1e-8
    solutions = {}
    if not args.no_gmres and args.only is None:
        del res
        head = None
        torch.cuda.empty_cache()
        act = penny_active_mask(m)
        mask = torch.as_tensor(act, device="cuda")
        B = rhs_columns(n, NRHS, 2101) * 1e6
        B[0] = 0.0
        B[0, 2::3] = -1e6                        # uniform pressure on the crack
        B = B.reshape(NRHS, m.ne, 3) * act[None, :, None]
        Bt = torch.as_tensor(B.reshape(NRHS, n), device="cuda")
        g = {}
        for name, kw, runs in (
                ("fp64", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64),
                 (("fp64_plain", dict(precond=hm.HM_PC_BLOCK3)), ("fp64_leaf", dict(precond=hm.HM_PC_LEAF)),
                  ("fp64_ilu", dict(precond=hm.HM_PC_ILU)), ("fp64_jacobi", dict(precond=hm.HM_PC_JACOBI)))),
                ("mixed", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1),
                 (("mixed_bf16_refined", dict(refine=1, precond=hm.HM_PC_BLOCK3)),
                  ("mixed_bf16_refined_leaf", dict(refine=1, precond=hm.HM_PC_LEAF)))),
                ("fp32", dict(near_prec=hm.HM_F32, far_prec=hm.HM_F32, keep_f64_reference=1),
                 (("fp32_refined", dict(refine=1, precond=hm.HM_PC_BLOCK3)),))):
            op = hm.Operator(mesh, YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
            for rname, sol in runs:
                # a fresh tangent per run: the leaf preconditioner's set-up is inside the timed solve
                op.set_tangent(None, mask)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, rep = op.solve(Bt, rtol=1e-8, restart=100, max_iter=2000, raise_on_notconv=False, **sol)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                g[rname] = {"time_to_1e-8_s": round(dt, 3), "iterations": rep["iterations"],
                            "refinements": rep["refinements"], "rel_residual": rep["rel_residual"],
                            "converged": bool(rep["converged"]),
                            "precond_setup_ms": round(rep["precond_setup_ms"], 2)}
                if sol.get("precond") == hm.HM_PC_ILU:
                    g[rname].update(ilu_nnz=rep["precond_nnz"], ilu_colours=rep["precond_colors"])
                solutions[rname] = x.cpu().numpy()
                log(f"gmres {rname}: {g[rname]}")
            del op
            torch.cuda.empty_cache()
        g["speedup_mixed_vs_fp64"] = round(g["fp64_plain"]["time_to_1e-8_s"] / g["mixed_bf16_refined"]["time_to_1e-8_s"], 3)
        g["speedup_mixed_leaf_vs_fp64"] = round(g["fp64_plain"]["time_to_1e-8_s"]
                                                / g["mixed_bf16_refined_leaf"]["time_to_1e-8_s"], 3)
        g["system"] = ("A11 = E on a penny crack of radius 0.45 x side (41,000 active elements), identity "
                       "elsewhere; 16 RHS (uniform 1 MPa pressure + 15 seeded tractions); GMRES(100), "
                       "3x3 block-Jacobi (plain), leaf block-Jacobi (_leaf), ILU(0) of the 1 % largest near-field "
                       "entries (_ilu) or point Jacobi (_jacobi), set-up included, FP64 Arnoldi; "
                       "rel_residual with the FP64 H-operator")
        out["gmres"] = g

    # ---------------------------------------------------------- the other configurations
    extra = {}
    if not args.no_forms and args.only is None:
        torch.cuda.empty_cache()
        out["precision_form"], extra["precision"] = precision_record(steps=10)
        torch.cuda.empty_cache()
        out["batched_form"], extra["batched"] = batched_record(steps=10, warmup=3, n_meshes=args.meshes)
        torch.cuda.empty_cache()

    # ---------------------------------------------------------- CPU oracle leg
    # the oracle timed on this host's cores (cpu_baseline), and every result
    # above stated against it
    if not args.no_cpu_baseline and args.only is None:
        oracle_leg(args, out, m, X.cpu().numpy(), outputs, solutions, B if solutions else None, extra)
    print(json.dumps(out), flush=True)


def product_bytes(st, n, snear, sfar, sacc, reference=False):
    """Algorithmic bytes of one 16-column product from the operator's stored
    entries, without padding: the whole product (panels once, the FP64
    self blocks of mixed forms once, FP64 vectors in and out at the
    boundary), phase B (dense entries, U entries, X chunks in near
    precision, Y rows in accumulation precision), phase A (V entries, X
    chunks in far precision), the T chunks phase B reads, and the padding
    phase B's panels carry beyond that."""
    dense, lr, lr_u = st["dense_entries_stored"], st["lowrank_entries"], st["lowrank_entries_u"]
    selfb = 0 if reference else st["self_f64_entries"] * 8
    vec = NRHS * n
    d = {"product": dense * snear + lr * sfar + selfb + vec * 16,
         "phaseB": dense * snear + lr_u * sfar + vec * snear + vec * sacc,
         "phaseA": (lr - lr_u) * sfar + vec * sfar,
         "t_chunks": st["rank_sum"] * NRHS * sfar}
    if not reference:
        d["phaseB_padding"] = st["bytes_near"] + st["bytes_far_u"] - (dense * snear + lr_u * sfar)
    return d


def cpu_model() -> str:
    """lscpu's model name (with family/model numbers), else /proc/cpuinfo's."""
    import subprocess

    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in txt.splitlines() if ":" in l)}
        if "Model name" in f:
            return f"{f['Model name']} (family {f.get('CPU family', '?')}, model {f.get('Model', '?')}, " \
                   f"{f.get('Socket(s)', '?')} socket(s), {f.get('CPU(s)', '?')} CPUs listed)"
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_leg(args, out, m, Xh, outputs, solutions, B, extra):
    """The CPU oracle on this host: its exact-row product timed on a bounded
    sample (cpu_baseline), and the errors of every GPU result above against
    the oracle's exact operator (Toeplitz sum of the uniform grids by FFT,
    exact rows of the triangle meshes by Peach-Koehler quadrature)."""
    import numpy as np

    import oracle

    n = m.ndof
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    probe = rng.choice(m.ne, 64, replace=False)
    oracle.rows_matvec(m, YOUNG, NU, probe, Xh)
    tp = time.perf_counter() - t0
    nrows = int(min(m.ne, max(64, 64 * args.cpu_seconds / max(tp, 1e-3))))
    rows = rng.choice(m.ne, nrows, replace=False)
    t0 = time.perf_counter()
    oracle.rows_matvec(m, YOUNG, NU, rows, Xh)
    tc = time.perf_counter() - t0
    cpu_value = NRHS * (nrows / m.ne) / tc
    out["cpu_baseline"] = {"value": round(cpu_value, 6), "unit": "matvecs/s", "cores": threads, "kind": "oracle",
                           "cpu_model": cpu_model(),
                           "sample": f"exact FP64 rows (coplanar closed form, direct summation) for {nrows} of "
                                     f"{m.ne} elements x 16 RHS in {tc:.1f} s, scaled to whole products"}
    log(f"cpu oracle: {out['cpu_baseline']}")
    # 256 x 256 products of every form against the exact Toeplitz product
    nx = m.meta["nx"]
    table = oracle.grid_table(YOUNG, NU, nx, nx)
    ref = oracle.grid_matvec_fft(table, nx, nx, Xh)

    def errs(Y, R):
        col = [float(np.linalg.norm(Y[c] - R[c]) / np.linalg.norm(R[c])) for c in range(R.shape[0])]
        ent = [float(np.abs(Y[c] - R[c]).max() / np.abs(R[c]).max()) for c in range(R.shape[0])]
        return {"max_column_rel_err": max(col), "max_entry_rel_err": max(ent)}

    err = {k: errs(v, ref) for k, v in outputs.items()}
    for k, v in err.items():
        rec = out if k == "fp32" else out.get({"fp64": "fp64_form", "mixed_bf16": "mixed_bf16_form",
                                               "mixed_bf16_single": "mixed_bf16_single_form"}[k], {})
        rec["error_vs_oracle"] = v
    log(f"product errors vs exact operator: {err}")
    # GMRES solutions: exact residual b - A11 x with A11 = E on the crack, identity elsewhere
    if solutions:
        from workloads import penny_active_mask

        act3 = np.repeat(penny_active_mask(m).astype(bool), 3)
        for k, x in solutions.items():
            Ex = oracle.grid_matvec_fft(table, nx, nx, x)
            Bf = B.reshape(NRHS, n)
            r = np.where(act3[None, :], Bf - Ex, Bf - x)
            rel = max(float(np.linalg.norm(r[c]) / np.linalg.norm(Bf[c])) for c in range(NRHS))
            out["gmres"][k]["exact_rel_residual"] = rel
        log("gmres exact residuals: " + str({k: out["gmres"][k]["exact_rel_residual"] for k in solutions}))
    if "precision" in extra:
        d = extra["precision"]
        rows = d["rows"]
        t0 = time.perf_counter()
        R = oracle.rows_matvec(d["mesh"], YOUNG, NU, rows, np.concatenate([d["X"], d["x"]]), method=1)
        dof = (3 * rows[:, None] + np.arange(3)).ravel()
        rec = out["precision_form"]
        rec["product_error_vs_oracle_rows"] = {k: errs(Y[:, dof], R[:NRHS]) for k, Y in d["Y"].items()}
        bh = d["b"][0, dof]
        rec["precision_bf16"]["exact_rel_residual_rows"] = float(np.linalg.norm(bh - R[NRHS]) / np.linalg.norm(bh))
        rec["oracle_rows"] = f"{rows.size} rows (32 at the largest load, the rest seeded), PK quadrature, " \
                             f"{time.perf_counter() - t0:.1f} s"
        log(f"precision form vs oracle rows: {rec['product_error_vs_oracle_rows']}, "
            f"refined residual {rec['precision_bf16']['exact_rel_residual_rows']:.2e}")
    if "batched" in extra:
        d = extra["batched"]
        worst = 0.0
        for mesh, X1, Y1 in zip(d["meshes"], d["X"], d["Y"]):
            t = oracle.grid_table(YOUNG, NU, mesh.meta["nx"], mesh.meta["ny"])
            R1 = oracle.grid_matvec_fft(t, mesh.meta["nx"], mesh.meta["ny"], X1)
            worst = max(worst, errs(Y1, R1)["max_column_rel_err"])
        out["batched_form"]["error_vs_oracle"] = {"max_column_rel_err_all_meshes": worst,
                                                  "columns": int(d["X"][0].shape[0])}
        log(f"batched vs exact Toeplitz products: worst {worst:.2e}")


def precision_record(steps=10):
    """Three intersecting disk fractures (the precision form's workload):
    GMRES to 1e-8 in the plain FP64 form and in the precision form (FP32
    near, BF16 far, FP64 refinement), each with 3x3 and leaf block-Jacobi;
    products of 16 columns timed.  Returns (record, arrays for the oracle
    leg)."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import gaussian_pressure_traction, rhs_columns, three_disks

    m = three_disks()
    n = m.ndof
    log(f"precision form: {m.ne} triangles")
    bh = gaussian_pressure_traction(m)[None, :]
    b = torch.as_tensor(bh, device="cuda")
    Xh = rhs_columns(n, NRHS, 3101)
    X = torch.as_tensor(Xh, device="cuda")
    Y = torch.empty_like(X)
    rec = {"workload": f"three intersecting 40 m disk fractures, {m.ne} triangles, {n} DOF; leaf 64, eta 2, "
                       "ACA 1e-6; Gaussian pressure load 5 MPa, sigma 8 m; GMRES(100) to 1e-8 (FP64 residual "
                       "with the FP64 H-operator); set-up of the leaf preconditioner inside the timed solve"}
    keep = {"mesh": m, "X": Xh, "b": bh, "Y": {}}
    for name, kw, sol in (("fp64_plain", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64), dict()),
                          ("precision_bf16", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1),
                           dict(refine=1)),
                          ("precision_bf16_single", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16_1,
                                                         keep_f64_reference=1), dict(refine=1))):
        t0 = time.perf_counter()
        op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        st = op.stats()
        for _ in range(3):
            op.apply(X, Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            op.apply(X, Y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        keep["Y"][name] = Y.cpu().numpy()
        snear = 8 if kw["near_prec"] == hm.HM_F64 else 4
        sfar = {hm.HM_F64: 8, hm.HM_BF16: 2, hm.HM_BF16_1: 2}[kw["far_prec"]]
        alg = product_bytes(st, n, snear, sfar, snear)
        r = {"matvec16_ms": round(ms, 4), "matvecs_per_s": round(NRHS * 1000.0 / ms, 1),
             "hbm_gbs": round(alg["product"] / (ms * 1e-3) / 1e9, 1),
             "product_roofline_frac": round(alg["product"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "build_s": round(build_s, 2), "bytes_near": st["bytes_near"], "bytes_far": st["bytes_far"]}
        for pname, pc in (("block3", hm.HM_PC_BLOCK3), ("leaf", hm.HM_PC_LEAF), ("ilu", hm.HM_PC_ILU)):
            op.set_tangent(None, None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, rep = op.solve(b, rtol=1e-8, restart=100, max_iter=3000, raise_on_notconv=False, precond=pc, **sol)
            torch.cuda.synchronize()
            r[pname] = {"time_to_1e-8_s": round(time.perf_counter() - t0, 3), "iterations": rep["iterations"],
                        "refinements": rep["refinements"], "rel_residual": rep["rel_residual"],
                        "converged": bool(rep["converged"]), "precond_setup_ms": round(rep["precond_setup_ms"], 2)}
            if name == "precision_bf16" and pname == "leaf":
                keep["x"] = x.cpu().numpy()
        log(f"{name}: {r}")
        rec[name] = r
        del op
        torch.cuda.empty_cache()
    base = rec["fp64_plain"]["block3"]["time_to_1e-8_s"]
    rec["speedup_vs_fp64_plain"] = {f"{f}_{p}": round(base / rec[f][p]["time_to_1e-8_s"], 3)
                                    for f in ("fp64_plain", "precision_bf16", "precision_bf16_single")
                                    for p in ("block3", "leaf", "ilu")}
    rng = np.random.default_rng(3)
    big = np.argsort(-np.abs(bh[0, 2::3]))[:32]
    rows = np.unique(np.concatenate([big, rng.choice(m.ne, 40, replace=False)]))[:64]
    keep["rows"] = rows
    return rec, keep


def batched_record(steps=10, warmup=3, n_meshes=64):
    """The batched form's workload (64 planar faults, 2k-40k elements, FP32):
    one merged graph-captured product (autotuned) vs one product per mesh
    with each operator's default layout, 1 and 16 columns.  Returns
    (record, arrays for the oracle leg)."""
    import torch

    import paper_2605_14397_amd as hm
    from workloads import batched_faults, rhs_columns

    meshes = batched_faults(n_meshes=n_meshes, seed=4001)
    ne = sum(m.ne for m in meshes)
    log(f"batched: {len(meshes)} meshes, {ne} elements")
    t0 = time.perf_counter()
    ops = [hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6,
                       near_prec=hm.HM_F32, far_prec=hm.HM_F32) for m in meshes]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    stats = [op.stats() for op in ops]
    alg16 = sum(product_bytes(st, m.ndof, 4, 4, 4)["product"] for st, m in zip(stats, meshes))
    vecs = {}
    for nrhs in (1, 16):
        Xs = [torch.as_tensor(rhs_columns(m.ndof, nrhs, 4101 + 100 * k), device="cuda") for k, m in enumerate(meshes)]
        vecs[nrhs] = (Xs, [torch.empty_like(x) for x in Xs])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the separate products first, each operator with its own default layout
    # (the batch's autotuner then rewrites the operators' task lists)
    ms_single = {nrhs: timed(lambda: [op.apply(x, y) for op, x, y in zip(ops, *vecs[nrhs])]) for nrhs in (1, 16)}
    t0 = time.perf_counter()
    batch = hm.Batch(ops, use_graph=True, autotune=True)
    tune_s = time.perf_counter() - t0
    info = batch.info()
    res, keep = {}, {"meshes": meshes}
    for nrhs in (1, 16):
        Xs, Ys = vecs[nrhs]
        ms_b = timed(lambda: batch.apply(Xs, Ys))
        if nrhs == 16:
            keep["X"] = [x[:4].cpu().numpy() for x in Xs]
            keep["Y"] = [y[:4].cpu().numpy() for y in Ys]
        ms_s = ms_single[nrhs]
        r = {"batched_graph_ms": round(ms_b, 4), "per_mesh_ms": round(ms_s, 4), "speedup": round(ms_s / ms_b, 3),
             "batched_matvecs_per_s": round(nrhs * len(meshes) * 1000.0 / ms_b, 1)}
        if nrhs == 16:
            r["hbm_gbs"] = round(alg16 / (ms_b * 1e-3) / 1e9, 1)
            r["product_roofline_frac"] = round(alg16 / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        res[nrhs] = r
        log(f"batched nrhs {nrhs}: {r}")
    rec = {"workload": f"{len(meshes)} planar faults, {ne} square elements in total, 2k-40k each, aspect 1-4, "
                       "random orientations; leaf 64, eta 2, ACA 1e-6, FP32 form",
           "nrhs": {str(k): v for k, v in res.items()}, "build_s": round(build_s, 2), "autotune_s": round(tune_s, 2),
           "autotune": {"candidates": info["tune_candidates"], "ms": [round(x, 4) for x in info["tune_ms"]],
                        "chosen_leaves_per_task": info["leaves_per_task_a"],
                        "phase_b_window_candidates": info["tune_b_candidates"],
                        "phase_b_window_ms": [round(x, 4) for x in info["tune_b_ms"]],
                        "chosen_phase_b_window": info["phase_b_window"]},
           "alg_bytes_16": alg16}
    del batch, ops
    return rec, keep


def bench_precision(args):
    """The precision form on its own (bench.py --form precision): the
    three-disk record of the default run as its own JSON line."""
    rec, _ = precision_record(steps=args.steps)
    out = {"metric": "GMRES time to relative residual 1e-8, precision form vs plain FP64", "unit": "s",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "scaling": "weak", "vs_baseline": None,
           "value": rec["precision_bf16"]["leaf"]["time_to_1e-8_s"], "config": {"workload": rec["workload"]},
           "forms": rec}
    print(json.dumps(out), flush=True)


def law_tangent_states(hm, m, n_states=20):
    """D_k = C^ep + eta/dt of the interface law (hm_interface_update, in place
    on the GPU) after step k of the seeded injection path, k = 0..n_states-1."""
    import numpy as np
    import torch

    from workloads.interface import injection_path

    p = injection_path(m, n_states)
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    t, dp, chi, mid = cu(p["t"]), cu(p["dp"]), cu(p["chi"]), cu(p["mat_id"], torch.int32)
    Ds, modes = [], []
    for k in range(n_states):
        r = hm.interface_update(p["mats"], cu(p["dd"][k]), t, dp, chi, mat_id=mid, eta_dt=cu(p["eta_dt"][k]),
                                want_D=True, out=dict(t=t, dp=dp, chi=chi))
        Ds.append(r["D"])
        modes.append(np.bincount(r["mode"].cpu().numpy(), minlength=5).tolist())
    log(f"interface-law tangent states: modes elastic/shear/tensile/corner/open at steps 0, 15, 19: "
        f"{modes[0]}, {modes[15]}, {modes[-1]}")
    return Ds, modes


def newton_tangent_states(hm, m, op, n_states=20, max_cuts=3):
    """D_k = C^ep + eta/dt at the converged implicit step k of an injection
    whose pore pressure rises over n_states steps (injection_pressure):
    hm_newton_step (precision form with leaf block-Jacobi, FP64 residual to
    1e-8), then the state advances; k = 0..n_states-1.  A step whose Newton
    iteration does not converge is cut into two half steps (half the pressure
    increment, half the time step; adaptive time stepping, Sec. 3.4), at most
    max_cuts times in a row; the quasi-dynamic term's previous increment is
    rescaled to the new time step."""
    import numpy as np
    import torch

    from workloads.interface import injection_path, injection_pressure

    p = injection_path(m, n_states)
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    st = {"t": cu(p["t"]), "dp": cu(p["dp"]), "chi": cu(p["chi"]), "dd": None, "eta_dt": None}
    mid = cu(p["mat_id"], torch.int32)

    def advance(dpress, eta_dt, depth, acc):
        ratio = 1.0 if st["eta_dt"] is None else float(st["eta_dt"][0, 0] / eta_dt[0, 0])
        dd_prev = torch.zeros_like(st["t"]) if st["dd"] is None else st["dd"] * ratio
        dd, t_new, dp_new, chi_new, rep = op.newton_step(p["mats"], st["t"], st["dp"], st["chi"], dpress=dpress,
                                                         eta_dt=eta_dt, dd_prev=dd_prev, mat_id=mid, rtol=1e-8,
                                                         lin_rtol=1e-6, lin_precond=hm.HM_PC_LEAF, lin_refine=1,
                                                         raise_on_notconv=False)
        acc["newton"] += rep["iterations"]
        acc["gmres"] += sum(rep["gmres_iterations"])
        if not rep["converged"]:
            if depth >= max_cuts:
                raise RuntimeError(f"Newton step not converged after {max_cuts} cuts: {rep['residual']}")
            acc["cuts"] += 1
            for _ in range(2):
                rep = advance(0.5 * dpress, 2.0 * eta_dt, depth + 1, acc)
            return rep
        st["last"] = (st["t"], st["dp"], st["chi"], dd, eta_dt)   # start state and increment of this step
        st.update(t=t_new, dp=dp_new, chi=chi_new, dd=dd, eta_dt=eta_dt)
        return rep

    Ds, modes, steps = [], [], []
    for k in range(n_states):
        dpress = cu(injection_pressure(m, k, n_states) - injection_pressure(m, k - 1, n_states))
        acc = {"newton": 0, "gmres": 0, "cuts": 0}
        t0 = time.perf_counter()
        rep = advance(dpress, cu(p["eta_dt"][k]), 0, acc)
        # tangent at the converged end of the (last sub)step, evaluated from that step's start state
        t_s, dp_s, chi_s, dd_s, eta_s = st["last"]
        r = hm.interface_update(p["mats"], dd_s, t_s, dp_s, chi_s, mat_id=mid, eta_dt=eta_s, want_D=True)
        Ds.append(r["D"])
        modes.append(rep["modes"])
        steps.append({"s": round(time.perf_counter() - t0, 3), "newton": acc["newton"], "gmres": acc["gmres"],
                      "cuts": acc["cuts"]})
        log(f"injection step {k}: {steps[-1]}, modes {rep['modes']}")
    return Ds, modes, steps


def bench_learned(args):
    """Learned correction of the block preconditioner on the tangent solves
    of an injection sequence on the HF x fault mesh (20 tangent states,
    paper Sec. 3.1.1 / 3.3.1): by default D = C^ep + eta/dt at the
    converged implicit steps (hm_newton_step) of a rising-pressure
    injection; --tangents law: the interface law along prescribed
    increments; --tangents closed-form: the closed-form synthetic states.

    Training data: for states 0..15 (with the Newton sequence also 8 states
    of the prescribed-increment law path, a second loading scenario), 128
    FP64 GMRES solves each of A11 x = b with b = A11 x0 for seeded white x0
    (the method's own tangent solves; white solutions make the loss measure
    ||M^-1 A11 - I||).
    Training: Adam, 16 samples per step, 8 steps per state per epoch (one
    pass over the state's samples).
    Held-out states 16..19, 16 right-hand sides each (white tractions and
    Gaussian normal-pressure bumps), GMRES(50) to a relative FP64 residual
    of 1e-8 in four forms: FP64 operator with block-Jacobi (the plain
    baseline), FP64 with the learned correction, and the precision form
    (FP32 near / BF16 far, FP64 refinement) with either preconditioner."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import hf_fault_mesh, rhs_columns, tangent_rhs, tangent_state

    t0 = time.perf_counter()
    m = hf_fault_mesh(h=args.hf_h)
    n = m.ndof
    log(f"learned form: {m.ne} triangles ({time.perf_counter() - t0:.1f} s to mesh)")
    cuda = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    ops = {}
    for name, kw in (("fp64", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64)),
                     ("precision_bf16", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1))):
        t0 = time.perf_counter()
        ops[name] = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
        torch.cuda.synchronize()
        log(f"built {name} in {time.perf_counter() - t0:.1f} s")
    op = ops["fp64"]
    law_modes = None
    newton_log = None
    if args.tangents == "newton":
        Ds, law_modes, newton_log = newton_tangent_states(hm, m, ops["precision_bf16"])
        tangent = lambda k: Ds[k]
    elif args.tangents == "law":
        Ds, law_modes = law_tangent_states(hm, m)
        tangent = lambda k: Ds[k]
    else:
        tangent = lambda k: cuda(tangent_state(m, k))
    # training states: 0-15 of the sequence, plus (Newton sequence) some states of the
    # prescribed-increment path, a second loading scenario with open and yielded elements early on
    train_D = [tangent(k) for k in range(16)]
    if args.tangents == "newton" and args.train_extra_law > 0:
        Ds_law, _ = law_tangent_states(hm, m)
        for i in np.linspace(0, 15, args.train_extra_law).round().astype(int):
            train_D.append(Ds_law[int(i)])
        del Ds_law
    n_train = len(train_D)
    # training pairs from the method's own FP64 solves
    t0 = time.perf_counter()
    data = []
    solve_its = []
    per_state = 8 * NRHS
    for k in range(n_train):
        op.set_tangent(train_D[k])
        bs, xs = [], []
        for j in range(per_state // NRHS):
            x0 = cuda(rhs_columns(n, NRHS, 7000 + per_state * k + NRHS * j))
            b = op.apply(x0, tangent=True)
            x, rep = op.solve(b, rtol=1e-8, restart=50, max_iter=3000)
            solve_its.append(rep["iterations"])
            bs.append(b)
            xs.append(x)
        data.append((torch.cat(bs), torch.cat(xs)))
        log(f"training state {k}: {per_state} solves, {solve_its[-1]} iterations in the last batch")
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    def train(base):
        net = hm.Learned(hidden=64, neighbors=args.neighbors, seed=5)
        net.set_base(base)
        hist = []
        for ep in range(args.train_epochs):
            for k in range(n_train):
                op.set_tangent(train_D[k])
                b, x = data[k]
                hist.extend(net.train(op, b, x, steps=8, batch=16, lr=1e-3))
            log(f"epoch {ep} (base {base}): mean loss {np.mean(hist[-128:]):.4g}")
        torch.cuda.synchronize()
        return net, hist

    t0 = time.perf_counter()
    net, hist = train(hm.HM_PC_BLOCK3)
    train_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    net_leaf, hist_leaf = train(hm.HM_PC_LEAF)
    train_leaf_s = time.perf_counter() - t0
    steps = len(hist)
    forms = {f: {"time_s": 0.0, "iterations": [], "rel_residual": 0.0, "fallbacks": 0}
             for f in ("fp64_block_jacobi", "fp64_learned", "fp64_leaf_block", "fp64_learned_on_leaf",
                       "precision_block_jacobi", "precision_learned", "precision_leaf_block",
                       "precision_learned_on_leaf")}
    attach_s = 0.0
    for k in range(16, 20):
        D = tangent(k)
        rhs = cuda(tangent_rhs(m, NRHS, 9000 + k))
        for name, o in ops.items():
            o.set_tangent(D)
            sol = dict(refine=1) if name != "fp64" else {}
            tag = "fp64" if name == "fp64" else "precision"
            # the leaf preconditioner's set-up (after the tangent change) is inside its timed solve;
            # attaching a correction (its forward pass, and for the leaf base the leaf inverses)
            # is timed apart
            for pc, pname in ((hm.HM_PC_BLOCK3, "block_jacobi"), (hm.HM_PC_LEARNED, "learned"),
                              (hm.HM_PC_LEAF, "leaf_block"), (hm.HM_PC_LEARNED, "learned_on_leaf")):
                if pc == hm.HM_PC_LEARNED:
                    t0 = time.perf_counter()
                    (net if pname == "learned" else net_leaf).attach(o)
                    attach_s += time.perf_counter() - t0
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, rep = o.solve(rhs, rtol=1e-8, restart=50, max_iter=3000, precond=pc,
                                 raise_on_notconv=False, **sol)
                torch.cuda.synchronize()
                f = forms[f"{tag}_{pname}"]
                f["time_s"] += time.perf_counter() - t0
                f["iterations"].append(rep["iterations"])
                f["rel_residual"] = max(f["rel_residual"], rep["rel_residual"])
                f["fallbacks"] += int(rep["fallback"] != 0)
                f.setdefault("converged", True)
                f["converged"] = f["converged"] and bool(rep["converged"])
                log(f"state {k} {tag}_{pname}: {rep['iterations']} iterations, {rep['solve_ms']:.0f} ms, "
                    f"residual {rep['rel_residual']:.2e}, fallback {rep['fallback']}")
    for f in forms.values():
        f["time_s"] = round(f["time_s"], 3)
    base = forms["fp64_block_jacobi"]["time_s"]
    out = {"metric": "GMRES time to relative residual 1e-8 on held-out tangent states, learned/precision forms "
                     "vs plain FP64 block-Jacobi",
           "value": forms["precision_learned"]["time_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "scaling": "weak", "vs_baseline": None, "dtype": "f64 residual, f32/bf16 operator",
           "config": {"workload": f"HF x fault, {m.ne} triangles, {n} DOF; leaf 64, eta 2, ACA 1e-6; "
                                  "tangent states 16-19 of 20, 16 right-hand sides each; GMRES(50)",
                      "tangents": {"newton": "converged implicit steps (hm_newton_step) of a rising-pressure "
                                             "injection, D = C^ep + eta/dt at each",
                                   "law": "interface law along prescribed increments (hm_interface_update)",
                                   "closed-form": "closed-form synthetic states"}[args.tangents],
                      "network": f"32-64-64-9 MLP, {args.neighbors} neighbours", "training_states": n_train,
                      "training_samples": n_train * per_state, "adam_steps": steps},
           "forms": forms, "law_modes_elastic_shear_tensile_corner_open": law_modes,
           "injection_steps": newton_log,
           "speedup_vs_fp64_block_jacobi": {k: round(base / v["time_s"], 3) for k, v in forms.items()},
           "training": {"train_leaf_base_s": round(train_leaf_s, 2),
                        "loss_last_epoch_leaf_base": round(float(np.mean(hist_leaf[-128:])), 5),
                        "data_s": round(data_s, 2), "data_solves": n_train * per_state, "data_solve_iterations": {"min": min(solve_its), "mean": round(float(np.mean(solve_its)), 1), "max": max(solve_its)}, "train_s": round(train_s, 2),
                        "ms_per_step": round(1000 * train_s / max(1, steps), 2),
                        "loss_first_epoch": round(float(np.mean(hist[:128])), 5),
                        "loss_last_epoch": round(float(np.mean(hist[-128:])), 5),
                        "attach_s_total": round(attach_s, 3)}}
    print(json.dumps(out), flush=True)


IF_BYTES_PER_ELEMENT = 4 * 24 + 4 + 24 + 3 * 24 + 72 + 4 + 72


def bench_interface(args):
    """Interface elasto-plastic update with consistent tangent and D = C^ep +
    eta/dt for 199,880 elements (the HF x fault mesh's element count; the
    first 11,180 are intact joints of the hydraulic fracture, the rest a
    weakening fault).  Two seeded state sets: every regime mixed (a quarter
    each compressed and shear-loaded, near the cut-off, partly weakened, fully
    damaged) and all elastic (the memory path alone)."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads.interface import interface_materials, interface_states

    n, n_hf = 199_880, 11_180
    mats = interface_materials()
    mat_id = np.full(n, 2, np.int32)
    mat_id[:n_hf] = 0
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    eta = cu(np.full((n, 3), 2.0e8))
    res = {}
    names = ("mixed", "elastic") if args.if_states == "both" else (args.if_states,)
    for name in names:
        st = interface_states(n, 9201, mats, mat_id)
        if name == "elastic":
            st["dd"][:] = 0.0
            st["t"][:] = [0.0, 0.0, -20e6]
            st["dp"][:] = 0.0
            st["chi"][:] = 0.0
        dd, t, dp, chi, mid = cu(st["dd"]), cu(st["t"]), cu(st["dp"]), cu(st["chi"]), cu(st["mat_id"], torch.int32)
        out = hm.interface_update(mats, dd, t, dp, chi, mat_id=mid, eta_dt=eta, want_D=True)
        for _ in range(args.warmup):
            hm.interface_update(mats, dd, t, dp, chi, mat_id=mid, eta_dt=eta, want_D=True, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            hm.interface_update(mats, dd, t, dp, chi, mat_id=mid, eta_dt=eta, want_D=True, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        modes = np.bincount(out["mode"].cpu().numpy(), minlength=5)
        res[name] = {"ms": round(ms, 4), "elements_per_s": round(n / (ms * 1e-3), 1),
                     "hbm_gbs": round(n * IF_BYTES_PER_ELEMENT / (ms * 1e-3) / 1e9, 1),
                     "modes_elastic_shear_tensile_corner_open": modes.tolist()}
        log(f"interface {name}: {res[name]}")
    if "mixed" not in res:
        print(json.dumps({"interface_states": res}), flush=True)
        return
    ms = res["mixed"]["ms"]
    alg = n * IF_BYTES_PER_ELEMENT
    line = {
        "metric": "interface-law updates/s (return map + consistent tangent + D, one launch)",
        "value": res["mixed"]["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n} interface elements (HF x fault count): {n_hf} intact joints, "
                               f"{n - n_hf} weakening-fault elements; every regime mixed"},
        "roofline": {"kernel": "k_interface_update", "bound": "hbm",
                     "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(alg / (ms * 1e-3) / 1e9 / 8000.0, 4), "traffic": interface_traffic(),
                     "alg_bytes_per_launch": alg, "launch_ms": ms},
        "states": res,
    }
    if not args.no_cpu_baseline:
        from oracle import interface as ifo

        st = interface_states(n, 9201, mats, mat_id)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds and done < n:
            sl = slice(done, min(n, done + 2000))
            ifo.update(mats, st["mat_id"][sl], st["dd"][sl], st["t"][sl], st["dp"][sl], st["chi"][sl])
            done = sl.stop
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(done / el, 1), "unit": "elements/s", "cores": 1, "kind": "oracle",
                                "sample": f"first {done} of the {n} mixed-regime elements in {el:.1f} s"}
    print(json.dumps(line), flush=True)


def bench_newton(args):
    """One implicit step of the mechanical problem on the HF x fault mesh
    (199,880 triangles): the hydraulic fracture an intact joint, the fault a
    pre-existing one (friction 0.6), initial effective tractions as on the
    injection path, and a Gaussian pore-pressure rise (peak 8 MPa, sigma
    10 m) around the injection point; eta/dt of a 1 s step.  Newton to a
    residual of 1e-8 of the initial one, each linear solve to 1e-6 of the
    current residual (a constant forcing term) or with Eisenstat-Walker
    forcing (_ew), with FP64 GMRES (3x3 and leaf block-Jacobi) and with the
    precision form (FP32 near / BF16 far inner solves refined in FP64); the
    residual always uses the FP64 operator."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import hf_fault_mesh
    from workloads.interface import injection_path

    m = hf_fault_mesh(h=args.hf_h)
    p = injection_path(m, 1)
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x = m.vertex_means()
    r2 = ((x - np.array([20.0, 0.0, 0.0])) ** 2).sum(axis=1)
    dpress = 8e6 * np.exp(-r2 / (2 * 10.0 ** 2))
    G = YOUNG / (2 * (1 + NU))
    rho = 2700.0
    cs, cp = np.sqrt(G / rho), np.sqrt((YOUNG / (3 * (1 - 2 * NU)) + 4 * G / 3) / rho)
    eta_dt = np.tile(0.5 * np.array([G / cs, G / cs, G / cp]) / 1.0, (m.ne, 1))
    t, dp, chi, mid = cu(p["t"]), cu(p["dp"]), cu(p["chi"]), cu(p["mat_id"], torch.int32)
    res = {}
    for name, kw, lin in (
            ("fp64_block_jacobi", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64), dict(lin_precond=hm.HM_PC_BLOCK3)),
            ("fp64_leaf_block", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64), dict(lin_precond=hm.HM_PC_LEAF)),
            ("precision_leaf_block", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1),
             dict(lin_precond=hm.HM_PC_LEAF, lin_refine=1)),
            ("precision_leaf_block_ew", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1),
             dict(lin_precond=hm.HM_PC_LEAF, lin_refine=1, forcing=1))):
        op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dd, t_new, _, _, rep = op.newton_step(p["mats"], t, dp, chi, dpress=cu(dpress), eta_dt=cu(eta_dt),
                                              mat_id=mid, rtol=1e-8, lin_rtol=1e-6, lin_restart=50,
                                              raise_on_notconv=False, **lin)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[name] = {"time_s": round(wall, 3), "newton_iterations": rep["iterations"],
                     "gmres_iterations": rep["gmres_iterations"], "converged": rep["converged"],
                     "residual_history": [float(f"{h:.4e}") for h in rep["residual"]],
                     "modes_elastic_shear_tensile_corner_open": rep["modes"],
                     "max_opening_mm": round(float(dd[:, 2].max()) * 1e3, 4),
                     "max_slip_mm": round(float(dd[:, :2].norm(dim=1).max()) * 1e3, 4), "dd": dd.cpu().numpy()}
        log(f"newton {name}: {wall:.3f} s, {rep['iterations']} Newton iterations, GMRES {rep['gmres_iterations']}, "
            f"residuals {[f'{h:.2e}' for h in rep['residual']]}, modes {rep['modes']}")
        del op
    ref = res["fp64_block_jacobi"].pop("dd")
    for k in list(res)[1:]:
        d = res[k].pop("dd")
        res[k]["diff_vs_fp64_block_jacobi"] = float(f"{np.linalg.norm(d - ref) / np.linalg.norm(ref):.3e}")
    base = res["fp64_block_jacobi"]["time_s"]
    out = {"metric": "time of one implicit mechanical step (Newton to 1e-8 of the initial residual)",
           "value": res["precision_leaf_block_ew"]["time_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "scaling": "weak", "vs_baseline": None, "dtype": "f64 residual, f32/bf16 operator",
           "config": {"workload": f"HF x fault, {m.ne} triangles, {m.ndof} DOF; intact-joint fracture, "
                                  "pre-existing fault (friction 0.6); Gaussian pressure rise 8 MPa / 10 m; "
                                  "leaf 64, eta 2, ACA 1e-6; GMRES(50) to 1e-6 per Newton iteration"},
           "forms": res, "speedup_vs_fp64_block_jacobi": {k: round(base / v["time_s"], 3) for k, v in res.items()}}
    print(json.dumps(out), flush=True)


def bench_injection(args):
    """Adaptive implicit run of the HF x fault injection (199,880 triangles):
    pore pressure injection_pressure_time over 20 s, materials and initial
    tractions of the injection path, eta/dt of the current step.  Each step
    is one hm_newton_step (precision form, leaf block-Jacobi,
    Eisenstat-Walker forcing, FP64 residual to 1e-8 of the initial one); a
    step whose Newton iteration does not converge is rejected and retried
    with half the step; an accepted step's truncation-error estimate
    (hm_lte_estimate; the first step, without a previous rate, counts as on
    target) and Newton count set the next step (hm_timestep_next: eps 1e-2,
    6 target iterations, growth at most 1.2)."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import hf_fault_mesh
    from workloads.interface import injection_path, injection_pressure_time

    m = hf_fault_mesh(h=args.hf_h)
    p = injection_path(m, 1)
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    G = YOUNG / (2 * (1 + NU))
    rho = 2700.0
    cs, cp = np.sqrt(G / rho), np.sqrt((YOUNG / (3 * (1 - 2 * NU)) + 4 * G / 3) / rho)
    eta = 0.5 * np.array([G / cs, G / cs, G / cp])
    op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6,
                     near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1)
    torch.cuda.synchronize()
    t_end, t, dt = 20.0, 0.0, 1.0
    dt_prev, e_prev = 0.0, 0.0
    st, dp, chi, mid = cu(p["t"]), cu(p["dp"]), cu(p["chi"]), cu(p["mat_id"], torch.int32)
    total = torch.zeros_like(st)
    dd_prev = None
    steps, rejected, newton_its, gmres_its = [], 0, 0, 0
    t0 = time.perf_counter()
    while t < t_end - 1e-12 and len(steps) < 400:
        dt = min(dt, t_end - t)
        dpress = cu(injection_pressure_time(m, t + dt) - injection_pressure_time(m, t))
        prev = torch.zeros_like(st) if dd_prev is None else dd_prev * (dt / dt_prev)
        dd, t_new, dp_new, chi_new, rep = op.newton_step(p["mats"], st, dp, chi, dpress=dpress,
                                                         eta_dt=cu(np.tile(eta / dt, (m.ne, 1))), dd_prev=prev,
                                                         mat_id=mid, rtol=1e-8, lin_rtol=1e-6, forcing=1,
                                                         lin_precond=hm.HM_PC_LEAF, lin_refine=1,
                                                         raise_on_notconv=False)
        newton_its += rep["iterations"]
        gmres_its += sum(rep["gmres_iterations"])
        if not rep["converged"]:
            rejected += 1
            dt *= 0.5
            log(f"t {t:.4f}: step {dt * 2:.4g} s rejected ({rep['iterations']} Newton iterations)")
            continue
        total += dd
        # the first step has no previous rate to compare with: take it as on target
        e = 1e-2 if dd_prev is None else hm.lte_estimate(dd.reshape(-1), dt, dd_prev.reshape(-1), dt_prev,
                                                         total.reshape(-1))
        t += dt
        steps.append({"t": round(t, 5), "dt": round(dt, 5), "newton": rep["iterations"],
                      "gmres": sum(rep["gmres_iterations"]), "lte": float(f"{e:.3e}"), "modes": rep["modes"]})
        log(f"t {t:.4f}: dt {dt:.4g} s, {rep['iterations']} Newton, lte {e:.2e}, modes {rep['modes']}")
        st, dp, chi, dd_prev = t_new, dp_new, chi_new, dd
        dt_next = hm.timestep_next(dt, dt_prev, e, e_prev, max(1, rep["iterations"]), eps_tol=1e-2, n_target=6,
                                   growth_max=1.2, dt_min=1e-4)
        dt_prev, e_prev, dt = dt, e, dt_next
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"metric": "wall time of the adaptive implicit injection run (20 s of injection)",
           "value": round(wall, 2), "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 residual, f32/bf16 operator",
           "config": {"workload": f"HF x fault, {m.ne} triangles, {m.ndof} DOF; pore pressure rising to 8 MPa "
                                  "over 20 s (Gaussian, 6 -> 20 m); intact-joint fracture, pre-existing fault; "
                                  "precision form, leaf block-Jacobi, Eisenstat-Walker forcing; step controller "
                                  "eps 1e-2, 6 target Newton iterations, growth 1.2"},
           "accepted_steps": len(steps), "rejected_steps": rejected, "newton_iterations": newton_its,
           "gmres_iterations": gmres_its, "final_modes_elastic_shear_tensile_corner_open": steps[-1]["modes"],
           "max_opening_mm": round(float(total[:, 2].max()) * 1e3, 4),
           "max_slip_mm": round(float(total[:, :2].norm(dim=1).max()) * 1e3, 4), "steps": steps}
    print(json.dumps(out), flush=True)


def bench_precond(args):
    """The plain preconditioners of the A11 solves side by side on the HF x
    fault mesh (199,880 triangles at the default leg): point Jacobi (the
    paper's first choice), 3x3 block-Jacobi, leaf block-Jacobi and the
    paper's ILU(0) of C^ep plus the 1 % largest near-field entries (its
    second choice), in the FP64 form and the precision form, on the
    closed-form tangent states 16-19 of the injection sequence, 16
    right-hand sides each, GMRES(50) to 1e-8; set-up inside the timed solve."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    import workloads as W

    m = W.hf_fault_mesh(h=args.hf_h)
    log(f"preconditioners: HF x fault, {m.ne} triangles")
    pcs = (("jacobi", hm.HM_PC_JACOBI), ("block3", hm.HM_PC_BLOCK3), ("leaf", hm.HM_PC_LEAF), ("ilu", hm.HM_PC_ILU))
    forms = {}
    for fname, kw, sol in (("fp64", dict(near_prec=hm.HM_F64, far_prec=hm.HM_F64), dict()),
                           ("precision", dict(near_prec=hm.HM_F32, far_prec=hm.HM_BF16, keep_f64_reference=1),
                            dict(refine=1))):
        op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6, **kw)
        res = {p: {"time_s": 0.0, "iterations": [], "setup_ms": [], "converged": True} for p, _ in pcs}
        for k in range(16, 20):
            D = torch.as_tensor(W.tangent_state(m, k), device="cuda")
            b = torch.as_tensor(W.tangent_rhs(m, NRHS, 9000 + k), device="cuda")
            for pname, pc in pcs:
                op.set_tangent(D)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, rep = op.solve(b, precond=pc, restart=50, rtol=1e-8, max_iter=3000, raise_on_notconv=False,
                                  **sol)
                torch.cuda.synchronize()
                r = res[pname]
                r["time_s"] += time.perf_counter() - t0
                r["iterations"].append(rep["iterations"])
                r["setup_ms"].append(round(rep["precond_setup_ms"], 1))
                r["converged"] &= bool(rep["converged"])
                if pc == hm.HM_PC_ILU:
                    r["nnz"], r["colours"] = rep["precond_nnz"], rep["precond_colors"]
                log(f"{fname} state {k} {pname}: {rep['iterations']} its, {time.perf_counter() - t0:.3f} s")
        for r in res.values():
            r["time_s"] = round(r["time_s"], 3)
        forms[fname] = res
        del op
        torch.cuda.empty_cache()
    base = forms["fp64"]["jacobi"]["time_s"]
    out = {"metric": "A11 solve time to 1e-8 by preconditioner (4 tangent states x 16 RHS)", "unit": "s",
           "value": forms["precision"]["ilu"]["time_s"], "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "scaling": "weak", "vs_baseline": None,
           "config": {"workload": f"HF x fault, {m.ne} triangles, {m.ndof} DOF; leaf 64, eta 2, ACA 1e-6; "
                                  "closed-form tangent states 16-19; GMRES(50)"},
           "forms": forms,
           "speedup_vs_fp64_jacobi": {f"{f}_{p}": round(base / forms[f][p]["time_s"], 3)
                                      for f in forms for p, _ in pcs}}
    print(json.dumps(out), flush=True)


def bench_coupled(args):
    """Coupled hydro-mechanical steps on the HF x fault mesh (Sec. 3.3): fluid
    injected at the intersection (0.01 m^3/s into the hydraulic fracture and,
    the meshes being independent, as much into the fault next to it), P1
    flow with the cubic law from residual widths of 0.5 mm (fracture) and
    0.2 mm (fault), steps of 1 s, the interface law of the injection path's
    materials; Newton
    on (dd, dp) to 1e-6 of the first scaled residual, each Jacobian solve by
    FGMRES(30) with P_up to 1e-4, its A11 solves by GMRES(50) to 1e-3 with
    the paper's point Jacobi, 3x3 or leaf block-Jacobi or ILU(0) of the 1 %
    largest near-field entries; scales of Sec. 3.3.2 carried from step to
    step; the ILU variant also with the paper's second Schur complement (S~
    from the ILU approximation of A11, applied matrix-free, inverted by
    GMRES to 1e-2).  Reports Newton iterations per step, outer (Jacobian) and
    inner (A11) iterations per solve and the time per step, as in Tab. 1-2."""
    import numpy as np
    import torch

    import paper_2605_14397_amd as hm
    from workloads import hf_fault_mesh
    from workloads.interface import injection_path

    m = hf_fault_mesh(h=args.hf_h)
    p = injection_path(m, 1)
    cu = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    G = YOUNG / (2 * (1 + NU))
    rho, dt = 2700.0, 1.0
    cs, cp = np.sqrt(G / rho), np.sqrt((YOUNG / (3 * (1 - 2 * NU)) + 4 * G / 3) / rho)
    eta_dt = cu(np.tile(0.5 * np.array([G / cs, G / cs, G / cp]) / dt, (m.ne, 1)))
    (h0, nh), (f0, nf) = m.meta["parts"]
    w0 = np.full(m.ne, 2e-4)          # residual hydraulic widths: fault 0.2 mm, fracture 0.5 mm
    w0[h0:h0 + nh] = 5e-4
    inj = np.array([20.0, 0.0, 0.0])
    src = np.zeros(m.nv)
    for lo, n in ((h0, nh), (f0, nf)):
        nodes = np.unique(m.conn[lo:lo + n])
        src[nodes[np.argmin(np.sum((m.xyz[nodes] - inj) ** 2, axis=1))]] = 0.01   # m^3/s
    log(f"coupled: HF x fault {m.ne} triangles, {m.nv} nodes, injection {src.sum()} m^3/s, dt {dt} s")
    steps = max(1, min(args.steps, 12))
    res = {}
    for name, pc, schur in (("jacobi", hm.HM_PC_JACOBI, 0), ("block3", hm.HM_PC_BLOCK3, 0),
                            ("leaf", hm.HM_PC_LEAF, 0), ("ilu", hm.HM_PC_ILU, 0), ("ilu_schur_ilu", hm.HM_PC_ILU, 1)):
        op = hm.Operator(hm.Mesh.from_workload(m), YOUNG, NU, leaf_size=64, eta=2.0, aca_tol=1e-6)
        fl = hm.Flow(hm.Mesh.from_workload(m), 2.2e9, 1e-3, hm.HM_PERM_CUBIC)
        t, dp, chi, mid = cu(p["t"]), cu(p["dp"]), cu(p["chi"]), cu(p["mat_id"], torch.int32)
        p_n = torch.zeros(m.nv, dtype=torch.float64, device="cuda")
        dn = torch.zeros(m.ne, dtype=torch.float64, device="cuda")
        dd_prev = torch.zeros(m.ne, 3, dtype=torch.float64, device="cuda")
        Lx, Lr = [1e-4 / dt, 1e6 / dt], [1e6, float(src.sum() * dt)]
        rec = {"time_s": [], "newton": [], "outer_per_solve": [], "inner_per_a11_solve": [], "converged": True}
        for k in range(steps):
            scales = (1.0 / (Lx[0] * dt), 1.0 / (Lx[1] * dt), 1.0 / Lr[0], 1.0 / Lr[1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dd, dpn, t_new, dp_new, chi_new, rep = hm.coupled_step(
                op, fl, p["mats"], t, dp, chi, p_n, cu(w0), dt, eta_dt=eta_dt, dd_prev=dd_prev,
                p_o=torch.zeros_like(p_n), source=cu(src), dn_start=dn, mat_id=mid, scales=scales, rtol=1e-6,
                outer_rtol=1e-4, outer_restart=30, outer_max_iter=200, inner_precond=pc, inner_rtol=1e-3,
                inner_restart=50, inner_max_iter=1000, max_newton=20, schur=schur, schur_rtol=1e-2,
                schur_max_iter=30, raise_on_notconv=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rec["time_s"].append(round(wall, 3))
            rec["newton"].append(rep["iterations"])
            its = max(1, sum(rep["outer_iterations"]))
            rec["outer_per_solve"].append(round(its / max(1, rep["iterations"]), 2))
            rec["inner_per_a11_solve"].append(round(sum(rep["inner_iterations"]) / its, 2))
            rec["converged"] &= rep["converged"]
            rec.setdefault("schur_per_solve", []).append(round(sum(rep["schur_iterations"]) / its, 2))
            log(f"coupled {name} step {k}: {wall:.3f} s, Newton {rep['iterations']}, outer {rep['outer_iterations']}, "
                f"inner {rep['inner_iterations']}, schur {rep['schur_iterations']}, modes {rep['modes']}, "
                f"max dp {float(dpn.max()) / 1e6:.3f} MPa")
            # the next step starts from this one's end; scales follow Sec. 3.3.2
            rate_x = [float(dd.abs().max()) / dt, float(dpn.abs().max()) / dt]
            Lx = [hm.scale_update(Lx[i], max(rate_x[i], 1e-30)) for i in range(2)]
            Lr = [hm.scale_update(Lr[0], rep["residual_mech"][0] or Lr[0]),
                  hm.scale_update(Lr[1], rep["residual_flow"][0] or Lr[1])]
            t, dp, chi = t_new, dp_new, chi_new
            p_n = p_n + dpn
            dn = dn + dd[:, 2]
            dd_prev = dd
        rec["modes_last"] = rep["modes"]
        rec["total_s"] = round(sum(rec["time_s"]), 3)
        rec["max_pressure_MPa"] = round(float(p_n.max()) / 1e6, 4)
        rec["max_opening_mm"] = round(float(dn.max()) * 1e3, 4)
        res[name] = rec
        del op, fl
        torch.cuda.empty_cache()
    out = {"metric": "coupled hydro-mechanical step time (Newton on DD and pressure, P_up-preconditioned FGMRES)",
           "value": round(res["ilu"]["total_s"] / steps, 3), "unit": "s per step", "n_gpus": 1,
           "higher_is_better": False, "data": "synthetic", "scaling": "weak", "vs_baseline": None,
           "config": {"workload": f"HF x fault, {m.ne} triangles ({m.ndof} mechanical + {m.nv} pressure DOF); "
                                  f"injection 0.01 m^3/s into each part at the intersection, dt {dt} s, {steps} steps; "
                                  "residual widths 0.5 mm (fracture), 0.2 mm (fault); "
                                  "cubic law, M 2.2 GPa, mu 1 mPa s; FP64 operator, leaf 64, eta 2, ACA 1e-6"},
           "inner_preconditioners": res}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """The batched form on its own (bench.py --form batched)."""
    rec, _ = batched_record(steps=args.steps, warmup=args.warmup, n_meshes=args.meshes)
    r16 = rec["nrhs"]["16"]
    out = {"metric": "batched H-matvecs/s (64 meshes, one graph-captured merged launch set)",
           "value": r16["batched_matvecs_per_s"], "unit": "mesh-matvecs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r16["batched_graph_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": rec["workload"]}, "batched": rec}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
