"""Benchmark: self-gravity field cells/s of the log-polar FFT path on the
1024 x 2048 two-fluid disc (gas h = 0.05, dust h = 0.005, all four ordered
pairs fused), one MI355X.

A step is one sg_field_fft call (phi transform of Sigma, fused u transform /
spectral multiply / inverse u transform, inverse phi transform) on inputs
resident in HBM; the kernel spectra are built once beforehand (the paper
precomputes the kernel once per simulation).  Every timed step starts with
cold caches: a 512 MiB buffer is rewritten before it, outside its events
(the disc's 118 MB would otherwise stay in the 256 MB Infinity Cache
between steps); back-to-back (warm) numbers are reported beside it.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
  python bench.py --copy-calibration   (plain 1 GiB device copy, for scaling
                                        rocprofv3 FETCH_SIZE / WRITE_SIZE)
  python bench.py --semispectral       (only the semi-spectral App. D measurement,
                                        one JSON line; for its kernel trace)
  python bench.py --direct             (only the direct sums: FP64 64x128 and FP32
                                        256x512, one JSON line; for their VALU counters)
  python bench.py --batch              (only the 64-disc batch: warm-up runs, then cold
                                        runs after a cache flush; for its traffic counters)
  python bench.py --oracle-rates       (CPU only: the oracle's cells/s on the other
                                        workloads, full fields or seeded samples)
  python bench.py --summarize-rocprof DIR
        (CPU only) turns the rocprofv3 CSV output of PROFILE_COMMANDS, run
        with DIR as their output root, into the text summaries in profiles/
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SG field cells/s at 1024×2048 bi-fluid; %HBM roofline; rel err vs FP64"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_passes_bifluid_1024x2048.json")
# pass 2 of the two-fluid 1024 x 2048 disc, any tuned variant (radix order,
# tile shape); the summaries use the variant launched most often, which is
# the one the tuned plan runs
DOMINANT_PREFIX = "k_pass2<2048, 2,"

# The rocprofv3 runs behind profiles/ (run from /tmp with TMPDIR=/tmp; {out}
# is the output root, {repo} the repository).  Counter runs are separate
# (one TCC counter group each) and never combined with tracing; they run the
# untuned plan so that both see the same pass-2 variant (all variants move
# the same bytes).
PROFILE_COMMANDS = {
    "kt": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/kt -o run -- "
          "python3 {repo}/bench.py --steps 50 --warmup 10 --no-cpu --no-extra",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/fetch -o run -- "
             "python3 {repo}/bench.py --steps 5 --warmup 2 --no-cpu --no-extra --no-tune",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/write -o run -- "
             "python3 {repo}/bench.py --steps 5 --warmup 2 --no-cpu --no-extra --no-tune",
    "cfetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/cfetch -o run -- "
              "python3 {repo}/bench.py --copy-calibration",
    "cwrite": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/cwrite -o run -- "
              "python3 {repo}/bench.py --copy-calibration",
    "p2_sq": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_LDS SQ_ACTIVE_INST_LDS "
             "SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv "
             "-d {out}/p2_sq -o run -- python3 {repo}/bench.py --steps 5 --warmup 2 --no-cpu --no-extra "
             "--no-tune",
    "b_kt": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/b_kt -o run -- "
            "python3 {repo}/bench.py --batch --steps 20 --warmup 5",
    "b_sq": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_LDS SQ_ACTIVE_INST_LDS "
            "SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv "
            "-d {out}/b_sq -o run -- python3 {repo}/bench.py --batch --steps 5 --warmup 2 --no-tune",
    "b_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/b_fetch -o run -- "
               "python3 {repo}/bench.py --batch --steps 5 --warmup 2 --no-tune",
    "b_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/b_write -o run -- "
               "python3 {repo}/bench.py --batch --steps 5 --warmup 2 --no-tune",
    "ss_kt": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/ss_kt -o run -- "
             "python3 {repo}/bench.py --semispectral",
    "ss_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}/ss_fetch -o run -- "
                "python3 {repo}/bench.py --semispectral",
    "ss_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}/ss_write -o run -- "
                "python3 {repo}/bench.py --semispectral",
    "dir_kt": "rocprofv3 --kernel-trace --stats --output-format csv -d {out}/dir_kt -o run -- "
              "python3 {repo}/bench.py --direct",
    "dir_valu": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 "
                "SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 "
                "--output-format csv -d {out}/dir_valu -o run -- python3 {repo}/bench.py --direct",
}
# VALU issue: one wave64 instruction per SIMD every 4 cycles (16 lanes),
# 256 CUs x 4 SIMDs at 2.4 GHz; FP32 (packed instructions disabled in the
# library's compile flags) and FP64 both issue at that rate: 78.6 TFLOP/s with FMA
VALU_SIMDS, VALU_CLOCK_HZ, VALU_PEAK_TFLOPS = 1024, 2.4e9, 78.6
COPY_BYTES = 4 << 28   # --copy-calibration copies 2^28 floats
FLUSH_FLOATS = 1 << 27  # 512 MiB rewritten before a cold step (Infinity Cache: 256 MB)


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_10812_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def pass_bytes(nr, nphi, nf):
    """Algorithmic (compulsory) bytes of each pass of one sg_field_fft call."""
    ncol = nphi // 2 + 1
    sig = 4 * nf * nr * nphi                 # Sigma read (float)
    st = 8 * nf * nr * ncol                  # Sigma~ (complex64 half spectra)
    spec = 8 * nf * nf * 2 * (nr + 1) * ncol  # kernel spectra, all pairs, both comps
    gh = 8 * 2 * nf * nr * ncol              # g^ (complex64 half spectra)
    g = 4 * 2 * nf * nr * nphi               # g_r, g_phi write (float)
    return {"pass1": sig + st, "pass2": st + spec + gh, "pass3": gh + g,
            "path": sig + spec + g}


def pass2_kernel_name(nr, nf, tuned):
    """Kernel name of the pass-2 variant the (tuned) plan runs for this disc."""
    nu = 2 * nr
    sf, gm = False, 1
    for r in tuned:
        if r["pass"] == 2 and r["length"] == nu and r["n_fluids"] == nf:
            g_default = max(1, 256 // (nf * max(1, nu // 8)))
            sf, gm = bool(r["small_radix_first"]), r["groups_per_wg"] // g_default
    return f"k_pass2<{nu}, {nf}, {'true' if sf else 'false'}, {gm}>"


def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"bench.py: no *{suffix} under {d}")
    with open(files[0], newline="") as fh:
        return list(csv.DictReader(fh))


def _counter_mean(d, kernel, counter):
    """Mean per-dispatch value (KiB) of one counter over the dispatches of a kernel
    (the most frequent kernel whose name starts with `kernel`)."""
    rows = [r for r in _csv_rows(d, "_counter_collection.csv")
            if r["Kernel_Name"].replace("void ", "").startswith(kernel) and r["Counter_Name"] == counter]
    if not rows:
        raise SystemExit(f"bench.py: no {counter} rows for {kernel} under {d}")
    names = {}
    for r in rows:
        names[r["Kernel_Name"]] = names.get(r["Kernel_Name"], 0) + 1
    top = max(names, key=names.get)
    vals = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == top]
    return sum(vals) / len(vals), len(vals), top.split("(")[0].replace("void ", "")


def _last_json(path):
    """The last JSON line a bench.py run printed, or None."""
    try:
        with open(path) as fh:
            rows = [x for x in fh.read().splitlines() if x.startswith("{")]
        return json.loads(rows[-1]) if rows else None
    except (OSError, ValueError):
        return None


def _kname(r):
    return r["Kernel_Name"].split("(")[0].replace("void ", "")


def _cold_dispatch_us(d, prefix, before):
    """Mean duration (us) of the dispatches of kernels named `prefix...` whose
    preceding dispatches (in start order) match the name prefixes `before`
    (nearest first): e.g. pass 2 right after pass 1 right after the cache
    flush, i.e. the pass 2 of a cold step."""
    rows = _csv_rows(d, "_kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [_kname(r) for r in rows]
    dur = []
    for i, n in enumerate(names):
        if not n.startswith(prefix) or i < len(before):
            continue
        if all(before[k] in names[i - 1 - k] for k in range(len(before))):
            dur.append((int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"])) / 1e3)
    return (sum(dur) / len(dur) if dur else None), len(dur)


def _counter_sums(d, prefix):
    """{counter: [per-dispatch values]} over the dispatches of kernels named
    `prefix...` (values summed over the counter's dimensions by rocprofv3)."""
    out = {}
    for r in _csv_rows(d, "_counter_collection.csv"):
        if _kname(r).startswith(prefix):
            out.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def summarize_rocprof(out):
    """Writes the summaries in profiles/ from the rocprofv3 output of
    PROFILE_COMMANDS under `out` (plus each command's stdout in <key>.out)."""
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    cmd = {k: v.format(out="<out>", repo="<repo>") for k, v in PROFILE_COMMANDS.items()}
    stats = _csv_rows(os.path.join(out, "kt"), "_kernel_stats.csv")
    lines = ["# Kernel time, two-fluid 1024x2048 FFT path (bench.py workload)", "",
             "Command (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output "
             "root):", "", "    " + cmd["kt"], "",
             "The run tunes the plan, times warm steps (launched back to back), cold steps "
             "(each after a 512 MiB cache flush, the headline) and cold steps pass by pass "
             "(sg_field_fft_profile with reps = 1 after a flush), then warm passes back to back. "
             "All dispatches of a kernel are averaged in the table.", "",
             "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share (%) |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    live = _last_json(os.path.join(out, "kt.out"))
    if live and "roofline" in live:
        rl = live["roofline"]
        cold_us, ncold = _cold_dispatch_us(os.path.join(out, "kt"), rl["kernel_name"],
                                           ["k_pass1", "FillFunctor"])
        if cold_us:
            us = rl["kernel_ms"] * 1e3
            lines += ["", f"Cold pass 2: the {ncold} dispatches of `{rl['kernel_name']}` that follow "
                          f"pass 1 right after the cache flush (the cold steps, and the cold steps "
                          f"timed pass by pass) average {cold_us:.2f} us in the trace; bench.py's own HIP-event "
                          f"timing of the cold pass in the same, profiled run (the roofline's kernel time) is "
                          f"{us:.2f} us ({abs(us - cold_us) / cold_us * 100:.1f} % apart; the profiler "
                          f"delays the events around each launch)."]
            plain = _last_json(os.path.join(os.path.dirname(os.path.abspath(out)), "bench.json"))
            if plain and "roofline" in plain and plain["roofline"].get("kernel_name") == rl["kernel_name"]:
                pu = plain["roofline"]["kernel_ms"] * 1e3
                lines[-1] += (f"  The plain `python3 bench.py` run of the same session (no profiler) "
                              f"timed it at {pu:.2f} us ({abs(pu - cold_us) / cold_us * 100:.1f} % from "
                              f"the trace).")
    with open(os.path.join(prof, "kernels_bifluid_1024x2048.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    cf, _, _ = _counter_mean(os.path.join(out, "cfetch"), "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    cw, _, _ = _counter_mean(os.path.join(out, "cwrite"), "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    pb = pass_bytes(1024, 2048, 2)
    per_pass = {}
    for key, prefix in (("pass1", "k_pass1<"), ("pass2", DOMINANT_PREFIX), ("pass3", "k_pass3<")):
        fk, nf_, kname = _counter_mean(os.path.join(out, "fetch"), prefix, "FETCH_SIZE")
        wk, nw_, kname_w = _counter_mean(os.path.join(out, "write"), prefix, "WRITE_SIZE")
        if kname_w != kname:
            raise SystemExit(f"bench.py: FETCH and WRITE runs ran different variants ({kname}, {kname_w})")
        per_pass[key] = (fk, wk, nf_, nw_, kname, fk * 1024.0 * f_scale, wk * 1024.0 * w_scale)
    fk, wk, nf_, nw_, kname, read_b, write_b = per_pass["pass2"]
    alg = pb["pass2"]
    tr = {"kernel": "pass2", "kernel_name": kname,
          "kernel_source_hash": kernel_source_hash(),
          "fetch_size_kib": round(fk, 1), "write_size_kib": round(wk, 1),
          "dispatches": [nf_, nw_],
          "copy_fetch_kib_per_gib": round(cf, 1), "copy_write_kib_per_gib": round(cw, 1),
          "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
          "bytes_read": round(read_b), "bytes_written": round(write_b),
          "bytes_per_launch": round(read_b + write_b), "algorithmic_bytes": alg,
          "passes": {k: {"kernel_name": v[4], "bytes_read": round(v[5]), "bytes_written": round(v[6]),
                         "algorithmic_bytes": pb[k]} for k, v in per_pass.items()},
          "commands": [cmd["fetch"], cmd["write"], cmd["cfetch"], cmd["cwrite"]]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(tr, fh, indent=1)
        fh.write("\n")
    md = ["# HBM traffic of the three passes, two-fluid 1024x2048 (bench.py workload)", "",
          "Commands (from /tmp, TMPDIR=/tmp):", ""] + \
         ["    " + cmd[k] for k in ("fetch", "write", "cfetch", "cwrite")] + \
         ["", f"Copy calibration (1 GiB device copy): FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE "
              f"{cw:.1f} KiB per launch, so FETCH_SIZE is scaled by {f_scale:.4f} and "
              f"WRITE_SIZE by {w_scale:.4f}.  Counters count L2 traffic to and from the fabric "
              f"(Infinity Cache hits included), so they do not depend on the cache's state.", "",
          "| Pass | Kernel | Dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | Read (MB) | "
          "Written (MB) | Total / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    for k, v in per_pass.items():
        md.append(f"| {k[-1]} | `{v[4]}` | {v[2]} / {v[3]} | {v[0]:.1f} | {v[1]:.1f} | "
                  f"{v[5] / 1e6:.2f} | {v[6] / 1e6:.2f} | {(v[5] + v[6]) / 1e6:.2f} / "
                  f"{pb[k] / 1e6:.2f} MB = {(v[5] + v[6]) / pb[k]:.3f}x |")
    md += ["", f"Kernel sources hash: {tr['kernel_source_hash']}."]
    with open(os.path.join(prof, "traffic_passes_bifluid_1024x2048.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    stale = os.path.join(prof, "traffic_pass2_bifluid_1024x2048.md")
    if os.path.exists(stale):
        os.remove(stale)

    if os.path.isdir(os.path.join(out, "p2_sq")):
        summarize_pass2_sq(out, prof, cmd)
    if os.path.isdir(os.path.join(out, "b_fetch")) and os.path.isdir(os.path.join(out, "b_write")):
        summarize_batch_traffic(out, prof, cmd, f_scale, w_scale, cf, cw)
    if os.path.isdir(os.path.join(out, "b_sq")):
        summarize_batch_sq(out, prof, cmd)
    ss_dir = os.path.join(out, "ss_kt")
    if os.path.isdir(ss_dir):
        stats = _csv_rows(ss_dir, "_kernel_stats.csv")
        lines = ["# Kernel time, semi-spectral path, App. D flaring gas disc 1200x2048", "",
                 "Command (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output "
                 "root):", "", "    " + cmd["ss_kt"], "",
                 "The run builds the radial operators twice (k_ss_rows, k_ss_scatter, self cells), "
                 "tunes the batch, then times solves (k_pass1, k_ss_pass, k_pass3) and per-pass "
                 "launches.", "",
                 "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share (%) |",
                 "|---|---|---|---|---|---|"]
        for r in stats:
            name = r["Name"].split("(")[0].replace("void ", "")
            lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                         f"{float(r['Percentage']):.2f} |")
        with open(os.path.join(prof, "kernels_semispectral_flaring_1200x2048.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    if os.path.isdir(os.path.join(out, "ss_fetch")) and os.path.isdir(os.path.join(out, "ss_write")):
        summarize_ss_traffic(out, prof, cmd, f_scale, w_scale)
    if os.path.isdir(os.path.join(out, "dir_kt")) and os.path.isdir(os.path.join(out, "dir_valu")):
        summarize_direct(out, prof, cmd)
    print(json.dumps(tr))


def summarize_pass2_sq(out, prof, cmd):
    """profiles/sq_pass2_bifluid_1024x2048.md: VALU, LDS and occupancy counters
    of pass 2 (per dispatch; rocprofv3's derived-metric formulas applied to
    the raw counters)."""
    v = _counter_sums(os.path.join(out, "p2_sq"), DOMINANT_PREFIX)
    if not v:
        return
    m = {k: sum(x) / len(x) for k, x in v.items()}
    n = len(v.get("SQ_WAVES", []))
    cu, xcc = 256, 8
    gui = m["GRBM_GUI_ACTIVE"] / xcc  # summed over the 8 XCDs by rocprofv3; per XCD
    waves = m["SQ_WAVES"]
    rows = [("waves per dispatch", f"{waves:.0f}"),
            ("VALU instructions per wave", f"{m['SQ_INSTS_VALU'] / waves:.0f}"),
            ("LDS instructions per wave", f"{m['SQ_INSTS_LDS'] / waves:.0f}"),
            ("GPU-active cycles (GRBM_GUI_ACTIVE per XCD)", f"{gui:.0f}"),
            ("VALUBusy = 100 SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE",
             f"{100 * m['SQ_ACTIVE_INST_VALU'] / cu / gui:.1f} %"),
            ("VALU issue = 4 SQ_INSTS_VALU / (4 SIMDs x CU_NUM x GRBM_GUI_ACTIVE)",
             f"{100 * 4 * m['SQ_INSTS_VALU'] / (4 * cu * gui):.1f} %"),
            ("LDS active = 100 SQ_ACTIVE_INST_LDS / CU_NUM / GRBM_GUI_ACTIVE",
             f"{100 * m['SQ_ACTIVE_INST_LDS'] / cu / gui:.1f} %"),
            ("LDSBankConflict = 100 SQ_LDS_BANK_CONFLICT / GRBM_GUI_ACTIVE / CU_NUM",
             f"{100 * m['SQ_LDS_BANK_CONFLICT'] / gui / cu:.2f} %"),
            ("OccupancyPercent = 400 SQ_WAVE_CYCLES / GRBM_GUI_ACTIVE / CU_NUM / 32",
             f"{400 * m['SQ_WAVE_CYCLES'] / gui / cu / 32:.1f} % (of 32 waves per CU)"),
            ("SQ_BUSY_CYCLES / (GRBM_GUI_ACTIVE x 4 SEs x 8 XCDs)",
             f"{m['SQ_BUSY_CYCLES'] / (gui * 4 * xcc):.2f}")]
    kname = [k for k in v][0]
    lines = ["# Pass 2 execution counters, two-fluid 1024x2048 (bench.py workload)", "",
             "Command (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output root):", "",
             "    " + cmd["p2_sq"], "",
             f"Means over {n} dispatches of the pass-2 kernel (untuned plan).  rocprofv3 sums each "
             "counter over its dimensions; GRBM_GUI_ACTIVE is divided by the 8 XCDs to give the "
             "cycles of one XCD (the formulas take its maximum).  Raw means:", ""]
    lines += [f"    {k} = {m[k]:.6g}" for k in sorted(m)]
    lines += ["", "| Quantity | Value |", "|---|---|"] + [f"| {a} | {b} |" for a, b in rows]
    with open(os.path.join(prof, "sq_pass2_bifluid_1024x2048.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_batch_traffic(out, prof, cmd, f_scale, w_scale, cf, cw):
    """profiles/traffic_batch64.md: HBM bytes of one 64-disc batch run (all
    pass kernels of the graph) against the algorithmic bytes."""
    fetch = _counter_sums(os.path.join(out, "b_fetch"), "k_pass")
    write = _counter_sums(os.path.join(out, "b_write"), "k_pass")
    meta = _last_json(os.path.join(out, "b_fetch.out"))
    if not fetch or not write or not meta:
        return
    runs = meta["graph_runs"]
    rd = sum(fetch["FETCH_SIZE"]) * 1024.0 * f_scale / runs
    wr = sum(write["WRITE_SIZE"]) * 1024.0 * w_scale / runs
    alg, cells = meta["algorithmic_bytes"], meta["cells"]
    lines = ["# HBM traffic of the 64-disc batch (bench.py --batch)", "",
             "Commands (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output root):", "",
             "    " + cmd["b_fetch"], "    " + cmd["b_write"], "",
             f"Counters summed over every pass-kernel dispatch of the run and divided by its "
             f"{runs} graph runs (untuned plan); scaled by the copy calibration of "
             f"traffic_passes_bifluid_1024x2048.md (FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x "
             f"{w_scale:.4f}).", "",
             f"Per run: {rd / 1e6:.1f} MB read, {wr / 1e6:.1f} MB written, {(rd + wr) / 1e6:.1f} MB in "
             f"all for {cells} cells = {(rd + wr) / cells:.1f} B/cell, against {alg / 1e6:.1f} MB "
             f"algorithmic ({alg / cells:.1f} B/cell): {(rd + wr) / alg:.2f}x."]
    with open(os.path.join(prof, "traffic_batch64.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_ss_traffic(out, prof, cmd, f_scale, w_scale):
    """profiles/traffic_semispectral_flaring_1200x2048.md: HBM bytes per
    dispatch of the semi-spectral middle pass, per launch variant (the tuner
    runs several; each reads the stored operators once) against the
    algorithmic bytes."""
    per = {}
    for key, counter, scale in (("ss_fetch", "FETCH_SIZE", f_scale), ("ss_write", "WRITE_SIZE", w_scale)):
        for r in _csv_rows(os.path.join(out, key), "_counter_collection.csv"):
            n = _kname(r)
            if n.startswith("k_ss_pass") and r["Counter_Name"] == counter:
                per.setdefault(n, {}).setdefault(counter, []).append(float(r["Counter_Value"]) * 1024.0 * scale)
    meta = _last_json(os.path.join(out, "ss_fetch.out"))
    if not per or not meta or "middle_pass" not in meta:
        return
    mp = meta["middle_pass"]
    ar, aw = mp["algorithmic_read"], mp["algorithmic_write"]
    lines = ["# HBM traffic of the semi-spectral middle pass, App. D flaring gas disc 1200x2048", "",
             "Commands (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output root):", "",
             "    " + cmd["ss_fetch"], "    " + cmd["ss_write"], "",
             f"Per dispatch of `k_ss_pass`, by launch variant (the run tunes the middle pass, so "
             f"several variants run); counters scaled by the copy calibration of "
             f"traffic_passes_bifluid_1024x2048.md (FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x "
             f"{w_scale:.4f}).  Algorithmic bytes: {ar / 1e6:.1f} MB read (the stored operators, "
             f"{meta['table_bytes'] / 1e6:.1f} MB, and Sigma~) and {aw / 1e6:.1f} MB written (g^_r, g^_phi).",
             "", "| Variant | Dispatches | Read (MB) | Read / alg. | Written (MB) | Written / alg. |",
             "|---|---|---|---|---|---|"]
    for n in sorted(per):
        f, w = per[n].get("FETCH_SIZE"), per[n].get("WRITE_SIZE")
        if not f or not w:
            continue
        rd, wr = sum(f) / len(f), sum(w) / len(w)
        lines.append(f"| `{n}` | {len(f)} / {len(w)} | {rd / 1e6:.1f} | {rd / ar:.3f} | {wr / 1e6:.1f} | "
                     f"{wr / aw:.3f} |")
    with open(os.path.join(prof, "traffic_semispectral_flaring_1200x2048.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_batch_sq(out, prof, cmd):
    """profiles/sq_batch64.md: VALU and LDS work of one 64-disc batch run (all
    pass kernels of the graph) and the time the VALU issue rate alone needs."""
    v = _counter_sums(os.path.join(out, "b_sq"), "k_pass")
    meta = _last_json(os.path.join(out, "b_sq.out"))
    if not v or not meta:
        return
    runs = meta["graph_runs"]
    per = {k: sum(x) / runs for k, x in v.items()}
    alg, cells = meta["algorithmic_bytes"], meta["cells"]
    # one wave64 VALU instruction per SIMD every 4 cycles, 1024 SIMDs
    floor_s = per["SQ_INSTS_VALU"] * 4 / (VALU_SIMDS * VALU_CLOCK_HZ)
    gui = sum(v["GRBM_GUI_ACTIVE"]) / 8  # summed over the 8 XCDs
    busy = 100 * sum(v["SQ_ACTIVE_INST_VALU"]) / 256 / gui
    lines = ["# VALU work of the 64-disc batch (bench.py --batch)", "",
             "Command (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output root):", "",
             "    " + cmd["b_sq"], "",
             f"Counters summed over every pass-kernel dispatch of the run (untuned plan) and divided "
             f"by its {runs} graph runs.  Per run:", "",
             "| Quantity | Value |", "|---|---|",
             f"| waves | {per['SQ_WAVES']:.0f} |",
             f"| VALU wave-instructions (SQ_INSTS_VALU) | {per['SQ_INSTS_VALU'] / 1e6:.1f} M |",
             f"| LDS wave-instructions (SQ_INSTS_LDS) | {per['SQ_INSTS_LDS'] / 1e6:.1f} M |",
             f"| VALU instructions per cell | {per['SQ_INSTS_VALU'] * 64 / cells:.0f} lane-ops |",
             f"| VALUBusy over the pass kernels (100 SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE) | "
             f"{busy:.1f} % |",
             f"| time at the full VALU issue rate (4 cycles per wave-instruction, "
             f"{VALU_SIMDS} SIMDs, {VALU_CLOCK_HZ / 1e9:.1f} GHz) | {floor_s * 1e6:.1f} us |",
             f"| HBM fraction if the run took only that time ({alg / 1e6:.1f} MB algorithmic) | "
             f"{alg / floor_s / (HBM_PEAK_GBS * 1e9):.2f} |"]
    with open(os.path.join(prof, "sq_batch64.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_direct(out, prof, cmd):
    """profiles/valu_direct_sum.md: VALU instruction mix and issue rate of the
    direct-sum kernels (the FP64 64x128 and FP32 256x512 workloads)."""
    stats = {r["Name"].split("(")[0].replace("void ", ""): r for r in _csv_rows(os.path.join(out, "dir_kt"),
                                                                               "_kernel_stats.csv")}
    rows = _csv_rows(os.path.join(out, "dir_valu"), "_counter_collection.csv")
    lines = ["# VALU use of the direct sums (bench.py --direct)", "",
             "Commands (from /tmp, TMPDIR=/tmp; `<repo>` = repository root, `<out>` = output root):", "",
             "    " + cmd["dir_kt"], "    " + cmd["dir_valu"], "",
             "Per dispatch (means): VALU instructions are wave64 instructions, per pair = "
             "instructions x 64 / (n_r n_phi)^2 (256x512 float, 64x128 double, one fluid); nominal "
             "issue ratio = instructions x 4 cycles / (1024 SIMDs x 2.4 GHz x kernel time), which "
             "is not a hard ceiling (a mix can exceed 1 when some of its instructions do not hold "
             "the SIMD for four cycles); FLOP rate = (add + mul + 2 fma) x 64 / kernel time "
             "against the 78.6 TFLOP/s vector issue rate (FP32 without packed instructions, FP64).",
             "",
             "| Kernel | Time (us) | VALU instr. | per pair | FP add/mul/fma | Nominal issue ratio "
             "| TFLOP/s | of 78.6 |",
             "|---|---|---|---|---|---|---|---|"]
    for kname, cells in (("k_direct<float, 1>", 256 * 512), ("k_direct<double, 1>", 64 * 128)):
        st = stats.get(kname)
        vals = {}
        for r in rows:
            if r["Kernel_Name"].replace("void ", "").startswith(kname):
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        if st is None or not vals:
            continue
        mean = {k: sum(v) / len(v) for k, v in vals.items()}
        t = float(st["AverageNs"]) * 1e-9
        sfx = "F32" if "float" in kname else "F64"
        add, mul, fma = (mean.get(f"SQ_INSTS_VALU_{o}_{sfx}", 0.0) for o in ("ADD", "MUL", "FMA"))
        issue = mean["SQ_INSTS_VALU"] * 4 / (VALU_SIMDS * VALU_CLOCK_HZ * t)
        tflops = (add + mul + 2 * fma) * 64 / t / 1e12
        per_pair = mean["SQ_INSTS_VALU"] * 64 / float(cells) ** 2
        lines.append(f"| `{kname}` | {t * 1e6:.1f} | {mean['SQ_INSTS_VALU']:.4g} | {per_pair:.1f} | "
                     f"{add:.3g} / {mul:.3g} / {fma:.3g} | {issue:.2f} | {tflops:.2f} | "
                     f"{tflops / VALU_PEAK_TFLOPS:.2f} |")
    with open(os.path.join(prof, "valu_direct_sum.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def direct_measurement(sg, T, W, dev):
    """The direct sums alone: the FP64 64 x 128 workload and an FP32 256 x 512
    single-fluid disc (h = 0.05), pairs per second."""
    import numpy as np
    import torch
    out = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w = W.direct_fp64()
    cases = [("fp64_64x128", w, torch.float64, 10)]
    ws = W.single_fft(seed=3, n_r=256, n_phi=512)
    cases.append(("fp32_256x512", dict(ws, sigma=ws["sigma"][0], h=ws["h"][0]), torch.float32, 3))
    for name, c, dt, reps in cases:
        g = sg.grid(c["n_r"], c["n_phi"], c["r_min"], c["r_max"])
        s = torch.tensor(np.asarray(c["sigma"]).reshape(1, c["n_r"], c["n_phi"]), dtype=dt, device=dev)
        h = [float(np.atleast_1d(c["h"])[0])]
        T.direct(g, h, s)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            T.direct(g, h, s)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pairs = (c["n_r"] * c["n_phi"]) ** 2
        out[name] = {"ms": round(ms, 4), "pairs_per_s": round(pairs / ms * 1e3, 1)}
    return out


def oracle_rates():
    """The oracle's own speed on this host (CPU only; offset-table FP64 sum,
    OpenMP over target cells): the full field of the 64 x 128 FP64 workload,
    of the 512 x 1024 single-fluid workload and of the 256 x 512 two-fluid
    adjoint workload, and 512 seeded cells of every disc of the 64-disc batch.
    Each call builds its disc's tables first; that build is timed alone (a
    one-cell call) and kept out of the per-cell rate."""
    import numpy as np
    import oracle as O
    from paper_2506_10812_amd import workloads as W

    def timed(w, h, targets=None):
        nr, nphi = w["n_r"], w["n_phi"]
        args = (nr, nphi, w["r_min"], w["r_max"], h, np.asarray(w["sigma"], dtype=np.float64))
        t0 = time.perf_counter()
        O.field_table(*args, targets=np.zeros(1, dtype=np.int64))
        build = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.field_table(*args, targets=targets)
        total = time.perf_counter() - t0
        n = nr * nphi if targets is None else len(targets)
        return build, max(total - build, 1e-9), n

    out = {"threads": O.threads(), "host_cpus": os.cpu_count(), "kind": "oracle, offset-table FP64"}
    for name, w in (("fp64_64x128_full", W.direct_fp64()), ("single_fluid_512x1024_full", W.single_fft()),
                    ("bifluid_256x512_full", W.adjoint())):
        print(f"bench: oracle rate, {name}", file=sys.stderr, flush=True)
        b, s, n = timed(w, w["h"])
        out[name] = {"cells": n, "table_build_s": round(b, 3), "sum_s": round(s, 3),
                     "cells_per_s": round(n / s, 1)}
    print("bench: oracle rate, 64-disc batch (512 cells per disc)", file=sys.stderr, flush=True)
    bs = ss = 0.0
    nt = 0
    for i, w in enumerate(W.batch64()):
        b, s, n = timed(w, w["h"], W.sample_cells(w["n_r"], w["n_phi"], 512, seed=100 + i))
        bs, ss, nt = bs + b, ss + s, nt + n
    out["batch64_sampled"] = {"cells": nt, "table_build_s": round(bs, 3), "sum_s": round(ss, 3),
                              "cells_per_s": round(nt / ss, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--summarize-rocprof", metavar="DIR")
    ap.add_argument("--semispectral", action="store_true")
    ap.add_argument("--direct", action="store_true")
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--oracle-rates", action="store_true")
    args = ap.parse_args()
    if args.oracle_rates:
        print(json.dumps(oracle_rates()))
        return
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (got --gpus {args.gpus}); "
              "the path's sharding across GPUs is a design, not implemented here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    import paper_2506_10812_amd as sg
    from paper_2506_10812_amd import torch_ops as T
    from paper_2506_10812_amd import workloads as W

    if args.semispectral:
        print(json.dumps(semispectral_measurement(sg, T, W, dev)))
        return
    if args.direct:
        print(json.dumps(direct_measurement(sg, T, W, dev)))
        return
    if args.batch:
        print(json.dumps(batch_measurement(sg, T, W, dev, args.steps, args.warmup, not args.no_tune)))
        return

    w = W.bifluid_fft()
    nr, nphi, nf = w["n_r"], w["n_phi"], len(w["h"])
    cells = nr * nphi
    print(f"bench: building tables for {nr}x{nphi} two-fluid disc", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    F = T.FFTField([w], device=dev)
    torch.cuda.synchronize()
    table_s = time.perf_counter() - t0
    # the first build of a process also loads the library's code objects; a
    # second build of the same tables shows the per-disc cost
    t0 = time.perf_counter()
    T.build_table(F.specs[0][0], F.specs[0][1], 0, dev)
    torch.cuda.synchronize()
    table_repeat_s = time.perf_counter() - t0
    F.set_sigma(0, w["sigma"])
    stream = torch.cuda.current_stream()
    # untuned per-pass times, then the autotuner (part of the library's normal
    # use: once per batch shape); the timed steps run the tuned plan
    ms_untuned = sg.field_fft_profile(F.discs, F.ws, 20, stream=stream)
    tuned = F.tune(stream=stream) if not args.no_tune else []

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # warm steps: launched back to back; the disc's 118 MB working set
    # then stays in the 256 MB Infinity Cache (reported in extra only)
    for _ in range(args.warmup):
        F.run()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        F.run()
    e1.record(stream)
    torch.cuda.synchronize()
    warm_ms = e0.elapsed_time(e1) / args.steps

    # the timed steps (the headline): every step starts cold.  Before each
    # one a 512 MiB buffer is rewritten (outside the step's events), which
    # evicts the L2s and the Infinity Cache; each step is timed alone with
    # HIP events on the launch stream and the K step times are summed
    flush = torch.empty(FLUSH_FLOATS, dtype=torch.float32, device=dev)
    for _ in range(2):
        flush.fill_(1.0)
        F.run()
    print(f"bench: timing {args.steps} cold steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold = []
    for _ in range(args.steps):
        flush.fill_(1.0)
        e0.record(stream)
        F.run()
        e1.record(stream)
        e1.synchronize()
        cold.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = float(np.sum(cold)) / args.steps
    value = cells / (ms_step * 1e-3)

    # one cold step pass by pass (sg_field_fft_profile with reps = 1 runs the
    # passes once each, in order, with events between them), repeated after
    # a flush each time: the roofline's kernel time is pass 2's mean here
    reps_c = max(10, min(args.steps, 50))
    cp = []
    for _ in range(reps_c):
        flush.fill_(1.0)
        cp.append(sg.field_fft_profile(F.discs, F.ws, 1, stream=stream))
    ms_pass = [float(v) for v in np.mean(np.array(cp), axis=0)]
    # the same after a clean eviction (reported in extra only): the rewrite is
    # followed by a read of a second 512 MiB buffer, which evicts the
    # rewritten lines, so the step starts with nothing of its own cached and
    # no dirty lines of the flush left to write back
    flush2 = torch.ones(FLUSH_FLOATS, dtype=torch.float32, device=dev)
    cc, cs = [], []
    for _ in range(reps_c):
        flush.fill_(1.0)
        flush2.sum()
        cc.append(sg.field_fft_profile(F.discs, F.ws, 1, stream=stream))
        flush.fill_(1.0)
        flush2.sum()
        e0.record(stream)
        F.run()
        e1.record(stream)
        e1.synchronize()
        cs.append(e0.elapsed_time(e1))
    ms_pass_clean = [float(v) for v in np.mean(np.array(cc), axis=0)]
    ms_step_clean = float(np.mean(cs))
    del flush, flush2
    # achievable HBM bandwidth for comparison with the 8 TB/s spec: a 1 GiB
    # device-to-device copy (4x the Infinity Cache), read plus written bytes
    # over its time, mean of 10 copies between HIP events
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    # warm per-pass durations (each pass's launches back to back)
    reps = max(10, min(args.steps, 200))
    ms_pass_warm = sg.field_fft_profile(F.discs, F.ws, reps, stream=stream)
    pb = pass_bytes(nr, nphi, nf)
    names = ["pass1", "pass2", "pass3"]
    dom = int(np.argmax(ms_pass))
    dom_name = names[dom]
    achieved = pb[dom_name] / (ms_pass[dom] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        # every variant of the pass moves the same bytes (radix order and tile
        # shape change the arithmetic order only), so the counters of any
        # variant of these kernel sources describe the timed one
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("kernel") == dom_name:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom_name, "kernel_name": pass2_kernel_name(nr, nf, tuned) if dom == 1 else None,
                "kernel_ms": round(ms_pass[dom], 5), "cache": "cold",
                "algorithmic_bytes": pb[dom_name]}

    # accuracy vs the FP64 oracle on 16384 seeded cells (also the CPU baseline:
    # its table build, done once per disc like the library's, is timed on its
    # own with a one-cell call and taken out of the per-cell rate)
    cpu = None
    acc = None
    if not args.no_cpu:
        import oracle as O
        idx = W.sample_cells(nr, nphi, 16384)
        sig32 = F.sigma[0].double().cpu().numpy()
        print(f"bench: CPU oracle on {len(idx)} sampled cells", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        O.field_table(nr, nphi, w["r_min"], w["r_max"], w["h"], sig32, targets=idx[:1])
        build_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        rr, rp = O.field_table(nr, nphi, w["r_min"], w["r_max"], w["h"], sig32, targets=idx)
        cpu_s = time.perf_counter() - t0
        gr = F.g_r[0].double().cpu().numpy().reshape(nf, -1)[:, idx]
        gp = F.g_phi[0].double().cpu().numpy().reshape(nf, -1)[:, idx]
        acc = {f"{['gas', 'dust'][b]}_{c}": float(np.linalg.norm(x[b] - y[b]) / np.linalg.norm(y[b]))
               for b in range(nf) for c, x, y in (("g_r", gr, rr), ("g_phi", gp, rp))}
        sum_s = max(cpu_s - build_s, 1e-9)
        cpu = {"value": round((len(idx) - 1) / sum_s, 2), "unit": "cells/s", "cores": O.threads(),
               "kind": "oracle",
               "sample": f"{len(idx)} seeded cells of the same disc, offset-table FP64 oracle: "
                         f"{cpu_s:.1f} s in all, of which its table build (all four pairs, "
                         f"once per disc, timed alone) {build_s:.1f} s; value = cells per second "
                         f"of the summation"}

    extra = {"table_build_s": round(table_s, 3), "table_build_repeat_s": round(table_repeat_s, 4),
             "wall_s_timed": round(wall, 3),
             "cold_ms_per_step_median": round(float(np.median(cold)), 5),
             "warm_ms_per_step": round(warm_ms, 5),
             "warm_cells_per_s": round(cells / (warm_ms * 1e-3), 1),
             "warm_path_hbm_frac": round(pb["path"] / (warm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "ms_per_pass_cold": [round(v, 5) for v in ms_pass],
             "cold_clean_ms_per_step": round(ms_step_clean, 5),
             "hbm_copy_1gib_gbs": round(copy_gbs, 1),
             "ms_per_pass_cold_clean": [round(v, 5) for v in ms_pass_clean],
             "ms_per_pass_warm": [round(v, 5) for v in ms_pass_warm],
             "ms_per_pass_warm_untuned": [round(v, 5) for v in ms_untuned],
             "pass_hbm_frac_cold": [round(pb[k] / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                    for k, t in zip(names, ms_pass)],
             "pass_hbm_frac_warm": [round(pb[k] / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                    for k, t in zip(names, ms_pass_warm)],
             "tuned": [{k: r[k] for k in ("pass", "length", "small_radix_first", "groups_per_wg", "cluster",
                                          "candidates", "rejected")} for r in tuned],
             "path_algorithmic_bytes": pb["path"],
             "path_hbm_frac": round(pb["path"] / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "rel_rms_vs_fp64_oracle": acc}
    if not args.no_extra:
        extra.update(extra_measurements(sg, T, W, dev))

    out = {"metric": METRIC, "value": round(value, 1), "unit": "cells/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "two-fluid log-polar disc 1024x2048, r in [0.2,5], "
                                  "h_g=0.05, h_d=0.005, gas spiral + dust clumps, "
                                  "FFT path, 4 ordered pairs fused",
                      "n_r": nr, "n_phi": nphi, "fluids": nf, "cells_per_step": cells,
                      "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out))


def ss_bytes(sg, g, nf, flags=0):
    """Algorithmic HBM bytes of the semi-spectral middle pass: the stored
    radial operators (the table, banded modes included), one read of the
    Sigma~ column of every source and one write of g^_r, g^_phi."""
    ncol = g.n_phi // 2 + 1
    return sg.ss_table_bytes(g, nf, flags) + 8 * ncol * 3 * nf * g.n_r


def semispectral_measurement(sg, T, W, dev, steps=20):
    """The App. D flaring disc (gas, H/r = 0.05 (r/r_0)^0.25) on the
    semi-spectral path at 1200 x 2048: table build, step time and the middle
    pass against the HBM roofline (its parity is a test)."""
    import torch
    w = W.flaring()
    nr, nphi, nf = w["n_r"], w["n_phi"], w["sigma"].shape[0]
    S = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], nf, device=dev)
    S.sigma.copy_(torch.tensor(w["sigma"], dtype=torch.float32))
    S.refresh(w["H"])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    S.refresh(w["H"])
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    S.release_workspace()
    ms_untuned = sg.field_fft_profile([S.disc], S.ws, 10)
    tuned = sg.field_fft_tune([S.disc], S.ws)
    for _ in range(3):
        S.run()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        S.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ms_pass = sg.field_fft_profile([S.disc], S.ws, 10)
    # reverse mode: dL/dSigma (transposed operators) and dL/dH(r) (derivative
    # operators sampled on the fly), for seeded lam of the output's shape
    gen = torch.Generator(device="cpu").manual_seed(5)
    lam_r = torch.randn(S.g_r.shape, generator=gen).to(dev)
    lam_p = torch.randn(S.g_r.shape, generator=gen).to(dev)
    dsig = torch.empty_like(S.sigma)
    aws = torch.empty(sg.field_adjoint_workspace_bytes(S.disc), dtype=torch.uint8, device=dev)
    Hd = torch.tensor(w["H"], dtype=torch.float64, device=dev)
    dH = torch.empty_like(Hd)
    gws = torch.empty(sg.ss_grad_H_workspace_bytes(S.disc), dtype=torch.uint8, device=dev)

    def rev_ms(fn, n):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    # the second-order operators (hat weights) of the same disc: their build
    S2 = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], nf, sg.SECOND_ORDER, device=dev)
    S2.refresh(w["H"])
    torch.cuda.synchronize()
    e0.record()
    S2.refresh(w["H"])
    e1.record()
    torch.cuda.synchronize()
    build2_ms = e0.elapsed_time(e1)
    del S2
    adj_ms = rev_ms(lambda: sg.field_adjoint(S.disc, lam_r, lam_p, dsig, None, aws), 10)
    grad_ms = rev_ms(lambda: sg.ss_grad_H(S.disc, Hd, lam_r, lam_p, dH, gws), 3)
    del aws, gws
    mid = ss_bytes(sg, S.g, nf)
    mid_write = 16 * (nphi // 2 + 1) * nf * nr  # g^_r, g^_phi
    ach = mid / (ms_pass[1] * 1e-3) / 1e9
    out = {"workload": f"App. D flaring gas disc {nr}x{nphi}, r in [20,250], p=0.25",
           "table_bytes": sg.ss_table_bytes(S.g, nf), "table_build_ms": round(build_ms, 2),
           "second_order_table_build_ms": round(build2_ms, 2),
           "ms_per_step": round(ms, 4), "cells_per_s": round(nr * nphi / ms * 1e3, 1),
           "ms_per_pass": [round(v, 4) for v in ms_pass],
           "ms_per_pass_untuned": [round(v, 4) for v in ms_untuned],
           "middle_pass_shape": [r["groups_per_wg"] for r in tuned if r["pass"] == 2],
           "adjoint_dsigma_ms": round(adj_ms, 4), "grad_H_ms": round(grad_ms, 2),
           "middle_pass": {"bound": "hbm", "algorithmic_bytes": mid, "algorithmic_read": mid - mid_write,
                           "algorithmic_write": mid_write, "achieved": round(ach, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}}
    del S
    torch.cuda.empty_cache()
    return out


def batch_measurement(sg, T, W, dev, steps, warmup, tune):
    """The 64-disc batch alone: `warmup` graph runs, then `steps` runs each
    after a cache flush (timed alone with HIP events); graph_runs counts
    every run, for per-run counter totals."""
    import numpy as np
    import torch
    discs = W.batch64()
    Fb = T.FFTField(discs, device=dev)
    for i, d in enumerate(discs):
        Fb.set_sigma(i, d["sigma"])
    if tune:
        Fb.tune()
    for _ in range(warmup):
        Fb.run()
    flush = torch.empty(FLUSH_FLOATS, dtype=torch.float32, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(steps):
        flush.fill_(1.0)
        e0.record()
        Fb.run()
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    cells = sum(d["n_r"] * d["n_phi"] for d in discs)
    byts = sum(pass_bytes(d["n_r"], d["n_phi"], 1)["path"] for d in discs)
    m = float(np.mean(ms))
    return {"workload": "64 uneven single-fluid discs", "cells": cells, "algorithmic_bytes": byts,
            "graph_runs": warmup + steps, "cold_ms": round(m, 4),
            "cells_per_s": round(cells / m * 1e3, 1),
            "path_hbm_frac": round(byts / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def extra_measurements(sg, T, W, dev):
    """Secondary numbers: 64-disc batch, adjoint, FP64 direct sum, the
    semi-spectral path."""
    import torch
    res = {}
    res["semi_spectral_flaring_1200x2048"] = semispectral_measurement(sg, T, W, dev)
    discs = W.batch64()
    Fb = T.FFTField(discs, device=dev)
    for i, d in enumerate(discs):
        Fb.set_sigma(i, d["sigma"])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    ms_untuned = timed(Fb.run, 50)
    t0 = time.perf_counter()
    Fb.tune()
    tune_s = time.perf_counter() - t0
    ms = timed(Fb.run, 50)
    flush = torch.empty(FLUSH_FLOATS, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(20):
        flush.fill_(1.0)
        e0.record()
        Fb.run()
        e1.record()
        e1.synchronize()
        cold.append(e0.elapsed_time(e1))
    del flush
    ms_cold = sum(cold) / len(cold)
    cells = sum(d["n_r"] * d["n_phi"] for d in discs)
    byts = sum(pass_bytes(d["n_r"], d["n_phi"], 1)["path"] for d in discs)
    # the same discs one call each (plain single-disc path)
    singles = [T.FFTField([d], device=dev) for d in discs]
    for s_, d in zip(singles, discs):
        s_.set_sigma(0, d["sigma"])
        s_.run()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        for s_ in singles:
            s_.run()
    e1.record()
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1) / 10
    res["batch64"] = {"cells": cells, "ms": round(ms, 4), "ms_untuned": round(ms_untuned, 4),
                      "ms_cold": round(ms_cold, 4), "tune_s": round(tune_s, 2),
                      "cells_per_s": round(cells / ms * 1e3, 1),
                      "path_hbm_frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "path_hbm_frac_cold": round(byts / (ms_cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "looped_single_disc_ms": round(ms_loop, 4),
                      "speedup_vs_looped": round(ms_loop / ms, 3)}
    del Fb, singles
    # adjoint on the 256x512 two-fluid workload: dL/dSigma and dL/dh
    wa = W.adjoint()
    ga = sg.grid(wa["n_r"], wa["n_phi"], wa["r_min"], wa["r_max"])
    fa = sg.fluids(wa["h"])
    tab = T.build_table(ga, fa, sg.WITH_DH, dev)
    sig = torch.tensor(wa["sigma"], dtype=torch.float32, device=dev)
    lr = torch.randn_like(sig)
    lp = torch.randn_like(sig)
    ds = torch.empty_like(sig)
    dh = torch.zeros(len(wa["h"]), dtype=torch.float64, device=dev)
    disc = sg.make_disc(ga, fa, sg.WITH_DH, sig, lr, lp, tab)
    wsa = torch.empty(sg.field_adjoint_workspace_bytes(disc), dtype=torch.uint8, device=dev)
    ms_adj = timed(lambda: sg.field_adjoint(disc, lr, lp, ds, dh, wsa), 50)
    res["adjoint_256x512"] = {"ms": round(ms_adj, 4),
                              "cells_per_s": round(wa["n_r"] * wa["n_phi"] / ms_adj * 1e3, 1)}
    del tab, sig, lr, lp, ds, dh, wsa
    # FP64 direct sum on the 64x128 workload
    w = W.direct_fp64()
    g = sg.grid(w["n_r"], w["n_phi"], w["r_min"], w["r_max"])
    s = torch.tensor(w["sigma"], dtype=torch.float64, device=dev)
    T.direct(g, w["h"], s)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        T.direct(g, w["h"], s)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    pairs = (w["n_r"] * w["n_phi"]) ** 2
    res["direct_fp64_64x128"] = {"ms": round(ms, 4), "pairs_per_s": round(pairs / ms * 1e3, 1)}
    res["exponential_disc"] = exponential_disc_accuracy(sg, T, W, dev)
    return res


def exponential_disc_accuracy(sg, T, W, dev):
    """Accuracy against Freeman's closed form (the exponential disc of
    Sect. 4.2-4.3, radii y = r/(2 r_0) in [0.05, 2.5]), median and max of the
    relative error of the azimuthally averaged g_r, with point-sampled and
    second-order (SG_SECOND_ORDER) weights: the FFT path with H = 1e-4 r at
    1024 x 2048, and the semi-spectral path with constant H = 0.01 at
    1200 x 2048 (the paper's N_r), whose level the paper gives as ~1e-4."""
    import numpy as np
    import torch
    from scipy import special

    def err(w, gr):
        r = np.exp(np.log(w["r_min"]) + (np.arange(w["n_r"]) + 0.5) * np.log(w["r_max"] / w["r_min"]) / w["n_r"])
        y = r / (2 * w["r0"])
        ref = -2 * np.pi * w["sigma0"] * y * (special.i0e(y) * special.k0e(y) - special.i1e(y) * special.k1e(y))
        prof = gr.reshape(w["n_r"], w["n_phi"]).mean(axis=1)
        sel = (y >= 0.05) & (y <= 2.5)
        rel = np.abs(prof[sel] - ref[sel]) / np.abs(ref[sel])
        return {"median": float(f"{np.median(rel):.3e}"), "max": float(f"{rel.max():.3e}")}

    out = {}
    w = W.exponential(n_r=1024, n_phi=2048, h=1e-4, q=1)
    for name, fl in (("point", 0), ("second_order", sg.SECOND_ORDER)):
        F = T.FFTField([dict(w, h=[1e-4])], flags=fl, device=dev)
        F.set_sigma(0, w["sigma"])
        F.run()
        torch.cuda.synchronize()
        out[f"fft_h1e-4_1024x2048_{name}"] = err(w, F.g_r[0][0].double().cpu().numpy())
        del F
    w = W.exponential(n_r=1200, n_phi=2048, h=0.01, q=0)
    for name, fl in (("point", 0), ("second_order", sg.SECOND_ORDER)):
        S = T.SemiSpectral(w["n_r"], w["n_phi"], w["r_min"], w["r_max"], 1, fl, device=dev)
        S.refresh(w["H"])
        S.release_workspace()
        S.sigma.copy_(torch.tensor(w["sigma"], dtype=torch.float32))
        S.run()
        torch.cuda.synchronize()
        out[f"semispectral_H0.01_1200x2048_{name}"] = err(w, S.g_r[0].double().cpu().numpy())
        del S
    return out


if __name__ == "__main__":
    main()
