"""Benchmark of the P1 assembly hot path on one MI355X.

Step (timed): the whole assembly of the 2048 x 2048-cell unit square
(8,388,608 triangles, jitter 0.2 h, random vertex relabelling, FP64 values,
int32 indices) from (q, me) resident in HBM:
    fem_pattern        symbolic phase (CSR pattern, triangle lists, and the
                       order of each row's triangles around its vertex)
    fem_assemble       mass M, weighted mass Mw (w = 1 + x^2 + y^2),
                       stiffness S and elasticity K (lambda = 1, mu = 0.5),
                       all four in one pass over the rows
    fem_elas_pattern   2x2-block elasticity pattern
value = triangles / step time (M triangles per second).

Also reported: per-call HIP-event times and the roofline of each numeric
kernel (algorithmic bytes), the stiffness + mass pair alone, the gather floor
(the kernels' random accesses without arithmetic), the same kernels on the
square without the relabelling, the batched
block-diagonal assembly of 512 meshes (one graph-captured launch) against a
per-mesh launch loop, the forward + backward / forward ratio of the
differentiable assembly, the general sparse(I, J, V) compression of the
OptV2 triplet arrays, P1 tetrahedra on a 128^3 cube, P2 triangles, and the
CPU oracle timed on the step's mesh (stiffness + mass; single-threaded full
and numeric-only runs, and an all-cores numeric run).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extras]

L2 fetch and write traffic per launch comes from the rocprofv3 counter
summaries committed under profiles/ (FETCH_SIZE and WRITE_SIZE, scaled by what
the same counters read for a plain 1 GiB device copy); for the gather kernels
it counts the lines the L2 misses on, most of them served by the MALL rather
than HBM.  It is reported only while the kernel sources hash to the value
recorded there.  `--summarize KT PF PW` turns the
csv output of the three rocprofv3 runs (kernel trace, FETCH_SIZE, WRITE_SIZE)
of `bench.py --steps 5 --warmup 1 --no-cpu --no-extras --calib` into those
summaries.
"""
from __future__ import annotations

import argparse
import csv
import ctypes as C
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
METRIC = "M triangles/s & % HBM peak, P1 K+M FP64 @8.4M tris; batched vs looped"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "step_square2048_l2_traffic.md")
# the single kernel each timed call launches (deterministic row-owner kernels:
# operator mask, unroll, register row length)
CALL_KERNEL = {
    "assemble_rows": "fem::k_rows_fan<15, 8, 8>",
    "stiff_mass": "fem::k_rows_fan<5, 8, 8>",
    "elas_pattern": "fem::k_elas_pattern",
}


# the sources whose kernels each profile covers
PROFILE_SOURCES = {
    "step_square2048": ("fem_common.hip", "fem_internal.h", "fem_pattern.hip", "fem_numeric.hip"),
    "sparse_optv2_square2048": ("fem_common.hip", "fem_internal.h", "fem_sparse.hip"),
    "p2_square2048": ("fem_common.hip", "fem_internal.h", "fem_sparse.hip", "fem_p2.hip"),
    "tet_cube128": ("fem_common.hip", "fem_internal.h", "fem_pattern.hip", "fem_sparse.hip", "fem_tet.hip"),
    "adjoint_square512": ("fem_common.hip", "fem_internal.h", "fem_pattern.hip", "fem_numeric.hip",
                          "fem_adjoint.hip"),
    "batched_512meshes": ("fem_common.hip", "fem_internal.h", "fem_pattern.hip", "fem_numeric.hip"),
}


def source_hash(name="step_square2048"):
    """sha256 over the HIP sources of the kernels a profile covers."""
    files = [os.path.join(ROOT, "paper_1305_3122_amd", "csrc", f) for f in PROFILE_SOURCES[name]]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_short_name(name):
    """'void fem::k_x<1, 2>(int, ...)' -> 'fem::k_x<1, 2>'."""
    name = name.strip().strip('"').replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def read_traffic():
    """{kernel: (fetch_bytes, write_bytes)} per dispatch from the committed
    counter summary, or {} when it is missing or the sources have changed."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return {}
    out, ok = {}, False
    with open(PROFILE_TRAFFIC) as f:
        for line in f:
            m = re.match(r"source-sha256:\s*([0-9a-f]{64})", line.strip())
            if m:
                ok = m.group(1) == source_hash()
            if line.startswith("| `"):
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                name = cells[0].strip("`")
                try:
                    out[name] = (float(cells[4]) * 1e6, float(cells[5]) * 1e6)
                except (ValueError, IndexError):
                    pass
    return out if ok else {}


PROFILE_TITLES = {
    "step_square2048": ("one assembly step on the 2048x2048-cell unit square",
                        "Workload: 8,388,608 triangles, 4,198,401 vertices (jitter 0.2h, random vertex\n"
                        "relabelling), nnz 29,372,417; FP64 values, int32 indices.  Per-call averages over\n"
                        "the run (1 warm-up + 5 timed steps + the same 5 steps again with HIP events around\n"
                        "each call, plus the stiffness + mass pair timed alone and a 1 GiB fill and copy used\n"
                        "to calibrate the counters)."),
    "sparse_optv2_square2048": ("sparse(I, J, V) of the OptV2 triplets of the 2048x2048-cell square",
                                "Workload: Ig, Jg of all 9 local entries of the 8,388,608 triangles (75,497,472\n"
                                "triplets, random FP64 values) compressed to the 29,372,417-entry CSR; calls with\n"
                                "and without contributor lists, and re-summations (fem_sparse_values).  The 1 GiB\n"
                                "fill and copy calibrate the counters."),
    "p2_square2048": ("P2 triangles on the 2048x2048-cell unit square",
                      "Workload: 8,388,608 triangles, 4,198,401 vertices + 12,587,008 edges = 16,785,409\n"
                      "P2 DOFs (jitter 0.2h, random vertex relabelling), nnz 192,970,753; 5 edge\n"
                      "numberings (25.2M side triplets), 6 patterns (302M triplets, then the triangles\n"
                      "of every DOF), 11 mass + stiffness assemblies (one lane per DOF row); FP64\n"
                      "values, int32 indices.  The 1 GiB fill and copy calibrate the counters."),
    "tet_cube128": ("P1 tetrahedra on the 128^3-cell unit cube",
                    "Workload: 12,582,912 Kuhn tetrahedra, 2,146,689 vertices (jitter 0.1h, random\n"
                    "relabelling), nnz 31,802,497; 5 patterns (50.3M incidences in 128-vertex\n"
                    "buckets), 11 mass + stiffness assemblies (one lane per row);"
                    " FP64 values, int32 indices.  The 1 GiB fill and copy calibrate the\n"
                    "counters."),
    "adjoint_square512": ("the adjoints on the 512x512-cell unit square",
                          "Workload: 524,288 triangles, 263,169 vertices (jitter 0.2h, random vertex\n"
                          "relabelling), nnz 1,838,081; FP64.  S + Mw forward and its adjoint (dq, dw),\n"
                          "then K forward and its adjoint (dq, dlambda, dmu): 5 warm-up and 200 timed\n"
                          "calls of each forward, each backward and each forward + backward.  The 1 GiB\n"
                          "fill and copy calibrate the counters."),
    "batched_512meshes": ("512 meshes assembled as one block-diagonal matrix",
                          "Workload: 512 unit squares of 8 to 512 cells per side (log-uniform, seeded),\n"
                          "16,010,429 vertices and 31,776,926 triangles in all; S + M FP64.  The batch\n"
                          "pattern, the autotuner's trial launches, 13 replays of the graph-captured\n"
                          "batched launch, the 512 per-mesh patterns, 13 loops of 512 per-mesh launches\n"
                          "and 13 replays of that loop captured in a graph.  The 1 GiB fill and copy\n"
                          "calibrate the counters."),
}


# the bench.py run each profile covers: (short name of the output folders, arguments)
PROFILE_RUNS = {
    "step_square2048": ("step", "--steps 5 --warmup 1 --no-cpu --no-extras --calib"),
    "sparse_optv2_square2048": ("sparse", "--only sparse --calib"),
    "p2_square2048": ("p2", "--only p2 --calib"),
    "tet_cube128": ("tet", "--only tet --no-local --calib"),
    "adjoint_square512": ("adjoint", "--only adjoint --calib"),
    "batched_512meshes": ("batched", "--only batched --calib"),
}


def profile_command(name):
    """The commands that produce the profiles/ summaries of `name`."""
    key, args = PROFILE_RUNS[name]
    run = f"python3 $ROOT/bench.py {args}"
    out = "$ROOT/gpurun_out/" + key
    return "\n".join([
        "cd /tmp && export TMPDIR=/tmp",
        f"rocprofv3 --kernel-trace --stats --output-format csv -d {out}_kt -o run -- {run}",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {out}_pf -o run -- {run}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {out}_pw -o run -- {run}",
        f"cd $ROOT && python3 bench.py --summarize gpurun_out/{key}_kt gpurun_out/{key}_pf "
        f"gpurun_out/{key}_pw --profile-name {name}",
        "($ROOT: the repository root; the library built beforehand by __graft_entry__.build())"])


def summarize_profiles(kt_dir, pf_dir, pw_dir, command, name="step_square2048"):
    """Write the two profiles/ summaries from rocprofv3 csv output."""
    title, workload = PROFILE_TITLES[name]
    command = command or profile_command(name)
    stats_path = os.path.join(ROOT, "profiles", f"{name}_kernel_stats.md")
    traffic_path = os.path.join(ROOT, "profiles", f"{name}_l2_traffic.md")
    def one(d, pattern):
        f = glob.glob(os.path.join(d, "**", pattern), recursive=True)
        if not f:
            raise SystemExit(f"no {pattern} under {d}")
        return list(csv.DictReader(open(f[0])))

    stats = one(kt_dir, "*kernel_stats.csv")
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    sh = source_hash(name)
    lines = [f"# Kernel statistics: {title}",
             "",
             workload,
             "",
             f"source-sha256: {sh}  (sha256 of {', '.join(PROFILE_SOURCES[name])})",
             "",
             "Commands (from the repository root; rocprofv3 writes csv into the -d directories):",
             "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{kernel_short_name(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / total:.1f} % |")
    with open(stats_path, "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(kernel_short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return acc

    fetch = per_kernel(one(pf_dir, "*counter_collection.csv"), "FETCH_SIZE")
    write = per_kernel(one(pw_dir, "*counter_collection.csv"), "WRITE_SIZE")
    # calibration: the largest device copy (1 GiB read + 1 GiB write)
    gib_kib = float(1 << 20)
    cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    sf = gib_kib / cf if cf > 0 else float("nan")
    sw = gib_kib / cw if cw > 0 else float("nan")
    lines = [f"# L2 fetch and write traffic per dispatch: {title}",
             "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the dispatches of the run),",
             "each scaled by what the same counter reads for a plain 1 GiB device-to-device copy",
             "(1 GiB read, 1 GiB written).  Scaled MB = raw KiB x 1024 x scale / 1e6.  These are",
             "the bytes the L2 caches fetch from and write to the memory side.  For streaming",
             "kernels that is HBM traffic; for the random gathers of q (67 MB) most fetched lines",
             "are served by the 256 MB last-level cache (MALL) in front of HBM, so the fetch",
             "figures of gather kernels are L2-miss line traffic, not HBM traffic (they can",
             "exceed what HBM could deliver in the kernel's time).",
             "",
             f"source-sha256: {sh}  (sha256 of {', '.join(PROFILE_SOURCES[name])})",
             "",
             f"fetch-scale: {sf:.4f}  (copy of 1 GiB: FETCH_SIZE {cf:.1f} KiB)",
             f"write-scale: {sw:.4f}  (copy of 1 GiB: WRITE_SIZE {cw:.1f} KiB)",
             "",
             "Commands (from the repository root):", "", "```", command, "```", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch MB (scaled) | write MB (scaled) |",
             "|---|---|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write), key=lambda k: -np.mean(fetch.get(k, [0.0]))):
        f_kib = float(np.mean(fetch[k])) if k in fetch else float("nan")
        w_kib = float(np.mean(write[k])) if k in write else float("nan")
        lines.append(f"| `{k}` | {len(fetch.get(k, write.get(k, [])))} | {f_kib:.1f} | {w_kib:.1f} | "
                     f"{f_kib * 1024 * sf / 1e6:.3f} | {w_kib * 1024 * sw / 1e6:.3f} |")
    with open(traffic_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(stats_path)
    print(traffic_path)


def algorithmic_bytes(nq, nme, nnz):
    """Bytes the method must move per call (inputs once, outputs once)."""
    me, q, w = 12 * nme, 16 * nq, 8 * nq
    vals = 8 * nnz
    return {
        "pattern": me + 4 * (nq + 1) + 4 * nnz,           # me -> row_ptr, col_idx
        "assemble": me + q + w + 7 * vals,                 # -> M, Mw, S, K (4 per entry)
        "assemble_rows": me + q + w + 7 * vals,            # the same pass, kernel alone
        "elas_pattern": 4 * (nq + 1) + 4 * nnz + 4 * (2 * nq + 1) + 16 * nnz,
        "stiff_mass": me + q + 2 * vals,
        "stiff_mass_full": me + q + 4 * (nq + 1) + 4 * nnz + 2 * vals,
    }


def design_bytes(nq, nme, nnz):
    """Bytes the row-owner kernels stream by design: their index arrays
    (row_ptr, the fan codes, col_idx; every row of these meshes has a fan
    code, so inc_ptr and inc_pos are not read), the unique inputs and the
    outputs (each once); the packed (x, y, w, 0) copy for Mw is written and
    read."""
    idx = 4 * (nq + 1) + 8 * nq + 4 * nnz
    q, vals = 16 * nq, 8 * nnz
    return {
        "assemble": idx + q + 8 * nq + 2 * 32 * nq + 7 * vals,
        "assemble_rows": idx + 32 * nq + 7 * vals,
        "stiff_mass": idx + q + 2 * vals,
    }


class Step:
    """Preallocated buffers and the raw C calls of one assembly step."""

    def __init__(self, fem, lib, torch, m, w, lam, mu):
        dev = torch.device("cuda:0")
        self.torch, self.fem, self.lib = torch, fem, lib
        self.nq, self.nme = m.nq, m.nme
        self.q = torch.from_numpy(m.q).to(dev)
        self.me = torch.from_numpy(m.me).to(dev)
        self.w = torch.from_numpy(w).to(dev)
        self.lam, self.mu = lam, mu
        ws = C.c_size_t(0)
        fem._lib.check(lib.fem_pattern_workspace(m.nq, m.nme, C.byref(ws)))
        self.ws = int(ws.value)
        self.cap = int(lib.fem_nnz_bound(m.nq, m.nme))
        i32 = dict(dtype=torch.int32, device=dev)
        self.row_ptr = torch.empty(m.nq + 1, **i32)
        self.col_idx = torch.empty(self.cap, **i32)
        self.inc_ptr = torch.empty(m.nq + 1, **i32)
        self.inc = torch.empty(3 * m.nme, **i32)
        self.inc_pos = torch.empty(3 * m.nme, **i32)
        self.fan = torch.empty(m.nq, dtype=torch.int64, device=dev)
        self.work = torch.empty(self.ws, dtype=torch.uint8, device=dev)
        self.rpe = torch.empty(2 * m.nq + 1, **i32)
        self.nnz = None
        self.pattern()
        torch.cuda.synchronize()
        f64 = dict(dtype=torch.float64, device=dev)
        self.M = torch.empty(self.nnz, **f64)
        self.Mw = torch.empty(self.nnz, **f64)
        self.S = torch.empty(self.nnz, **f64)
        self.K = torch.empty(4 * self.nnz, **f64)
        self.cie = torch.empty(4 * self.nnz, **i32)
        aw = C.c_size_t(0)
        fem._lib.check(lib.fem_assemble_workspace(m.nq, 15, C.byref(aw)))
        self.awork = torch.empty(max(int(aw.value), 1), dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream().cuda_stream

    def pattern(self):
        n = C.c_int64(0)
        s = self.torch.cuda.current_stream().cuda_stream
        self.fem._lib.check(self.lib.fem_pattern(
            self.nq, self.nme, self.me.data_ptr(), self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
            self.cap, self.inc_ptr.data_ptr(), self.inc.data_ptr(), self.inc_pos.data_ptr(),
            self.fan.data_ptr(), None, self.work.data_ptr(), self.ws, C.byref(n), s))
        self.nnz = int(n.value)

    def _pat(self):
        return (self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.inc_ptr.data_ptr(),
                self.inc_pos.data_ptr(), self.fan.data_ptr(), None)

    def assemble(self):
        # M, Mw, S and K in one pass (the gathers of q and w shared)
        self.fem._lib.check(self.lib.fem_assemble(
            15, self.nq, self.nme, self.nnz, self.q.data_ptr(), self.w.data_ptr(), self.me.data_ptr(),
            *self._pat(), self.lam, self.mu, self.M.data_ptr(), self.Mw.data_ptr(), self.S.data_ptr(),
            self.K.data_ptr(), self.awork.data_ptr(), self.awork.numel(), None, 0, self.stream))

    def assemble_rows(self):
        # the same pass on the (x, y, w) records the step's call left in the
        # workspace (FEM_PACKED_QW): the row-owner kernel alone
        self.fem._lib.check(self.lib.fem_assemble(
            15, self.nq, self.nme, self.nnz, self.q.data_ptr(), self.w.data_ptr(), self.me.data_ptr(),
            *self._pat(), self.lam, self.mu, self.M.data_ptr(), self.Mw.data_ptr(), self.S.data_ptr(),
            self.K.data_ptr(), self.awork.data_ptr(), self.awork.numel(), None,
            self.fem.FEM_PACKED_QW, self.stream))

    def elas_pattern(self):
        self.fem._lib.check(self.lib.fem_elas_pattern(
            self.nq, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.rpe.data_ptr(),
            self.cie.data_ptr(), self.stream))

    def stiff_mass(self):
        self.fem._lib.check(self.lib.fem_assemble_stiff_mass(
            self.nq, self.nme, self.nnz, self.q.data_ptr(), self.me.data_ptr(), *self._pat(),
            self.S.data_ptr(), self.M.data_ptr(), 0, self.stream))

    PARTS = ("pattern", "assemble", "elas_pattern")


def time_calls(torch, fn, reps):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def run_main(torch, fem, args):
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    t0 = time.time()
    m = mg.config_mesh(2)
    w = mg.weight_quadratic(m.q)
    log(f"[bench] cfg2 mesh nq={m.nq} nme={m.nme} built in {time.time() - t0:.1f}s")
    st = Step(fem, lib, torch, m, w, 1.0, 0.5)
    log(f"[bench] nnz={st.nnz}")
    for _ in range(args.warmup):
        for p in Step.PARTS:
            getattr(st, p)()
    torch.cuda.synchronize()
    # the timed steps, with no instrumentation inside them
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p in Step.PARTS:
            getattr(st, p)()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the per-call breakdown: the same steps again, each call bracketed by HIP
    # events on the launch stream (outside the timed region)
    ev = {p: [] for p in Step.PARTS}
    for _ in range(args.steps):
        for p in Step.PARTS:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            getattr(st, p)()
            b.record()
            ev[p].append((a, b))
    torch.cuda.synchronize()
    ab = algorithmic_bytes(m.nq, m.nme, st.nnz)
    us = {p: float(np.mean([a.elapsed_time(b) for a, b in ev[p]])) * 1e3 for p in Step.PARTS}
    # the stiffness + mass pair alone (not part of the step), warm and with the
    # 256 MB last-level cache flushed (a 1 GiB write) before every call
    us["stiff_mass"] = time_calls(torch, st.stiff_mass, args.steps)
    # like-for-like with the CPU baseline's full assembly: pattern (with the
    # fan codes) and then the stiffness + mass pair
    us["stiff_mass_full"] = time_calls(torch, lambda: (st.pattern(), st.stiff_mass()),
                                       max(args.steps // 2, 3))
    st.assemble()
    us["assemble_rows"] = time_calls(torch, st.assemble_rows, args.steps)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
    cold = []
    for _ in range(max(args.steps // 2, 3)):
        flush.fill_(0.0)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        st.stiff_mass()
        b.record()
        torch.cuda.synchronize()
        cold.append(a.elapsed_time(b) * 1e3)
    # practical ceiling: a plain 1 GiB device-to-device copy (1 GiB read + 1 GiB written)
    src = flush
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (a.elapsed_time(b) * 1e-3) / 1e9
    del flush, src, dst
    db = design_bytes(m.nq, m.nme, st.nnz)
    kern = {}
    for p, t in us.items():
        gbs = ab[p] / (t * 1e-6) / 1e9
        kern[p] = {"us": round(t, 2), "alg_bytes": ab[p], "alg_GBps": round(gbs, 1),
                   "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "Mtri_per_s": round(m.nme / t, 1)}
        if p in db:
            kern[p]["design_bytes"] = db[p]
            kern[p]["design_frac_hbm"] = round(db[p] / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    kern["stiff_mass"]["us_cold"] = round(float(np.median(cold)), 2)
    st.copy_gbs = round(copy_gbs, 1)
    log(f"[bench] step {ms_per_step:.3f} ms; " +
        ", ".join(f"{p} {kern[p]['us']:.0f}us" for p in kern))
    return m, st, ms_per_step, kern


def run_gather_floor(torch, fem, st, reps):
    """The random accesses of the row-owner kernels alone (fem_gather_probe):
    the column stream of the step's pattern gathering the 16-byte records of
    q with no arithmetic, in the relabelled order (random lines) and in
    stream order (the same loads with perfect locality)."""
    lib = st.lib
    sink = torch.empty(int(lib.fem_gather_probe_threads()), dtype=torch.float64, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream

    def probe(mode):
        fem._lib.check(lib.fem_gather_probe(st.nnz, st.nq, st.col_idx.data_ptr(), st.q.data_ptr(),
                                            mode, sink.data_ptr(), s))

    t_rand = time_calls(torch, lambda: probe(0), reps)
    t_seq = time_calls(torch, lambda: probe(1), reps)
    out = {"gathers": st.nnz, "record_bytes": 16,
           "random_us": round(t_rand, 1), "stream_order_us": round(t_seq, 1),
           "random_Ggathers_per_s": round(st.nnz / t_rand / 1e3, 1),
           "note": "col_idx read in order, q[col_idx[e]] gathered (random on the relabelled mesh) "
                   "or q[e mod nq] (stream order); the fan kernels gather the nnz - nq off-diagonal "
                   "records per call"}
    log(f"[bench] gather probe: {st.nnz} random gathers {t_rand:.0f}us, in stream order {t_seq:.0f}us")
    return out


def run_local(torch, fem, args):
    """The same kernels on the 2048 x 2048 square without the vertex
    relabelling (vertices numbered row by row, as a mesh generator emits
    them): the gathers of q are then local, and the kernels' own streams
    bound them."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    m = mg.unit_square(2048, seed=mg.BASE_SEED + 2, permute=False)
    w = mg.weight_quadratic(m.q)
    st = Step(fem, lib, torch, m, w, 1.0, 0.5)
    st.assemble()
    t_sm = time_calls(torch, st.stiff_mass, args.steps)
    t_rows = time_calls(torch, st.assemble_rows, args.steps)
    t_pat = time_calls(torch, st.pattern, max(args.steps // 4, 3))
    ab = algorithmic_bytes(m.nq, m.nme, st.nnz)
    out = {"workload": "unit square 2048x2048 cells, jitter 0.2h, vertices numbered row by row "
                       "(no relabelling); same kernels and calls as the step",
           "nnz": st.nnz}
    for key, t in (("stiff_mass", t_sm), ("assemble_rows", t_rows)):
        gbs = ab[key] / (t * 1e-6) / 1e9
        out[key] = {"kernel": CALL_KERNEL[key], "us": round(t, 1), "alg_bytes": ab[key],
                    "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["pattern_us"] = round(t_pat, 1)
    log(f"[bench] unrelabelled square: M+S {t_sm:.0f}us ({out['stiff_mass']['frac']:.3f}), "
        f"four operators {t_rows:.0f}us ({out['assemble_rows']['frac']:.3f}), pattern {t_pat:.0f}us")
    del st
    torch.cuda.empty_cache()
    return out


def run_batched(torch, fem, args):
    """512 meshes: one graph-captured batched launch vs a per-mesh launch loop."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    t0 = time.time()
    b = mg.config_mesh(4)
    dev = torch.device("cuda:0")
    log(f"[bench] cfg4 batch nb={b.nb} nq={b.q.shape[0]} nme={b.me.shape[0]} built in {time.time() - t0:.1f}s")
    q = torch.from_numpy(b.q).to(dev)
    me_g = fem.fem_batch_globalize(torch.from_numpy(b.me_local).to(dev),
                                   torch.from_numpy(b.vtx_off).to(dev),
                                   torch.from_numpy(b.elem_off).to(dev))
    nq_all = int(b.vtx_off[-1])
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    pat = fem.fem_pattern(me_g, nq_all)
    torch.cuda.synchronize()
    t_pat_batched = time.perf_counter() - tp0
    from paper_1305_3122_amd import autotune
    tune, table = autotune.tune_batched(fem, torch, pat, q, b.nb)
    S = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
    M = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    g = fem.Graph(side)
    with torch.cuda.stream(side):
        with g.capture():
            fem.fem_assemble_stiff_mass_batched(pat, q, b.nb, tune=tune, out_S=S, out_M=M, stream=side)
    # per-mesh patterns and buffers (setup, untimed)
    per = []
    tp0 = time.perf_counter()
    for i in range(b.nb):
        v0, v1 = int(b.vtx_off[i]), int(b.vtx_off[i + 1])
        e0, e1 = int(b.elem_off[i]), int(b.elem_off[i + 1])
        pm = fem.fem_pattern(torch.from_numpy(b.me_local[e0:e1]).to(dev), v1 - v0)
        per.append((pm, q[v0:v1], torch.empty(pm.nnz, dtype=torch.float64, device=dev),
                    torch.empty(pm.nnz, dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()
    t_pat_loop = time.perf_counter() - tp0
    s_ptr = side.cuda_stream

    def looped():
        for pm, qm, Sm, Mm in per:
            fem._lib.check(lib.fem_assemble_stiff_mass(
                pm.nq, pm.nme, pm.nnz, qm.data_ptr(), None, pm.row_ptr.data_ptr(),
                pm.col_idx.data_ptr(), pm.inc_ptr.data_ptr(), pm.inc_pos.data_ptr(),
                pm.fan.data_ptr(), None, Sm.data_ptr(), Mm.data_ptr(), 0, s_ptr))

    def batched():
        g.replay(side)

    res = {}
    for name, fn in (("batched_graph", batched), ("looped", looped)):
        for _ in range(3):
            fn()
        side.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        c = torch.cuda.Event(enable_timing=True)
        reps = 10
        a.record(side)
        for _ in range(reps):
            fn()
        c.record(side)
        side.synchronize()
        res[name] = a.elapsed_time(c) * 1e3 / reps
    # looped, captured in one graph (secondary)
    g2 = fem.Graph(side)
    with torch.cuda.stream(side):
        with g2.capture():
            looped()
    for _ in range(3):
        g2.replay(side)
    side.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    c = torch.cuda.Event(enable_timing=True)
    a.record(side)
    for _ in range(10):
        g2.replay(side)
    c.record(side)
    side.synchronize()
    res["looped_graph"] = a.elapsed_time(c) * 1e3 / 10
    # results agree block by block
    ok = True
    for i in (0, b.nb // 2, b.nb - 1):
        pm, qm, Sm, Mm = per[i]
        e0 = int(pat.row_ptr[int(b.vtx_off[i])])
        ok &= bool(torch.equal(S[e0:e0 + pm.nnz], Sm)) and bool(torch.equal(M[e0:e0 + pm.nnz], Mm))
    nme = int(b.elem_off[-1])
    out = {
        "workload": f"{b.nb} unit-square meshes, cells per side log-uniform in [8,512], S+M FP64",
        "nme": nme, "nnz": pat.nnz,
        "batched_graph_us": round(res["batched_graph"], 1),
        "looped_us": round(res["looped"], 1),
        "looped_graph_us": round(res["looped_graph"], 1),
        "speedup_vs_looped": round(res["looped"] / res["batched_graph"], 2),
        "batched_Mtri_per_s": round(nme / res["batched_graph"], 1),
        "pattern_batched_ms": round(t_pat_batched * 1e3, 1),
        "pattern_looped_ms": round(t_pat_loop * 1e3, 1),
        "tune": {"lds_entries": tune.lds_entries, "grid_blocks": tune.grid_blocks},
        "tune_table_us": table,
        "blocks_bitwise_equal": ok,
    }
    log(f"[bench] batched {out['batched_graph_us']}us vs looped {out['looped_us']}us "
        f"(x{out['speedup_vs_looped']})")
    return out


def run_adjoint(torch, fem, args):
    """Forward (S + Mw, one fused kernel after the (x, y, w) packing) against
    forward + adjoint on the 512 x 512 square, through the raw C calls with
    preallocated buffers, so that the ratio is that of the GPU work.  As in
    AssembleStiffWMass, the forward packs into the adjoint's workspace and the
    adjoint reuses those records (FEM_PACKED_QW)."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    dev = torch.device("cuda:0")
    m = mg.config_mesh(5)
    w = mg.weight_uniform(m.nq, 0.5, 2.0, seed=mg.BASE_SEED + 5)
    q = torch.from_numpy(m.q).to(dev)
    wd = torch.from_numpy(w).to(dev)
    pat = fem.fem_pattern(torch.from_numpy(m.me).to(dev), m.nq)
    fem.fem_transpose_map(pat)
    G = torch.from_numpy(mg.normal_seed(pat.nnz, seed=mg.BASE_SEED + 55)).to(dev)
    S = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
    Mw = torch.empty_like(S)
    dq = torch.empty((m.nq, 2), dtype=torch.float64, device=dev)
    dw = torch.empty(m.nq, dtype=torch.float64, device=dev)
    ops = fem.FEM_OP_STIFF | fem.FEM_OP_WMASS
    aw = C.c_size_t(0)
    fem._lib.check(lib.fem_adjoint_workspace(m.nq, pat.nnz, C.byref(aw)))
    awork = torch.empty(int(aw.value), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    P = (pat.row_ptr.data_ptr(), pat.col_idx.data_ptr(), pat.inc_ptr.data_ptr(),
         pat.inc_pos.data_ptr())

    def fwd():
        fem._lib.check(lib.fem_assemble(
            ops, m.nq, pat.nme, pat.nnz, q.data_ptr(), wd.data_ptr(), pat.me.data_ptr(), *P,
            pat.fan.data_ptr(), None, 0.0, 0.0, None, Mw.data_ptr(), S.data_ptr(), None,
            awork.data_ptr(), awork.numel(),
            None, 0, s))

    def bwd():
        fem._lib.check(lib.fem_adjoint_stiff_wmass(
            m.nq, pat.nme, pat.nnz, q.data_ptr(), wd.data_ptr(), *P, pat.fan.data_ptr(),
            pat.tpos.data_ptr(),
            G.data_ptr(), G.data_ptr(), dq.data_ptr(), dw.data_ptr(), awork.data_ptr(),
            awork.numel(), fem._lib.FEM_PACKED_QW, s))

    def t(fn, reps=200):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        c = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        c.record()
        torch.cuda.synchronize()
        return a.elapsed_time(c) * 1e3 / reps

    tf = t(fwd)
    fwd()
    tb = t(bwd)
    tfb = t(lambda: (fwd(), bwd()))
    out = {"workload": "unit square 512x512 (524288 triangles), S + Mw forward, adjoint of "
                       "<G, S + Mw> (dq, dw)",
           "fwd_us": round(tf, 1), "bwd_us": round(tb, 1), "fwd_bwd_us": round(tfb, 1),
           "ratio": round(tfb / tf, 2)}
    log(f"[bench] adjoint fwd {tf:.1f}us bwd {tb:.1f}us fwd+bwd {tfb:.1f}us ratio {tfb / tf:.2f}")
    # elasticity: K(q; lambda, mu) forward, adjoint for dq, dlambda, dmu
    lam, mu = 1.0, 0.5
    K = torch.empty(4 * pat.nnz, dtype=torch.float64, device=dev)
    GK = torch.from_numpy(mg.normal_seed(4 * pat.nnz, seed=mg.BASE_SEED + 56)).to(dev)
    ew = C.c_size_t(0)
    fem._lib.check(lib.fem_adjoint_elas_workspace(m.nq, pat.nnz, C.byref(ew)))
    ework = torch.empty(int(ew.value), dtype=torch.uint8, device=dev)
    dlm = torch.empty(2, dtype=torch.float64, device=dev)

    def efwd():
        fem._lib.check(lib.fem_assemble(
            fem.FEM_OP_ELAS, m.nq, pat.nme, pat.nnz, q.data_ptr(), None, pat.me.data_ptr(), *P,
            pat.fan.data_ptr(), None, lam, mu, None, None, None, K.data_ptr(), None, 0, None, 0, s))

    def ebwd():
        fem._lib.check(lib.fem_adjoint_elas(
            m.nq, pat.nme, pat.nnz, q.data_ptr(), *P, pat.fan.data_ptr(), pat.tpos.data_ptr(), lam,
            mu, GK.data_ptr(),
            dq.data_ptr(), dlm.data_ptr(), ework.data_ptr(), ework.numel(), 0, s))

    ef = t(efwd)
    eb = t(ebwd)
    efb = t(lambda: (efwd(), ebwd()))
    out["elasticity"] = {"workload": "same mesh, K (lambda=1, mu=0.5) forward, adjoint of <G, K> "
                                     "(dq, dlambda, dmu)",
                         "fwd_us": round(ef, 1), "bwd_us": round(eb, 1), "fwd_bwd_us": round(efb, 1),
                         "ratio": round(efb / ef, 2)}
    log(f"[bench] elasticity adjoint fwd {ef:.1f}us bwd {eb:.1f}us fwd+bwd {efb:.1f}us "
        f"ratio {efb / ef:.2f}")
    return out


def run_sparse(torch, fem, args):
    """General sparse(I, J, V, m, n) on the OptV2 triplet arrays of the
    2048 x 2048 square (Ig, Jg of all 9 local entries of every triangle, 75.5M
    triplets, random values): the compression the OptV2 assembly ends in."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    dev = torch.device("cuda:0")
    m = mg.config_mesh(2)
    a = np.tile(np.arange(3), 3)
    b = np.repeat(np.arange(3), 3)
    I = torch.from_numpy(np.ascontiguousarray(m.me[:, a].T.reshape(-1))).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(m.me[:, b].T.reshape(-1))).to(dev)
    nt = int(I.shape[0])
    V = torch.from_numpy(mg.normal_seed(nt, seed=mg.BASE_SEED + 202)).to(dev)
    ws = C.c_size_t(0)
    fem._lib.check(lib.fem_sparse_workspace(m.nq, m.nq, nt, C.byref(ws)))
    work = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    row_ptr = torch.empty(m.nq + 1, **i32)
    col = torch.empty(nt, **i32)
    vals = torch.empty(nt, dtype=torch.float64, device=dev)
    cptr = torch.empty(nt + 1, **i32)
    ctb = torch.empty(nt, **i32)
    s = torch.cuda.current_stream().cuda_stream
    nnz = C.c_int64(0)

    def call(with_contrib):
        fem._lib.check(lib.fem_sparse(
            m.nq, m.nq, nt, I.data_ptr(), J.data_ptr(), V.data_ptr(), row_ptr.data_ptr(),
            col.data_ptr(), vals.data_ptr(), nt, cptr.data_ptr() if with_contrib else None,
            ctb.data_ptr() if with_contrib else None, work.data_ptr(), int(ws.value),
            C.byref(nnz), s))

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record()
            fn()
            eb.record()
            torch.cuda.synchronize()
            out.append(ea.elapsed_time(eb) * 1e3)
        return float(np.median(out))

    t_plain = timed(lambda: call(False))
    t_contrib = timed(lambda: call(True))
    k = int(nnz.value)

    def values():
        fem._lib.check(lib.fem_sparse_values(k, cptr.data_ptr(), ctb.data_ptr(), V.data_ptr(),
                                             vals.data_ptr(), 0, s))

    t_values = timed(values, reps=10)
    alg = 16 * nt + 4 * (m.nq + 1) + 12 * k
    out = {"workload": "OptV2 triplets (Ig, Jg) of the 2048x2048 square, 75.5M triplets, FP64 values",
           "nt": nt, "nnz": k, "us": round(t_plain, 1), "us_with_contrib": round(t_contrib, 1),
           "Mtriplets_per_s": round(nt / t_plain, 1),
           "alg_bytes": alg, "alg_GBps": round(alg / (t_plain * 1e-6) / 1e9, 1),
           "resum_us": round(t_values, 1)}
    log(f"[bench] sparse nt={nt}: {t_plain:.0f}us ({nt / t_plain:.0f} Mtriplets/s), with "
        f"contributor lists {t_contrib:.0f}us, re-summation {t_values:.0f}us")
    del work
    return out


def run_tet(torch, fem, args):
    """P1 tetrahedra: the 128^3-cell unit cube (Kuhn, 12.6M tetrahedra, jitter
    0.1h, random relabelling), pattern and fused mass + stiffness (one lane
    per row)."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    dev = torch.device("cuda:0")
    n = 128
    m = mg.unit_cube(n, seed=mg.BASE_SEED + 128)
    me = torch.from_numpy(m.me).to(dev)
    q = torch.from_numpy(m.q).to(dev)
    ws = C.c_size_t(0)
    fem._lib.check(lib.fem_tet_pattern_workspace(m.nq, m.nme, C.byref(ws)))
    work = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
    cap = int(lib.fem_tet_nnz_bound(m.nq, m.nme))
    i32 = dict(dtype=torch.int32, device=dev)
    row_ptr = torch.empty(m.nq + 1, **i32)
    col = torch.empty(cap, **i32)
    inc_ptr = torch.empty(m.nq + 1, **i32)
    inc = torch.empty(4 * m.nme, **i32)
    inc_pos = torch.empty(4 * m.nme, **i32)
    s = torch.cuda.current_stream().cuda_stream
    nnz = C.c_int64(0)

    def pattern():
        fem._lib.check(lib.fem_tet_pattern(m.nq, m.nme, me.data_ptr(), row_ptr.data_ptr(),
                                           col.data_ptr(), cap, inc_ptr.data_ptr(), inc.data_ptr(),
                                           inc_pos.data_ptr(), work.data_ptr(), int(ws.value),
                                           C.byref(nnz), s))

    pattern()
    k = int(nnz.value)
    ops = fem.FEM_OP_MASS | fem.FEM_OP_STIFF
    M = torch.empty(k, dtype=torch.float64, device=dev)
    S = torch.empty_like(M)

    def assemble():
        fem._lib.check(lib.fem_tet_assemble(ops, m.nq, m.nme, k, q.data_ptr(), row_ptr.data_ptr(),
                                            col.data_ptr(), inc_ptr.data_ptr(), inc_pos.data_ptr(),
                                            M.data_ptr(), S.data_ptr(), 0, s))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record()
            fn()
            eb.record()
            torch.cuda.synchronize()
            out.append(ea.elapsed_time(eb) * 1e3)
        return float(np.median(out))

    tp = timed(pattern, 3)
    ta = timed(assemble, 10)
    # context: the same cube without the random relabelling (vertex ids in
    # grid order, so a row's neighbours are near it in memory)
    ta_o = None
    if not getattr(args, "no_local", False):
        mo = mg.unit_cube(n, seed=mg.BASE_SEED + 128, permute=False)
        me_o = torch.from_numpy(mo.me).to(dev)
        q_o = torch.from_numpy(mo.q).to(dev)
        pat_o = fem.fem_tet_pattern(me_o, mo.nq)
        vo = fem.fem_tet_assemble(pat_o, q_o)

        def assemble_o():
            fem.fem_tet_assemble(pat_o, q_o, out=vo)

        ta_o = timed(assemble_o, 10)
        del pat_o, vo, me_o, q_o
    # design bytes of the row kernel: q (24 per vertex), row_ptr and inc_ptr
    # (8 per vertex), col_idx (4 per entry), inc_pos (4 per incidence, 16 per
    # tetrahedron), M and S (16 per entry)
    alg = 32 * m.nq + 16 * m.nme + 20 * k
    out = {"workload": "unit cube 128^3 cells, 6 Kuhn tetrahedra per cell (12.6M), jitter 0.1h, "
                       "random relabelling; P1 mass + stiffness FP64",
           "nq": m.nq, "nme": m.nme, "nnz": k, "pattern_us": round(tp, 1),
           "assemble_us": round(ta, 1), "Mtets_per_s_assemble": round(m.nme / ta, 1),
           "Mtets_per_s_total": round(m.nme / (tp + ta), 1),
           "assemble_alg_bytes": alg, "assemble_alg_GBps": round(alg / (ta * 1e-6) / 1e9, 1),
           "assemble_us_unrelabelled": None if ta_o is None else round(ta_o, 1)}
    log(f"[bench] tet cube128 nme={m.nme}: pattern {tp:.0f}us, mass+stiffness {ta:.0f}us "
        f"({m.nme / ta:.0f} Mtets/s); unrelabelled mass+stiffness "
        + ("skipped" if ta_o is None else f"{ta_o:.0f}us"))
    return out


def run_p2(torch, fem, args):
    """P2 triangles on the 2048^2-cell unit square of the headline workload:
    edge numbering, pattern over nq + ne DOFs, fused mass + stiffness."""
    from paper_1305_3122_amd import meshgen as mg
    lib = fem._lib.load()
    dev = torch.device("cuda:0")
    m = mg.config_mesh(2)
    me = torch.from_numpy(m.me).to(dev)
    q = torch.from_numpy(m.q).to(dev)
    s = torch.cuda.current_stream().cuda_stream
    i32 = dict(dtype=torch.int32, device=dev)
    ws = C.c_size_t(0)
    fem._lib.check(lib.fem_p2_dofs_workspace(m.nq, m.nme, C.byref(ws)))
    dwork = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
    dofs = torch.empty((m.nme, 6), **i32)
    edges = torch.empty((3 * m.nme, 2), **i32)
    ne = C.c_int64(0)

    def dofs_call():
        fem._lib.check(lib.fem_p2_dofs(m.nq, m.nme, me.data_ptr(), dofs.data_ptr(), edges.data_ptr(),
                                       3 * m.nme, dwork.data_ptr(), int(ws.value), C.byref(ne), s))

    dofs_call()
    ndof = m.nq + int(ne.value)
    pw = C.c_size_t(0)
    fem._lib.check(lib.fem_p2_pattern_workspace(ndof, m.nme, C.byref(pw)))
    pwork = torch.empty(int(pw.value), dtype=torch.uint8, device=dev)
    cap = ndof + 30 * m.nme
    row_ptr = torch.empty(ndof + 1, **i32)
    col = torch.empty(cap, **i32)
    inc_ptr = torch.empty(ndof + 1, **i32)
    inc = torch.empty(6 * m.nme, **i32)
    inc_pos = torch.empty(6 * m.nme, dtype=torch.int64, device=dev)
    nnz = C.c_int64(0)

    def pattern():
        fem._lib.check(lib.fem_p2_pattern(ndof, m.nme, dofs.data_ptr(), row_ptr.data_ptr(), col.data_ptr(),
                                          cap, inc_ptr.data_ptr(), inc.data_ptr(), inc_pos.data_ptr(),
                                          pwork.data_ptr(), int(pw.value), C.byref(nnz), s))

    pattern()
    k = int(nnz.value)
    ops = fem.FEM_OP_MASS | fem.FEM_OP_STIFF
    aw = C.c_size_t(0)
    fem._lib.check(lib.fem_p2_assemble_workspace(m.nme, C.byref(aw)))
    awork = torch.empty(int(aw.value), dtype=torch.uint8, device=dev)
    M = torch.empty(k, dtype=torch.float64, device=dev)
    S = torch.empty_like(M)

    def assemble():
        fem._lib.check(lib.fem_p2_assemble(ops, m.nq, m.nme, ndof, k, q.data_ptr(), me.data_ptr(),
                                           row_ptr.data_ptr(), inc_ptr.data_ptr(), inc.data_ptr(),
                                           inc_pos.data_ptr(), M.data_ptr(), S.data_ptr(),
                                           awork.data_ptr(), awork.numel(), 0, s))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            ea = torch.cuda.Event(enable_timing=True)
            eb = torch.cuda.Event(enable_timing=True)
            ea.record()
            fn()
            eb.record()
            torch.cuda.synchronize()
            out.append(ea.elapsed_time(eb) * 1e3)
        return float(np.median(out))

    pattern()       # re-run once so that every buffer is touched before timing
    torch.cuda.synchronize()
    td = timed(dofs_call, 3)
    tp = timed(pattern, 3)
    ta = timed(assemble, 10)
    # inputs once (me, q), outputs once (two value arrays)
    alg = 12 * m.nme + 16 * m.nq + 16 * k
    # plus what the row design reads: row_ptr and inc_ptr (8 per DOF), inc and
    # inc_pos (12 per incidence, 72 per triangle), the four numbers per
    # triangle (written once, read back once per incidence: 6 x 32 B)
    design = alg + 8 * ndof + 72 * m.nme + 32 * m.nme + 6 * 32 * m.nme
    out = {"workload": "unit square 2048x2048 cells (8.4M triangles, jitter 0.2h, random relabelling); "
                       "P2 Lagrange, DOFs = vertices + edges; mass + stiffness FP64",
           "nq": m.nq, "ne": int(ne.value), "ndof": ndof, "nme": m.nme, "nnz": k,
           "dofs_us": round(td, 1), "pattern_us": round(tp, 1), "assemble_us": round(ta, 1),
           "Mtri_per_s_assemble": round(m.nme / ta, 1),
           "Mtri_per_s_total": round(m.nme / (td + tp + ta), 1),
           "assemble_alg_bytes": alg, "assemble_alg_GBps": round(alg / (ta * 1e-6) / 1e9, 1),
           "assemble_design_bytes": design,
           "assemble_design_GBps": round(design / (ta * 1e-6) / 1e9, 1)}
    log(f"[bench] p2 square2048 nme={m.nme} ndof={ndof} nnz={k}: dofs {td:.0f}us, pattern {tp:.0f}us, "
        f"mass+stiffness {ta:.0f}us ({m.nme / ta:.0f} Mtri/s)")
    return out


def run_cpu_baseline(args, m):
    """The oracle, as it stands, on the step's mesh (the 2048 x 2048 square):
    (i) the full assembly of stiffness + mass, the paper's OptV2 scope
    (pattern from the triangles, then both value arrays), single-threaded,
    median of 3; (ii) the oracle's numeric phase alone given that pattern,
    median of 5; (iii) the numeric phase on every host core (OpenMP over the
    rows, a separate C file beside the oracle), median of 5."""
    import oracle
    from oracle import cpu_baseline as cb

    def full():
        P = oracle.pattern(m.nq, m.me)
        oracle.assemble("stiff", m.q, m.me, P.slot, P.nnz)
        oracle.assemble("mass", m.q, m.me, P.slot, P.nnz)
        return P

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts

    t_full, ts_full = timed(full, args.cpu_reps_full)
    P = oracle.pattern(m.nq, m.me)
    t_num, _ = timed(lambda: (oracle.assemble("stiff", m.q, m.me, P.slot, P.nnz),
                              oracle.assemble("mass", m.q, m.me, P.slot, P.nnz)), 5)
    S = np.empty(P.nnz)
    M = np.empty(P.nnz)
    cb.stiff_mass_rows(m.q, m.me, P, S, M)
    t_omp, _ = timed(lambda: cb.stiff_mass_rows(m.q, m.me, P, S, M), 5)
    cores = cb.threads()
    log(f"[bench] cpu oracle square2048: full S+M {t_full:.2f}s, numeric {t_num:.2f}s, "
        f"numeric on {cores} threads {t_omp:.3f}s")
    return {"value": round(m.nme / t_full / 1e6, 4), "unit": "Mtri/s", "cores": 1, "kind": "oracle",
            "sample": f"the step's mesh (2048x2048 cells, {m.nme} triangles): stiffness + mass "
                      f"assembled from the triangles (pattern, then both value arrays; the OptV2 "
                      f"scope) by the single-threaded C oracle (-O2 -ffp-contract=off), median of "
                      f"{len(ts_full)} runs ({', '.join(f'{t:.2f}' for t in ts_full)} s)",
            "numeric_only": {"value": round(m.nme / t_num / 1e6, 4), "unit": "Mtri/s", "cores": 1,
                             "seconds": round(t_num, 3),
                             "sample": "the oracle's S + M values given its pattern, median of 5"},
            "all_cores": {"value": round(m.nme / t_omp / 1e6, 4), "unit": "Mtri/s", "cores": cores,
                          "cpu_count": os.cpu_count(), "seconds": round(t_omp, 4),
                          "sample": "S + M values given the oracle's pattern, OpenMP over the rows "
                                    "(oracle/cpu_rows_omp.c, not the oracle), median of 5"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-reps-full", type=int, default=3)
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for counter scaling)")
    ap.add_argument("--summarize", nargs=3, metavar=("KT", "PF", "PW"),
                    help="write the profiles/ summaries from rocprofv3 csv directories")
    ap.add_argument("--command", default="",
                    help="command text recorded by --summarize (default: that of the profile)")
    ap.add_argument("--profile-name", default="step_square2048", choices=sorted(PROFILE_TITLES),
                    help="which summary --summarize writes")
    ap.add_argument("--no-local", action="store_true",
                    help="tetrahedra: skip the unrelabelled cube (profiles of the relabelled one)")
    ap.add_argument("--only", choices=("sparse", "adjoint", "batched", "tet", "p2"),
                    help="run one of the extra measurements alone and print its JSON (profiling)")
    args = ap.parse_args()
    if args.summarize:
        summarize_profiles(*args.summarize, args.command, args.profile_name)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the assembly of one mesh runs on one GPU, and no "
              "multi-GPU split is implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_1305_3122_amd as fem
    if args.calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy of 1 GiB done")
        del src, dst
    if args.only:
        fn = {"sparse": run_sparse, "adjoint": run_adjoint, "batched": run_batched,
              "tet": run_tet, "p2": run_p2}[args.only]
        print(json.dumps({args.only: fn(torch, fem, args)}), flush=True)
        return
    m, st, ms, kern = run_main(torch, fem, args)
    extras = {"gather_floor": run_gather_floor(torch, fem, st, args.steps)}
    if not args.no_extras:
        extras["roofline_local"] = run_local(torch, fem, args)
        extras["batched"] = run_batched(torch, fem, args)
        extras["adjoint"] = run_adjoint(torch, fem, args)
        extras["sparse"] = run_sparse(torch, fem, args)
        extras["tet"] = run_tet(torch, fem, args)
        extras["p2"] = run_p2(torch, fem, args)
    traffic = read_traffic()

    def roof(p):
        k = kern[p]
        name = CALL_KERNEL[p]
        r = {"kernel": name, "call": p, "bound": "hbm", "achieved": k["alg_GBps"],
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(k["alg_GBps"] / HBM_PEAK_GBS, 4),
             "traffic": None, "alg_bytes": k["alg_bytes"], "us": k["us"]}
        if name in traffic:
            fb, wb = traffic[name]
            r["traffic"] = int(round(fb + wb))
            r["traffic_fetch"] = int(round(fb))
            r["traffic_write"] = int(round(wb))
            r["traffic_GBps"] = round((fb + wb) / (k["us"] * 1e-6) / 1e9, 1)
            r["traffic_kind"] = ("L2 fetch + write bytes (FETCH_SIZE, WRITE_SIZE, copy-calibrated); "
                                 "the fetches of random gathers are mostly served by the MALL, "
                                 "so this is L2-miss line traffic, not HBM traffic")
        return r

    line = {
        "metric": METRIC,
        "value": round(m.nme / (ms * 1e-3) / 1e6, 2),
        "unit": "Mtri/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "unit square 2048x2048 cells (jitter 0.2h, random vertex relabelling), "
                               "full assembly: pattern + one pass for M, Mw (w=1+x^2+y^2), S and "
                               "elasticity K (lambda=1, mu=0.5) + elasticity pattern; FP64 "
                               "values, int32 indices",
                   "nq": m.nq, "nme": m.nme, "nnz": st.nnz},
        # the longest single kernel of the step: the pass for all four
        # operators, timed alone on its packed records
        "roofline": roof("assemble_rows"),
        # the metric's K+M: stiffness and mass in one fused kernel
        "roofline_stiff_mass": roof("stiff_mass"),
        # measured practical ceiling: a plain 1 GiB device-to-device copy
        "stream_copy_GBps": st.copy_gbs,
        "kernels": kern,
    }
    line.update(extras)
    if not args.no_cpu:
        line["cpu_baseline"] = run_cpu_baseline(args, m)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
