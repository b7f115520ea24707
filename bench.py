"""Benchmark of the WCSPH / k-epsilon open-boundary step on one MI355X.

One "step" is one advection step of the whole per-step pipeline: cell-list
build, correction matrix, dual-criteria advection step (ARD / RANS pass and
the acoustic pressure / density sub-steps) and the bidirectional buffer
update.  Inputs are synthetic and resident in HBM before timing starts.

Prints ONE JSON line (rank 0) with particle-steps/s, neighbour pairs/s,
the FP64-path figures, the roofline of the dominant kernel (HIP events on
the library's stream over the timed region) and the CPU oracle baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
VALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # MI355X vector peaks, published
PROFILE_EVERY = 10        # steps between two event-timed steps

# Algorithmic cost of one launch of a neighbour pass: each particle's own
# input fields read once and its outputs written once (neighbour re-reads
# that the caches serve are not counted), bytes per particle as
# (FP32-mixed, FP64); and flops per directed pair within 2h (an FMA is 2,
# a square root 1), (2D, 3D).  The k-epsilon advection pass adds 20 bytes
# and 20 flops.
ALGO_BYTES = {("correction", 2): (60, 68), ("correction", 3): (104, 108),
              ("advection", 2): (64, 115), ("advection", 3): (96, 175),
              ("pressure", 2): (52, 100), ("pressure", 3): (76, 148),
              ("density", 2): (80, 108), ("density", 3): (104, 140)}
FLOPS_PER_PAIR = {"correction": (22, 32), "advection": (35, 55), "pressure": (32, 50),
                  "density": (26, 32)}

WORKLOADS = {
    # name: (generator, kwargs, label)
    "uchannel": ("make_uchannel", {}, "2D U-channel, dp=H/40, ~50k fluid particles, Re=50"),
    "channel": ("make_channel", {}, "2D straight channel 10Hx1H, dp=H/20, 4k fluid, Re=100"),
    "jet": ("make_jet", {}, "2D turbulent plane jet 20Dx20D, dp=D/20, 160k, k-eps"),
    "mixer": ("make_mixer", {}, "3D self-rotating micro-mixer: chamber 1 x 0.5, four "
              "tangential 0.1 x 0.1 inlets, axial outlet of diameter 0.2, dp=0.005, "
              "3.29M fluid + 0.46M wall particles, Re=50, FP32-mixed"),
    "adjoint_channel": ("make_adjoint_channel", {}, "2D channel 20Hx1H, dp=H/80, 128k"),
    "jet_640k": ("make_jet", {"dp": 0.025}, "2D jet geometry at dp=D/40, 640k"),
    "jet_2560k": ("make_jet", {"dp": 0.0125}, "2D jet geometry at dp=D/80, 2.56M"),
    "jet_10m": ("make_jet", {"dp": 0.00625}, "2D jet geometry at dp=D/160, 10.2M"),
}


# one-core oracle sample of a workload whose full step takes minutes on one
# core: the same geometry at a coarser spacing
CPU_SMALL = {"mixer": ("make_mixer", {"dp": 0.0125}, "the mixer geometry at dp = 0.0125")}
SWEEP = ("uchannel", "jet", "jet_640k", "jet_2560k")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixer", choices=sorted(WORKLOADS))
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the extra workloads (U-channel and the jet sizes)")
    ap.add_argument("--sweep-steps", type=int, default=50)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fp64-steps", type=int, default=0, help="steps of the FP64 run (0: --steps)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device to device 5 times (HBM counter "
                         "calibration under rocprofv3) and exit")
    ap.add_argument("--laminar-jet", action="store_true",
                    help="laminar plane jet (Re 40) against the closed-form jet; prints one JSON line")
    ap.add_argument("--jet-precision", type=int, default=1, choices=(0, 1),
                    help="--laminar-jet arithmetic: 0 FP64, 1 FP32-mixed")
    ap.add_argument("--jet-nf", type=int, default=20,
                    help="--laminar-jet particles across the slot (N_f)")
    ap.add_argument("--jet-steps", type=int, default=30000,
                    help="advection steps of --laminar-jet (the mean is over the last quarter, "
                         "at most 5000)")
    ap.add_argument("--config-run", choices=("jet", "uchannel_pressure", "mixer"),
                    help="run a configured workload for its stated steps in FP32-mixed and "
                         "FP64 (transport-velocity shift --tvf-alpha) and print one JSON line")
    ap.add_argument("--tvf-alpha", type=float, default=0.2)
    ap.add_argument("--p-far", type=float, default=0.0,
                    help="--config-run jet: pressure of the outlet and far-field buffers")
    ap.add_argument("--config-steps", type=int, default=0, help="--config-run steps (0: stated)")
    ap.add_argument("--obc-ablation", action="store_true",
                    help="only run the open-boundary ablation of Table 2 (Cases 1-4) on the "
                         "laminar channel and print its JSON line")
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--adjoint-checkpoint", type=int, default=10)
    ap.add_argument("--summarize-stats", nargs=3, metavar=("DIR", "OUT_MD", "COMMAND"),
                    help="write the Markdown table of a rocprofv3 --stats output directory "
                         "(COMMAND: the command that produced it) and exit; no GPU needed")
    ap.add_argument("--summarize-traffic", nargs=4,
                    metavar=("COPY_FETCH", "COPY_WRITE", "RUN_FETCH", "RUN_WRITE"),
                    help="fold four rocprofv3 --pmc output directories (FETCH_SIZE and "
                         "WRITE_SIZE of the copy calibration, then of a bench run of "
                         "--workload) into profiles/hbm_traffic.json and a Markdown table; "
                         "no GPU needed")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# rocprofv3 output summaries (profiles/)
# ---------------------------------------------------------------------------
def _kernel_label(name):
    import re
    n = re.sub(r"^void ", "", name)
    n = re.sub(r"^sphx::(\(anonymous namespace\)::)?", "", n)
    depth, out = 0, []
    for ch in n:                       # drop the argument list, keep template args
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


def _one_csv(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def summarize_stats(d, out_md, command):
    import csv
    rows = list(csv.DictReader(open(_one_csv(d, "kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"Command (repository root, one MI355X):", "", "```", command, "```", "",
             "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{_kernel_label(r['Name'])}` | {int(r['Calls'])} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    head = open(out_md).read().split("Command (repository root")[0] if os.path.exists(out_md) else ""
    with open(out_md, "w") as fh:
        fh.write(head + "\n".join(lines) + "\n")
    print(f"wrote {out_md}")


def _counter_per_kernel(d, counter):
    """Mean per dispatch of `counter` over the second half of each kernel's
    dispatches (the first half includes the warm-up's ramp)."""
    import csv
    per = {}
    for r in csv.DictReader(open(_one_csv(d, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        per.setdefault(_kernel_label(r["Kernel_Name"]), []).append(
            (int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    out = {}
    for k, v in per.items():
        v.sort()
        half = [x for _, x in v[len(v) // 2:]]
        out[k] = (sum(half) / len(half), max(x for _, x in v))
    return out


def summarize_traffic(args, cf, cw, bf, bw):
    copy_bytes = 256 * (1 << 20)
    fetch_copy = max(m for _, m in _counter_per_kernel(cf, "FETCH_SIZE").values())
    write_copy = max(m for _, m in _counter_per_kernel(cw, "WRITE_SIZE").values())
    fs = copy_bytes / 1024 / fetch_copy
    ws = copy_bytes / 1024 / write_copy
    fetch = _counter_per_kernel(bf, "FETCH_SIZE")
    write = _counter_per_kernel(bw, "WRITE_SIZE")
    names = {"k_pressure": "pressure", "k_density": "density", "k_advection": "advection",
             "k_correction": "correction"}
    kernels, rows = {}, []
    for label in sorted(fetch):
        base = label.split("<")[0]
        if base not in names or label not in write:
            continue
        f, w = fetch[label][0], write[label][0]
        b = int(round((f * fs + w * ws) * 1024))
        kernels[f"{args.workload}/fp32/{names[base]}"] = {
            "kernel": label, "FETCH_SIZE_KiB": round(f, 1), "WRITE_SIZE_KiB": round(w, 1),
            "bytes_per_launch": b}
        rows.append(f"| `{label}` | {f:.1f} | {w:.1f} | {b:,} |")
    run = (f"python bench.py --workload {args.workload} --steps {args.steps} --warmup "
           f"{args.warmup} --no-cpu --no-fp64 --no-adjoint --no-sweep")
    cmds = [f"rocprofv3 --pmc FETCH_SIZE -d {cf} -o cf --output-format csv -- python bench.py --calibrate-copy 256",
            f"rocprofv3 --pmc WRITE_SIZE -d {cw} -o cw --output-format csv -- python bench.py --calibrate-copy 256",
            f"rocprofv3 --pmc FETCH_SIZE -d {bf} -o bf --output-format csv -- {run}",
            f"rocprofv3 --pmc WRITE_SIZE -d {bw} -o bw --output-format csv -- {run}"]
    rec = {"description": "HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB "
                          "per dispatch), each scaled by its reading for a device-to-device copy "
                          "of 256 MiB; mean over the second half of each kernel's launches",
           "source_hash": kernel_source_hash(),
           "calibration": {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB_per_copy": fetch_copy,
                           "WRITE_SIZE_KiB_per_copy": write_copy, "fetch_scale": round(fs, 5),
                           "write_scale": round(ws, 5)},
           "commands": cmds, "kernels": kernels, "hashed_sources": list(TRAFFIC_SOURCES)}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if os.path.exists(path):   # keep the other workloads' figures of the same sources
        with open(path) as fh:
            old = json.load(fh)
        if old.get("source_hash") == rec["source_hash"]:
            merged = dict(old.get("kernels", {}))
            merged.update(kernels)
            rec["kernels"] = merged
            rec["commands_by_workload"] = dict(old.get("commands_by_workload", {}))
    rec.setdefault("commands_by_workload", {})[args.workload] = cmds
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    md = os.path.join(ROOT, "profiles", f"hbm_traffic_{args.workload}_fp32.md")
    with open(md, "w") as fh:
        fh.write(f"# HBM traffic per launch: {args.workload} workload, FP32-mixed (rocprofv3 counters)\n\n"
                 "FETCH_SIZE and WRITE_SIZE in separate runs, each scaled by the same counter's "
                 "reading for a plain device-to-device copy of 256 MiB (`bench.py "
                 f"--calibrate-copy 256`): FETCH_SIZE reads {fetch_copy:.0f} KiB per copy of "
                 f"{copy_bytes // 1024} KiB (scale {fs:.4f}), WRITE_SIZE reads {write_copy:.0f} KiB "
                 f"(scale {ws:.4f}).  Mean per launch over the second half of each kernel's "
                 "launches.\n\nCommands (repository root, one MI355X), then "
                 "`python bench.py --workload " + args.workload + f" --steps {args.steps} --warmup "
                 f"{args.warmup} --summarize-traffic {cf} {cw} {bf} {bw}`:\n\n```\n" + "\n".join(cmds) + "\n```\n\n"
                 "| kernel | FETCH KiB | WRITE KiB | HBM bytes per launch (scaled) |\n"
                 "|---|---:|---:|---:|\n" + "\n".join(rows) + "\n\n"
                 f"Digest of the neighbour-pass sources (`kernel_source_hash`: "
                 f"{', '.join(TRAFFIC_SOURCES)}): `{rec['source_hash']}`; bench.py reports the "
                 "figure of its dominant kernel as `roofline.traffic` only while the digest "
                 "matches.\n")
    print(f"wrote {path} and {md}")


def make_case(name):
    import cases
    gen, kw, _ = WORKLOADS[name]
    return getattr(cases, gen)(**kw)


def run_gpu(case, precision, steps, warmup, torch):
    from paper_2510_25702_amd import sph
    g = sph.Simulation(case, precision=precision)
    g.build_cells()
    g.buffer_update()                  # label the particles that start in buffers
    for _ in range(warmup):
        g.advance()
    torch.cuda.synchronize()
    g.pair_count()                     # reset the pair counter
    n_real0 = sph.sph_get_count(g.ctx)[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_ac = 0
    real_steps = 0
    outgrown = 0
    for i in range(steps):
        # HIP events around every kernel of one step in PROFILE_EVERY (the
        # event records cost host time; the sampled launches give the
        # per-kernel averages)
        g.profile(i % PROFILE_EVERY == 0)
        info, cnt = g.advance()
        n_ac += info.n_ac
        real_steps += cnt.n_real
        outgrown += info.list_outgrown > 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.profile(False)
    pairs = g.pair_count()
    stats = g.kernel_stats()
    dt = t1 - t0
    return dict(seconds=dt, particle_steps=real_steps, n_real=n_real0, pairs=pairs,
                n_ac=n_ac, stats=stats, sim=g, outgrown=outgrown)


def obc_ablation(steps=3000, navg=1000, precision=0):
    """The open-boundary ablation of Table 2 (Cases 1-4 = obc_mode 1-4) on a
    laminar straight channel with the paper's ratios: 20 particles across,
    Re = 50 on the bulk velocity, parabolic inlet, outlet pressure equal to
    the channel's Poiseuille pressure drop (the paper: 0.1 and 0.1), started
    from the developed state.  Over the last `navg` steps (every fifth) it
    averages the centre-line pressure, fitted over the interior (slope and
    inlet value against the Poiseuille ones) and the velocity profile of the
    last H before the outlet buffer (normwise L2 against the parabola)."""
    import numpy as np
    import cases
    from paper_2510_25702_amd import sph
    H, L, dp, Re, Um, c0 = 1.0, 6.0, 0.05, 50.0, 1.0, 10.0
    nu = (2.0 / 3.0) * Um * H / Re
    grad = 8.0 * nu * Um / H ** 2            # -dp/dx of the Poiseuille flow, rho0 = 1
    p_out = grad * L
    out = {"setup": f"{L}Hx{H} channel, dp = H/{round(H / dp)}, Re {Re:g}, c0 = {c0:g} U_max, "
                    f"p_out = {p_out:.3f} = the Poiseuille drop, {steps} steps, mean of the "
                    f"last {navg}", "p_inlet_theory": p_out + grad * L, "slope_theory": -grad}
    for mode in (1, 2, 3, 4):
        c = cases.make_channel(H=H, L=L, dp=dp, Re=Re, Umax=Um, c0=c0, ramp_time=0.0,
                               p_out=p_out, obc_mode=mode)
        fl = (c.tag & 3) != cases.WALL
        y = c.x[:, 1]
        c.v = c.v.copy()
        c.v[fl, 0] = 4 * Um * (y[fl] / H) * (1 - y[fl] / H)
        c.rho = c.rho.copy()
        c.rho[fl] = 1.0 + (p_out + grad * (L - c.x[fl, 0])) / c0 ** 2
        g = sph.Simulation(c, precision=precision)
        g.build_cells()
        g.buffer_update()
        nb, nx = int(round(H / dp)), int(round(L / (2 * dp)))
        au, nu_, ap, np_ = np.zeros(nb), np.zeros(nb), np.zeros(nx), np.zeros(nx)
        t0 = time.perf_counter()
        for k in range(steps):
            g.advance()
            if k < steps - navg or k % 5:
                continue
            st = g.state()
            x, v = st["x"], st["v"]
            real = (st["tag"] & 3) <= 1
            p = c0 ** 2 * (st["rho"] - 1.0)
            sel = real & (x[:, 0] > L - 4 * dp - H) & (x[:, 0] < L - 4 * dp - 0.5 * H)
            b = np.clip((x[sel, 1] / dp).astype(int), 0, nb - 1)
            np.add.at(au, b, v[sel, 0])
            np.add.at(nu_, b, 1)
            sel = real & (np.abs(x[:, 1] - H / 2) < 2 * dp)
            b = np.clip((x[sel, 0] / (2 * dp)).astype(int), 0, nx - 1)
            np.add.at(ap, b, p[sel])
            np.add.at(np_, b, 1)
        secs = time.perf_counter() - t0
        u = au / np.maximum(nu_, 1)
        yy = (np.arange(nb) + 0.5) * dp
        ua = 4 * Um * yy * (1 - yy)
        xc = (np.arange(nx) + 0.5) * 2 * dp
        m = (np_ > 0) & (xc > 4 * dp + 0.5) & (xc < L - 4 * dp - 0.5)
        slope, icpt = np.polyfit(xc[m], (ap / np.maximum(np_, 1))[m], 1)
        out[f"case{mode}"] = {
            "slope_rel_err": round(float(slope / -grad - 1.0), 4),
            "p_inlet_rel_err": round(float(icpt / (p_out + grad * L) - 1.0), 4),
            "outlet_u_L2": round(float(np.sqrt(np.mean((u - ua) ** 2) / np.mean(ua ** 2))), 4),
            "seconds": round(secs, 2)}
    return out


def laminar_jet(steps=20000, navg=5000, precision=1, nf=10, p_far=0.0):
    """The laminar plane jet of Sec. 4.3 (Re 40, slot D = 2, 40 D x 40 D, nf
    particles across the slot, six buffers of Table 3, transport-velocity
    shift on) against the closed-form plane laminar jet: centre-line speed
    u_c = 0.4543 (K^2 / (nu x))^(1/3) and half-width b = 3.2028 (nu^2 / K)^(1/3)
    x^(2/3) (u = u_c sech^2(0.8814 y / b)), K = U^2 D the momentum flux of the
    slot, x from a virtual origin.  The virtual origin is not fixed, so the
    checks are on slopes: u_c^-3 and b^(3/2) are linear in x with the stated
    slopes, and the profiles u / u_c against y / b collapse onto sech^2.
    Means over the last `navg` steps (every tenth), stations every D from
    10 D to 32 D."""
    import numpy as np
    import cases
    from paper_2510_25702_amd import sph
    c = cases.make_laminar_jet(nf=nf, p_far=p_far)
    D, U, Re = 2.0, 1.0, 40.0
    nu, K, dp, W = U * D / Re, U * U * D, D / nf, 40.0
    g = sph.Simulation(c, precision=precision)
    g.build_cells()
    g.buffer_update()
    xs = np.arange(10, 33) * D
    ny = int(round(2 * W / dp))
    acc, cnt = np.zeros((len(xs), ny)), np.zeros((len(xs), ny))
    ids = [b.id for b in c.buffers]
    inj, dele = np.zeros(len(ids), np.int64), np.zeros(len(ids), np.int64)
    n_real0 = sph.sph_get_count(g.ctx)[1]
    t0 = time.perf_counter()
    for k in range(steps):
        try:
            _, cn = g.advance()
        except sph.SphError as e:
            st = g.state()
            real = (st["tag"] & 3) <= 1
            return {"setup": f"Re {Re:g}, D {D:g}, 40Dx40D, N_f {nf}, {c.x.shape[0]} particles, "
                             f"tvf_alpha {c.params['tvf_alpha']}",
                    "failed_at_step": k + 1, "t": round(sph.sph_get_clock(g.ctx)[1], 3),
                    "error": str(e), "real_particles": [int(n_real0), int(real.sum())],
                    "buffers": {str(b): {"injected": int(i), "deleted": int(d)}
                                for b, i, d in zip(ids, inj, dele)},
                    "seconds": round(time.perf_counter() - t0, 1)}
        for q, b in enumerate(ids):
            inj[q] += cn.n_inject[b]
            dele[q] += cn.n_delete[b]
        if (k + 1) % 4000 == 0:
            print(f"laminar jet: step {k + 1} of {steps}, real particles "
                  f"{sph.sph_get_count(g.ctx)[1]}", file=sys.stderr, flush=True)
        if k < steps - navg or k % 10:
            continue
        st = g.state()
        x, v = st["x"], st["v"]
        real = (st["tag"] & 3) <= 1
        for q, x0 in enumerate(xs):
            sel = real & (np.abs(x[:, 0] - x0) < dp)
            b = np.clip(((x[sel, 1] + W) / dp).astype(int), 0, ny - 1)
            np.add.at(acc[q], b, v[sel, 0])
            np.add.at(cnt[q], b, 1)
    secs = time.perf_counter() - t0
    head = {"setup": f"Re {Re:g}, D {D:g}, 40Dx40D, N_f {nf}, {c.x.shape[0]} particles, "
                     f"tvf_alpha {c.params['tvf_alpha']}, far-field p {p_far:g}, {steps} steps (t = "
                     f"{sph.sph_get_clock(g.ctx)[1]:.0f}), mean of the last {navg}",
            "ms_per_step": round(1e3 * secs / max(steps, 1), 4),
            "real_particles": [int(n_real0), int(sph.sph_get_count(g.ctx)[1])],
            "buffers": {str(b): {"injected": int(i), "deleted": int(d)}
                        for b, i, d in zip(ids, inj, dele)}}
    u = acc / np.maximum(cnt, 1)
    yc = -W + (np.arange(ny) + 0.5) * dp
    uc = u[:, np.abs(yc) < dp].mean(axis=1)
    if not np.all(uc > 0.05):   # the jet has not reached every station yet
        return dict(head, note="jet not developed over the stations; no similarity figures")
    half = []
    for q in range(len(xs)):
        prof, up = u[q], yc > 0
        above = np.where(up & (prof < 0.5 * uc[q]))[0]
        j = above[0]                     # first bin above the centre line below u_c / 2
        y0, y1, f0, f1 = yc[j - 1], yc[j], prof[j - 1], prof[j]
        bp = y0 + (0.5 * uc[q] - f0) * (y1 - y0) / (f1 - f0)
        below = np.where(~up & (prof < 0.5 * uc[q]))[0]
        j = below[-1]
        y0, y1, f0, f1 = yc[j], yc[j + 1], prof[j], prof[j + 1]
        bm = y0 + (0.5 * uc[q] - f0) * (y1 - y0) / (f1 - f0)
        half.append(0.5 * (bp - bm))
    half = np.array(half)
    s_u, i_u = np.polyfit(xs, uc ** -3, 1)
    s_b, i_b = np.polyfit(xs, half ** 1.5, 1)
    th_u = nu / (0.4543 ** 3 * K * K)
    th_b = (3.2028 * (nu * nu / K) ** (1.0 / 3.0)) ** 1.5
    eta = yc[None, :] / half[:, None]
    m = np.abs(eta) < 2.5
    coll = u / uc[:, None]
    prof = 1.0 / np.cosh(0.8814 * eta) ** 2
    l2 = float(np.sqrt(np.mean((coll - prof)[m] ** 2) / np.mean(prof[m] ** 2)))
    mom = (u ** 2).sum(axis=1) * dp
    return {**head,
            "uc_m3_slope_rel_err": round(float(s_u / th_u - 1.0), 4),
            "uc_m3_corr": round(float(np.corrcoef(xs, uc ** -3)[0, 1]), 5),
            "uc_virtual_origin": round(float(-i_u / s_u), 2),
            "b_1p5_slope_rel_err": round(float(s_b / th_b - 1.0), 4),
            "b_1p5_corr": round(float(np.corrcoef(xs, half ** 1.5)[0, 1]), 5),
            "b_virtual_origin": round(float(-i_b / s_b), 2),
            "profile_collapse_L2": round(l2, 4),
            "momentum_flux_over_K": [round(float(mom[0] / K), 3), round(float(mom[-1] / K), 3)],
            "uc": [round(float(a), 4) for a in uc[::4]],
            "b": [round(float(a), 3) for a in half[::4]],
            "x": [float(a) for a in xs[::4]],
            "seconds": round(secs, 1)}


CONFIG_RUNS = {
    # name: (case builder taking the shift coefficient, configured steps, bin box, label)
    "jet": (lambda a, pf=0.0: cases_mod().make_jet(tvf_alpha=a, p_far=pf), 5000,
            ((0.0, 20.0), (-10.0, 10.0)),
            "2D turbulent plane jet, k-eps, 160k particles, Re 1e4, six buffers, 5000 steps"),
    "mixer": (lambda a, pf=0.0: cases_mod().make_mixer(), 500, ((-0.55, 0.55), (-0.55, 0.55)),
              "3D micro-mixer, 3.75M particles, Re 50, 500 steps (fields binned in x-y)"),
    "uchannel_pressure": (lambda a, pf=0.0: cases_mod().make_uchannel(inlet="pressure",
                                                                        tvf_alpha=a),
                          2000, ((0.0, 17.3), (0.0, 4.0)),
                          "2D U-channel, p = 1 pressure inlet, p = 0 outlet, Re 50, 2000 steps"),
}


def config_run(name, alpha, steps, torch, nbins=40, navg=1000, p_far=0.0):
    """A configured workload run for its stated number of steps in FP32-mixed
    and in FP64 on the GPU, each stopping at the first numerical error.  The
    real particles' velocity, pressure (and k, epsilon) are averaged on a
    nbins x nbins grid over the last `navg` steps (every tenth step); the
    FP32-mixed run's binned fields are compared with the FP64 run's (relative
    L2 over the bins both runs fill)."""
    import numpy as np
    from paper_2510_25702_amd import sph
    make, nsteps, box, label = CONFIG_RUNS[name]
    steps = steps or nsteps
    navg = min(navg, steps // 2)
    out = {"workload": name, "description": label, "tvf_alpha": alpha, "steps": steps,
           "averaged_steps": navg, "p_far": p_far}
    fields = {}
    for prec, key in ((sph.SPH_FP32_MIXED, "fp32_mixed"), (sph.SPH_FP64, "fp64")):
        case = make(alpha, p_far)
        P = case.params
        out["tvf_alpha"] = float(P.get("tvf_alpha", 0.0))
        g = sph.Simulation(case, precision=prec)
        g.build_cells()
        g.buffer_update()
        n0 = sph.sph_get_count(g.ctx)[1]
        ids = [b.id for b in case.buffers]
        inj, dele = np.zeros(len(ids), np.int64), np.zeros(len(ids), np.int64)
        acc = {f: np.zeros((nbins, nbins)) for f in ("u", "v", "p", "k", "eps")}
        cnt = np.zeros((nbins, nbins))
        rec = {}
        t0 = time.perf_counter()
        for k in range(steps):
            try:
                _, cn = g.advance()
            except sph.SphError as e:
                rec["failed_at_step"] = k + 1
                rec["error"] = str(e)
                break
            for q, b in enumerate(ids):
                inj[q] += cn.n_inject[b]
                dele[q] += cn.n_delete[b]
            if k >= steps - navg and k % 10 == 0:
                st = g.state()
                real = (st["tag"] & 3) <= 1
                x, v = st["x"][real], st["v"][real]
                kk, ee, rho = st["k"][real], st["eps"][real], st["rho"][real]
                p = P["rho0"] * P["c0"] ** 2 * (rho / P["rho0"] - 1.0)
                if P["turbulence"]:
                    p = p + 2.0 / 3.0 * rho * kk
                ix = np.floor((x[:, 0] - box[0][0]) / (box[0][1] - box[0][0]) * nbins).astype(int)
                iy = np.floor((x[:, 1] - box[1][0]) / (box[1][1] - box[1][0]) * nbins).astype(int)
                ok = (ix >= 0) & (ix < nbins) & (iy >= 0) & (iy < nbins)
                for f, val in (("u", v[:, 0]), ("v", v[:, 1]), ("p", p), ("k", kk),
                               ("eps", ee)):
                    np.add.at(acc[f], (ix[ok], iy[ok]), val[ok])
                np.add.at(cnt, (ix[ok], iy[ok]), 1)
            if (k + 1) % 1000 == 0:
                print(f"{name} {key}: step {k + 1} of {steps}", file=sys.stderr, flush=True)
        secs = time.perf_counter() - t0
        step, t, _ = sph.sph_get_clock(g.ctx)
        st = g.state()
        real = (st["tag"] & 3) <= 1
        rec["final_max"] = {"speed": float(np.linalg.norm(st["v"][real], axis=1).max()),
                            "k": float(st["k"][real].max()), "eps": float(st["eps"][real].max()),
                            "rho_min": float(st["rho"][real].min()),
                            "rho_max": float(st["rho"][real].max())}
        if cnt.any():
            m = cnt > 0
            rec["binned_rms"] = {f: float(f"{np.sqrt(np.mean((a / np.maximum(cnt, 1))[m] ** 2)):.4g}")
                                 for f, a in acc.items()}
        rec.update(steps_done=int(step), t=round(float(t), 4), seconds=round(secs, 1),
                   real_particles=[int(n0), int(sph.sph_get_count(g.ctx)[1])],
                   buffers={str(b): {"injected": int(i), "deleted": int(d)}
                            for b, i, d in zip(ids, inj, dele)})
        out[key] = rec
        if "failed_at_step" not in rec:
            fields[key] = ({f: a / np.maximum(cnt, 1) for f, a in acc.items()}, cnt > 0)
        del g
    if len(fields) == 2:
        (a, ma), (b, mb) = fields["fp32_mixed"], fields["fp64"]
        m = ma & mb
        err = {}
        for f in ("u", "v", "p", "k", "eps"):
            den = float(np.sqrt(np.mean(b[f][m] ** 2)))
            if den > 0:
                err[f] = float(f"{np.sqrt(np.mean((a[f][m] - b[f][m]) ** 2)) / den:.3g}")
        out["fp32_vs_fp64_binned_fields"] = {"bins": f"{nbins}x{nbins}", "filled": int(m.sum()),
                                             "rel_L2": err}
    return out


def _state_case(g, case):
    import dataclasses
    from paper_2510_25702_amd import sph
    st = g.state()
    step, t, npid = sph.sph_get_clock(g.ctx)
    return dataclasses.replace(case, x=st["x"], v=st["v"], rho=st["rho"], drho=st["drho"],
                               k=st["k"], eps=st["eps"], tag=st["tag"], pid=st["pid"],
                               npid=int(npid), step=int(step), t=float(t))


def stated_error(r32, case, threads):
    """Stated error of each GPU path against the FP64 oracle on one state,
    the one the timed FP32-mixed run ended in: the pair operators (pressure
    and viscous accelerations, continuity rate, correction matrix; with
    turbulence the velocity gradient and the k, epsilon rates) of the
    FP32-mixed and the FP64 path, normwise (max |GPU - oracle| / max |oracle|),
    matched by particle id.  Up to 300k particles the oracle evaluates every
    particle; above, a sample of 96 fluid particles away from the buffers,
    each with everything within 4h + 2dp of it (its neighbours and theirs)."""
    import dataclasses
    import numpy as np
    import oracle
    from paper_2510_25702_amd import sph
    c = _state_case(r32["sim"], case)
    fields = ["ap", "anu", "drho", "B"]
    if case.params["turbulence"]:
        fields += ["gradv", "dk", "deps"]
    h, dp = c.params["h"], c.params["dp"]
    if c.n <= 300000:
        sub, picks = c, np.nonzero((c.tag & 3) != cases_mod().WALL)[0]
        sample = f"all {len(picks)} real particles"
    else:
        from scipy.spatial import cKDTree
        cm = cases_mod()
        far = np.ones(c.n, bool)
        for b in c.buffers:
            R = np.array(b.frame, float).reshape(3, 3)
            y = (c.x - np.array(b.origin, float)) @ R.T
            hw = list(b.half_width) + [0.0]
            inside = (y[:, 0] > -10 * h) & (y[:, 0] < b.length + b.fringe + 10 * h)
            for k in range(1, c.params["dim"]):
                inside &= np.abs(y[:, k]) < hw[k - 1] + 10 * h
            far &= ~inside
        cand = np.nonzero(((c.tag & 3) == cm.FLUID) & far)[0]
        picks = np.random.default_rng(5).choice(cand, 96, replace=False)
        near = np.unique(np.concatenate(cKDTree(c.x).query_ball_point(c.x[picks],
                                                                       4 * h + 2 * dp)))
        sub = dataclasses.replace(c, x=c.x[near].copy(), v=c.v[near].copy(),
                                  rho=c.rho[near].copy(), k=c.k[near].copy(),
                                  eps=c.eps[near].copy(), tag=c.tag[near].copy(),
                                  pid=c.pid[near].copy(), drho=c.drho[near].copy())
        sample = (f"96 fluid particles away from the buffers, the oracle on their "
                  f"{len(near)}-particle neighbourhoods")
    ref = oracle.OracleSim(sub, threads=threads)
    Bo, _ = ref.correction()
    ro = ref.rates(Bo)
    ro["B"] = Bo
    si = {int(p): i for i, p in enumerate(sub.pid)}
    io = np.array([si[int(c.pid[p])] for p in picks])
    out = {"state": f"end of the timed FP32-mixed run (step {c.step})", "sample": sample,
           "norm": "max |GPU - FP64 oracle| / max |FP64 oracle| per operator"}
    for prec, key in ((sph.SPH_FP32_MIXED, "fp32_mixed"), (sph.SPH_FP64, "fp64")):
        g = sph.Simulation(c, precision=prec)
        g.build_cells()
        g.correction()
        r = g.rates()
        gi = {int(p): i for i, p in enumerate(g.state()["pid"])}
        ig = np.array([gi[int(c.pid[p])] for p in picks])
        e = {}
        for f in fields:
            a, b = np.asarray(r[f])[ig], np.asarray(ro[f])[io]
            den = float(np.abs(b).max())
            e[f] = float(f"{np.abs(a - b).max() / den:.3g}") if den > 0 else 0.0
        out[key] = e
        del g
    return out


def cases_mod():
    import cases
    return cases


def walked_pairs(g):
    """Directed pairs within 2h that one pair pass visits at the current
    state (sph_step_pairs' count over the real particles)."""
    import ctypes as C
    from paper_2510_25702_amd import sph
    torch = g.torch
    row = torch.zeros(g.n + 1, dtype=torch.int32, device=g.device)
    n = C.c_int64()
    st = sph.lib().sph_step_pairs(g.ctx, C.c_void_p(row.data_ptr()), None, 0, C.byref(n))
    if st not in (sph.SPH_OK, sph.SPH_E_CAPACITY):
        raise sph.SphError(st, "sph_step_pairs")
    return int(n.value)


def roofline(stats, dim, prec, pairs_per_launch, n_slots, turb):
    """Roofline of the dominant neighbour pass (most kernel time per step):
    its algorithmic bytes per launch (bytes per particle x the particle
    slots one launch processes) and flops per launch (flops per pair x the
    directed pairs within 2h it visits), over its average launch duration
    (HIP events recorded by the launch at the kernel's start and end on the
    library's stream).  Bound: the VALU when the arithmetic intensity is
    above the ridge point (peak flops / 8 TB/s), else HBM; both fractions are
    given."""
    passes = ("pressure", "density", "advection", "correction")
    dom = max(passes, key=lambda k: stats[k].total_ms)
    s = stats[dom]
    avg_s = s.total_ms * 1e-3 / max(1, s.launches)
    pi = 0 if prec == "fp32" else 1
    bpp = ALGO_BYTES[(dom, dim)][pi] + (20 if (turb and dom == "advection") else 0)
    fpp = FLOPS_PER_PAIR[dom][0 if dim == 2 else 1] + (20 if (turb and dom == "advection") else 0)
    nbytes = bpp * n_slots
    flops = fpp * pairs_per_launch
    gbs = nbytes / avg_s / 1e9
    tfs = flops / avg_s / 1e12
    peak_f = VALU_PEAK_TFLOPS[prec]
    ai = flops / nbytes
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    hbm = dict(achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(gbs / HBM_PEAK_GBS, 4))
    alu = dict(achieved=round(tfs, 3), peak=peak_f, unit="TFLOP/s", frac=round(tfs / peak_f, 4))
    main, other = (dict(bound="alu", **alu), dict(hbm=hbm)) if ai > ridge else \
        (dict(bound="hbm", **hbm), dict(alu=alu))
    return dom, dict(main, traffic=None, kernel=dom, avg_launch_us=round(avg_s * 1e6, 3),
                     launches=int(s.launches), algorithmic_bytes_per_launch=int(nbytes),
                     bytes_per_particle=bpp, particles_per_launch=int(n_slots),
                     flops_per_launch=int(flops), flops_per_pair=fpp,
                     pairs_per_launch=int(pairs_per_launch),
                     arithmetic_intensity=round(ai, 2), ridge=round(ridge, 2), **other)


def _adjoint_run(case, precision, steps, K, torch):
    from paper_2510_25702_amd import sph, sensitivity as sens
    sim = sph.Simulation(case, precision=precision)
    start = sim.save()
    desc = sph.make_objective(case.objective, 1)
    pid_cap = sens.default_pid_cap(sim, steps)
    # plain forward steps (cell build, correction, step, buffer update)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.advance()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    sim.restore(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, recs, ckpts = sens.rollout(sim, steps, desc, pid_cap, checkpoint_every=K)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    tim = {}
    t0 = time.perf_counter()
    g = sens.adjoint(sim, desc, recs, ckpts, pid_cap, torch.tensor([1.0, 1.0], dtype=torch.float64),
                     steps, K, timings=tim)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    return dict(g=g.cpu().numpy(), J=(J / steps).cpu().numpy(), t_plain=t_plain, t_fwd=t_fwd,
                t_bwd=t_bwd, tim=tim)


def adjoint_leg(steps, K, torch):
    """Inlet-profile sensitivity on the adjoint channel: FP32-mixed forward
    with the FP64 reverse sweep (the configured run) -- the recorded forward
    rollout, the checkpointed reverse sweep, and a plain forward rollout of
    the same steps for the cost ratio -- and the same with an FP64 forward,
    whose gradient the FP32-forward one is compared with."""
    import numpy as np
    import cases
    from paper_2510_25702_amd import sph
    case = cases.make_adjoint_channel(steps=steps)
    r = _adjoint_run(case, sph.SPH_FP32_MIXED, steps, K, torch)
    r64 = _adjoint_run(case, sph.SPH_FP64, steps, K, torch)
    g, g64 = r["g"], r64["g"]
    ms = lambda t: round(1e3 * t / steps, 4)
    tim = r["tim"]
    return {"workload": "adjoint_channel", "particles_total": int(case.n), "steps": steps,
            "checkpoint_every": K, "precision": "fp32-mixed forward, fp64 reverse",
            "objective": "mean over steps of J_Q (outlet slab mass flux) + J_tau (wall shear)",
            "J": [float(r["J"][0]), float(r["J"][1])], "grad_norm": float(np.linalg.norm(g)),
            "grad_rel_diff_vs_fp64_forward": float(np.abs(g - g64).max() / np.abs(g64).max()),
            "forward_ms_per_step": ms(r["t_plain"]), "recorded_forward_ms_per_step": ms(r["t_fwd"]),
            "backward_ms_per_step": ms(r["t_bwd"]),
            "adjoint_step_ms": ms(tim["adjoint_s"]), "recompute_ms_per_step": ms(tim["recompute_s"]),
            "adjoint_step_over_forward": round(tim["adjoint_s"] / r["t_plain"], 3),
            "backward_over_forward": round(r["t_bwd"] / r["t_plain"], 3),
            "fp64": {"forward_ms_per_step": ms(r64["t_plain"]),
                     "adjoint_step_ms": ms(r64["tim"]["adjoint_s"]),
                     "adjoint_step_over_forward": round(r64["tim"]["adjoint_s"] / r64["t_plain"], 3),
                     "backward_over_forward": round(r64["t_bwd"] / r64["t_plain"], 3)}}


TRAFFIC_SOURCES = ("k_pairs.hip", "sph_pairs.h", "sph_device.h", "sph_ctx.h")


def kernel_source_hash():
    """Digest of the sources of the neighbour-pass kernels: a recorded
    traffic figure is used only while they are the ones it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2510_25702_amd", "csrc")
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, kernel, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy calibration), or
    None when there is none for these sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    e = rec.get("kernels", {}).get(f"{workload}/{precision}/{kernel}")
    return None if e is None else e.get("bytes_per_launch")


def oracle_threads():
    """Host threads for the oracle: the cores this process may run on, at
    most OMP_NUM_THREADS when that is set (the host's share for one GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(case, seconds, threads, what):
    """The FP64 oracle timed on the host: advection steps of `case` from its
    initial state, each followed by its buffer update, until `seconds` have
    passed (at least one); particle-steps/s over the real particles."""
    import oracle
    s = oracle.OracleSim(case, threads=threads)
    s.buffer_update()
    t0 = time.perf_counter()
    psteps = 0
    k = 0
    while True:
        s.step()
        c = s.buffer_update()
        psteps += c.n_real
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=round(psteps / dt, 1), unit="particle-steps/s", cores=threads,
                kind="oracle", sample=f"the first {k} advection step(s) (+ buffer updates) of "
                                      f"{what} ({case.n} particles) from its initial state, "
                                      f"{dt:.1f} s")


def gpu_leg(case, precision, steps, warmup, torch):
    """One timed run and its figures (value, ms per step, pairs/s, roofline)."""
    from paper_2510_25702_amd import sph
    r = run_gpu(case, precision, steps, warmup, torch)
    g = r["sim"]
    prec = "fp32" if precision == sph.SPH_FP32_MIXED else "fp64"
    dom, roof = roofline(r["stats"], case.params["dim"], prec, walked_pairs(g), g.n,
                         bool(case.params["turbulence"]))
    kern = {k: {"avg_us": round(1e3 * v.total_ms / max(1, v.launches), 3),
                "launches": int(v.launches)} for k, v in r["stats"].items() if v.launches}
    return r, dict(value=round(r["particle_steps"] / r["seconds"], 1),
                   ms_per_step=round(1e3 * r["seconds"] / steps, 4),
                   pairs_per_s=round(r["pairs"] / r["seconds"], 1),
                   acoustic_substeps=int(r["n_ac"]), list_outgrown_steps=int(r["outgrown"]),
                   roofline=roof, kernels=kern)


def sweep(names, steps, warmup, torch):
    from paper_2510_25702_amd import sph
    out = {}
    for name in names:
        case = make_case(name)
        row = {"description": WORKLOADS[name][2], "particles_total": int(case.n),
               "steps": steps}
        for prec, key in ((sph.SPH_FP32_MIXED, "fp32_mixed"), (sph.SPH_FP64, "fp64")):
            r, fig = gpu_leg(case, prec, steps, warmup, torch)
            row[key] = fig
            del r
        row["fp32_over_fp64"] = round(row["fp32_mixed"]["value"] / row["fp64"]["value"], 3)
        out[name] = row
        print(f"sweep {name}: {row['fp32_mixed']['value']:.4g} / {row['fp64']['value']:.4g} "
              f"particle-steps/s", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.summarize_traffic:
        summarize_traffic(args, *args.summarize_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"decomposition is described, not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20)
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n, "copies": 5}), flush=True)
        return
    if args.laminar_jet:
        print(json.dumps({"laminar_jet": laminar_jet(steps=args.jet_steps,
                                                     navg=min(5000, args.jet_steps // 4),
                                                     precision=args.jet_precision,
                                                     nf=args.jet_nf, p_far=args.p_far)}),
              flush=True)
        return
    if args.config_run:
        print(json.dumps({"config_run": config_run(args.config_run, args.tvf_alpha,
                                                    args.config_steps, torch,
                                                    p_far=args.p_far)}), flush=True)
        return
    if args.obc_ablation:
        print(json.dumps({"obc_ablation": obc_ablation(steps=6000, navg=2000)}), flush=True)
        return
    from paper_2510_25702_amd import sph
    case = make_case(args.workload)
    r32, f32 = gpu_leg(case, sph.SPH_FP32_MIXED, args.steps, args.warmup, torch)
    print(f"{args.workload} FP32-mixed: {f32['value']:.4g} particle-steps/s", file=sys.stderr,
          flush=True)
    roof = f32["roofline"]
    roof["traffic"] = recorded_traffic(args.workload, roof["kernel"], "fp32")
    out = {
        "metric": "particle-steps/s + neighbor pairs/s, FP32-mixed vs FP64 at stated error",
        "value": f32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload][2],
                   "particles_real": int(r32["n_real"]), "particles_total": int(case.n),
                   "precision": "fp32-mixed (f32 pair arithmetic with f64 pressure and "
                                "continuity sums; f64 density, position, correction inverse)",
                   "acoustic_substeps": f32["acoustic_substeps"]},
        "pairs_per_s": f32["pairs_per_s"],
        "pairs_per_step": round(r32["pairs"] / args.steps, 1),
        "list_outgrown_steps": f32["list_outgrown_steps"],
        "roofline": roof,
        "kernels_sampled_every": PROFILE_EVERY,
        "kernels": {k: {"ms": round(v.total_ms, 3), "launches": int(v.launches),
                        "avg_us": round(1e3 * v.total_ms / max(1, v.launches), 3),
                        "GBps_all_own_fields": round(v.bytes / max(1e-12, v.total_ms * 1e-3) / 1e9, 1)}
                    for k, v in r32["stats"].items() if v.launches},
    }
    if not args.no_fp64:
        steps64 = args.fp64_steps or args.steps
        r64, f64 = gpu_leg(case, sph.SPH_FP64, steps64, args.warmup, torch)
        out["fp64"] = dict(f64, unit="particle-steps/s", steps=steps64)
        out["fp32_over_fp64"] = round(f32["value"] / f64["value"], 3)
        del r64
    threads = oracle_threads()
    out["stated_error_vs_fp64_oracle"] = stated_error(r32, case, threads)
    del r32
    if not args.no_sweep:
        out["sweep"] = sweep([w for w in SWEEP if w != args.workload], args.sweep_steps,
                             args.warmup, torch)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.adjoint_steps, args.adjoint_checkpoint, torch)
    if not args.no_cpu:
        big = args.workload in CPU_SMALL
        cb = cpu_baseline(make_case(args.workload), 0.0 if big else args.cpu_seconds, threads,
                          f"the {args.workload} workload")
        if big:
            gen, kw, what = CPU_SMALL[args.workload]
            import cases
            small = getattr(cases, gen)(**kw)
        else:
            small, what = make_case(args.workload), f"the {args.workload} workload"
        cb["single_core"] = cpu_baseline(small, 0.0 if big else args.cpu_seconds, 1, what)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
