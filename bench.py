"""Benchmark of the hot path on one MI355X.

Workload: the 53-species / 325-reaction methane-shaped synthetic mechanism,
100,000 thermochemical states resident in HBM.  One step = one pass of the hot
path over the batch: the dense analytical Jacobian (the kernel evaluates the
rates, production rates and RHS on the way) followed by the batched Newton
solve of I - h gamma J in mixed precision (FP32 LU on the matrix cores + FP64
refinement), with per-state step sizes that keep the systems solvable
(h = c / (gamma ||J||_inf), c log-uniform on [1, 3e3]).

The JSON line also carries: the roofline position of the Jacobian kernel
(HIP events on its launch stream), the Newton solve timed alone in both modes
(and on the configured step sizes h ~ logU[1e-9, 1e-5] s, where the systems
are numerically singular), a short Poisson serving run (p50/p99 latency, vs
the plain per-request FP64 path), and the CPU oracle's throughput on a
bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CFG = 1


def log(msg: str) -> None:
    """Progress of the benchmark legs on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kinetics.hip", "tables.hpp", "loader.cpp"):
        with open(os.path.join(ROOT, "paper_1605_03262_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(shape=None):
    """HBM bytes per launch of the Jacobian kernel from the committed rocprofv3
    counter summary, valid only while the kernel source is unchanged and for
    the launch shape that was measured."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash() or shape is None:
        return None
    e = d.get("shapes", {}).get(f"{shape[0]}x{shape[1]}")
    return None if e is None else e["bytes_per_launch"]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobian_c1_100k_traffic.json")
COPY_BYTES = 1 << 30     # calibration copy: reads and writes this many bytes


def pmc_pass(n_launch: int = 3) -> int:
    """Program profiled by the counter runs: warm-up and n_launch launches of
    the Jacobian, the rates kernel (every output) and the mixed Newton solve
    on the benchmark workload, then one plain device copy of COPY_BYTES (read
    COPY_BYTES, write COPY_BYTES) that calibrates the traffic counters."""
    import torch
    from paper_1605_03262_amd import Mechanism
    from synth import config_mechanism, config_states
    mech = config_mechanism(CFG)
    phi, p = config_states(CFG)
    M = Mechanism(text=mech.to_text(), device=0)
    N, n = mech.n_species, phi.shape[1]
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    jac = torch.empty((N * N, n), dtype=torch.float64, device="cuda")
    M.autotune(1, d_phi, d_p, out=jac, reps=3)      # the same launch shape bench.py times
    for _ in range(n_launch + 1):
        M.eval_jacobian(d_phi, d_p, out=jac)
    # the rates kernel (every output) and the mixed Newton solve of the benchmark step
    from paper_1605_03262_amd import NEWTON_MIXED
    from synth import NEWTON_GAMMA, conditioned_steps, draw_newton_inputs
    for _ in range(n_launch + 1):
        M.eval_rates(d_phi, d_p)
    rows = torch.abs(jac.view(N, N, n)).sum(dim=1).cpu().numpy()
    d_h = torch.from_numpy(conditioned_steps(3262 + 41, rows)).cuda()
    d_b = torch.from_numpy(draw_newton_inputs(3262 + 40, N, n)[1]).cuda()
    ws = torch.empty((M.newton_workspace_bytes(n, NEWTON_MIXED) + 256,), dtype=torch.uint8, device="cuda")
    for _ in range(n_launch + 1):
        M.newton_solve(jac, d_h, d_b, NEWTON_GAMMA, mode=NEWTON_MIXED, max_refine=4, rtol=1e-14, workspace=ws)
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"pmc pass done: {n_launch + 1} Jacobian, rates and mixed Newton launches of {n} states, "
          f"Jacobian shape {M.get_variant(1)[:2]}, copy of {COPY_BYTES} B", flush=True)
    return 0


PMC_COMMAND = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {c} -d $OUT/{d} "
               "-o {o} --output-format csv -- python3 $R/bench.py --pmc-pass   "
               "(R = repository root, OUT = output folder)")


def jacobian_only(cfg: int, steps: int) -> int:
    """Autotuned Jacobian kernel alone on one workload (for the other mechanism
    sizes; the benchmark step itself runs the 53-species workload)."""
    import torch
    from paper_1605_03262_amd import Mechanism
    from synth import WORKLOADS, config_mechanism, config_states
    mech = config_mechanism(cfg)
    phi, p = config_states(cfg)
    N, n = mech.n_species, phi.shape[1]
    M = Mechanism(text=mech.to_text(), device=0)
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    jac = torch.empty((N * N, n), dtype=torch.float64, device="cuda")
    tuned = M.autotune(1, d_phi, d_p, out=jac, reps=3)
    med, mean = time_stream(lambda: M.eval_jacobian(d_phi, d_p, out=jac), max(3, steps), torch)
    rmed, _ = time_stream(lambda: M.eval_rates(d_phi, d_p, rop_f=False, rop_r=False, pres_mod=False,
                                               wdot=False), max(3, steps), torch)
    # Newton solve of the same batch, both modes, conditioned steps
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED
    from synth import NEWTON_GAMMA, conditioned_steps, draw_newton_inputs
    M.eval_jacobian(d_phi, d_p, out=jac)
    rows = torch.abs(jac.view(N, N, n)).sum(dim=1).cpu().numpy()
    d_h = torch.from_numpy(conditioned_steps(3262 + 41, rows)).cuda()
    d_b = torch.from_numpy(draw_newton_inputs(3262 + 40, N, n)[1]).cuda()
    ws = torch.empty((max(M.newton_workspace_bytes(n, 0), M.newton_workspace_bytes(n, 1), 1),),
                     dtype=torch.uint8, device="cuda")
    newton = {}
    for mode, name in ((NEWTON_FP64, "fp64_lu"), (NEWTON_MIXED, "fp32_lu_fp64_refine")):
        run = lambda: M.newton_solve(jac, d_h, d_b, NEWTON_GAMMA, mode=mode, max_refine=4,  # noqa: E731
                                     rtol=1e-14, workspace=ws)
        nmed, _ = time_stream(run, 3, torch)
        _, info = run()
        torch.cuda.synchronize()
        newton[name] = {"ms_median": nmed, "fallbacks": int((info[:n] == -2).sum().item())}
    newton["mixed_speedup"] = newton["fp64_lu"]["ms_median"] / newton["fp32_lu_fp64_refine"]["ms_median"]
    # one SDIRK3 integrator step of the batch: h = c / (gamma ||J||_inf), c log-uniform on [0.1, 10],
    # 4 simplified-Newton iterations per stage
    import numpy as np
    c = np.exp(np.random.default_rng(3262 + 42).uniform(np.log(0.1), np.log(10.0), n))
    d_hs = torch.from_numpy(c / (NEWTON_GAMMA * rows.max(axis=0))).cuda()
    del ws
    out_phi = torch.empty_like(d_phi)
    sdirk = {"newton_iters": 4, "h": "c / (gamma ||J||_inf), c log-uniform on [0.1, 10]"}
    for mode, name in ((NEWTON_FP64, "fp64_lu"), (NEWTON_MIXED, "fp32_lu_fp64_refine")):
        sws = torch.empty((max(_sdirk_ws(M, n, mode), 1),), dtype=torch.uint8, device="cuda")
        run = lambda: M.sdirk3_step(d_phi, d_p, d_hs, newton_iters=4, mode=mode, out=out_phi,  # noqa: E731
                                    workspace=sws)
        smed, _ = time_stream(run, 3, torch)
        sdirk[name] = {"ms_median": smed, "state_steps_per_s": n / (smed * 1e-3)}
        del sws
    by = n * (8.0 * N * N + 8.0 * (N + 1))
    print(json.dumps({"workload": WORKLOADS[cfg]["name"], "n_states": n, "n_species": N, "newton": newton,
                      "sdirk3_step": sdirk,
                      "jacobian_ms_median": med, "jacobian_evals_per_s": n / (med * 1e-3),
                      "hbm_frac": by / (med * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "rhs_ms_median": rmed, "rhs_evals_per_s": n / (rmed * 1e-3),
                      "shape": M.get_variant(1)[:2], "autotune": tuned}), flush=True)
    return 0


def _sdirk_ws(M, n, mode):
    from paper_1605_03262_amd import _lib
    return _lib.pyjac_sdirk3_workspace_bytes(M.handle, n, n, mode)


def _counter_rows(d: str, counter: str):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def write_traffic(fetch_dir: str, write_dir: str) -> int:
    """Turn the FETCH_SIZE and WRITE_SIZE runs of pmc_pass into HBM bytes per
    Jacobian launch for every launch shape the autotuner ran (mean over its
    dispatches), each counter scaled by what it reads for the plain copy
    (COPY_BYTES read and written).  Stored with a hash of the kernel source,
    so that a later kernel change invalidates them."""
    import re
    from synth import WORKLOADS
    out = {"kernel_source_hash": kernel_source_hash(), "workload": WORKLOADS[CFG]["name"],
           "copy_bytes": COPY_BYTES, "unit": "bytes per launch of 100,000 states", "shapes": {},
           "commands": [PMC_COMMAND.format(c="FETCH_SIZE", d=os.path.basename(os.path.normpath(fetch_dir)), o="f"),
                        PMC_COMMAND.format(c="WRITE_SIZE", d=os.path.basename(os.path.normpath(write_dir)), o="w")]}
    scale = {}
    per = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, name)
        cpy = [v for k, v in rows if "copy" in k.lower()]
        if not cpy:
            print(f"{name}: no copy-kernel row in {d}", file=sys.stderr)
            return 1
        scale[name] = (COPY_BYTES / 1024.0) / cpy[-1]
        for k, v in rows:
            m = re.search(r"tile_kernel<(\d+), (\d+), \d+, true(?:, (?:true|false))?>", k)
            if m:
                per.setdefault(f"{m.group(1)}x{m.group(2)}", {}).setdefault(name, []).append(v)
    for shape, d in per.items():
        if len(d) < 2:
            continue
        e = {c: sum(v) / len(v) * 1024.0 * scale[c] for c, v in d.items()}
        e["bytes_per_launch"] = e["FETCH_SIZE"] + e["WRITE_SIZE"]
        e["dispatches"] = len(d["FETCH_SIZE"])
        out["shapes"][shape] = e
    out["scale"] = scale
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)
    return 0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_leg(ref, phi, p, threads: int, budget_s: float):
    """Oracle Jacobians on the first states of the batch for about budget_s."""
    import numpy as np
    probe = 64 if threads == 1 else 256
    t0 = time.perf_counter()
    ref.eval_jacobian(phi[:, :probe], p[:probe], nthreads=threads)
    per_state = (time.perf_counter() - t0) / probe
    n = phi.shape[1]
    n_s = int(min(n, max(probe, budget_s / max(per_state, 1e-9))))
    sub_phi, sub_p = np.ascontiguousarray(phi[:, :n_s]), np.ascontiguousarray(p[:n_s])
    t0 = time.perf_counter()
    ref.eval_jacobian(sub_phi, sub_p, nthreads=threads)
    dt = time.perf_counter() - t0
    return n_s / dt, n_s, dt


def cpu_baseline(mech, phi, p, budget_s: float = 10.0):
    """The oracle (plain C++, OpenMP over states, not tuned) on the host:
    one thread and every available thread, each on the first states of the
    benchmark batch for about budget_s seconds."""
    from oracle import RefMech
    ref = RefMech(text=mech.to_text())
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    v1, n1, t1 = _oracle_leg(ref, phi, p, 1, budget_s)
    vn, nn, tn = _oracle_leg(ref, phi, p, threads, budget_s)
    return {"value": vn, "unit": "Jacobian evals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nn} of the {phi.shape[1]} states, {threads} OpenMP threads, {tn:.1f} s; "
                      f"single thread: first {n1} states, {t1:.1f} s",
            "single_thread_value": v1, "cpu_model": _cpu_model()}


def time_stream(fn, reps, torch):
    """Median and mean of `reps` runs of fn timed with HIP events on the
    current stream (where fn launches)."""
    import numpy as np
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return float(np.median(ms)), float(ms.mean())


R_GAS = 8314.462618      # J / (kmol K)


def parity_sample(mech, phi, p, jac, x, h, rhs, gamma, n_sample=64, seed=3262 + 50):
    """The timed step's own outputs on sampled states against the oracle:
    E_norm of the Jacobian (the gate is 1e-10) and the relative error of the
    Newton solution against a dense FP64 solve of (I - h gamma J_oracle) x = b
    (LAPACK, partial pivoting), next to that system's condition number."""
    import numpy as np
    from oracle import RefMech
    n, N = phi.shape[1], mech.n_species
    idx = np.sort(np.random.default_rng(seed).choice(n, size=min(n_sample, n), replace=False))
    import torch
    sel = torch.from_numpy(idx).to(jac.device)
    Jg = jac.index_select(1, sel).cpu().numpy()
    xg = x.index_select(1, sel).cpu().numpy()
    Jr = RefMech(text=mech.to_text()).eval_jacobian(np.ascontiguousarray(phi[:, idx]), p[idx])
    scale = np.max(np.abs(Jr), axis=0)
    scale[scale == 0] = 1.0
    e = np.linalg.norm((Jg - Jr) / scale, axis=0) / np.linalg.norm(Jr / scale, axis=0)
    xe, kap = [], []
    for s, i in enumerate(idx):
        A = np.eye(N) - h[i] * gamma * Jr[:, s].reshape(N, N)
        xr = np.linalg.solve(A, rhs[:, i])
        xe.append(np.linalg.norm(xg[:, s] - xr) / np.linalg.norm(xr))
        kap.append(np.linalg.cond(A, np.inf))
    return {"states": int(idx.size), "seed": seed, "jacobian_max_enorm": float(e.max()),
            "jacobian_gate": 1e-10, "jacobian_pass": bool(e.max() <= 1e-10),
            "newton_max_rel_err": float(max(xe)), "newton_max_cond_inf": float(max(kap))}


def conc_states(mech, phi, p):
    """(T, p, Y_1..Y_{N-1}) -> (T, [X_1..X_N]) by the ideal-gas law."""
    import numpy as np
    W = mech.molecular_weights()
    Y = np.vstack([phi[1:], 1.0 - phi[1:].sum(axis=0)])
    rho = p / (R_GAS * phi[0] * (Y / W[:, None]).sum(axis=0))
    return np.ascontiguousarray(np.vstack([phi[:1], rho * Y / W[:, None]]))


def conc_leg(M, mech, phi, p, torch, n_sample=32, seed=3262 + 51):
    """Concentration-based, constant-volume Jacobian (sparse species block) on
    the benchmark batch: autotuned launch shape, time per launch, algorithmic
    bytes (state in, dense temperature row/column + u_k + the nnz values of S
    out) and E_norm of sampled states against the oracle's dense Jacobian."""
    import numpy as np
    from oracle import RefMech
    N, n = mech.n_species, phi.shape[1]
    c = conc_states(mech, phi, p)
    d_c = torch.from_numpy(c).cuda()
    colptr, rowidx = M.conc_pattern()
    nnz = len(rowidx)
    rows = 3 * N + 1 + nnz
    out = torch.empty((rows, n), dtype=torch.float64, device="cuda")
    tuned = M.autotune(2, d_c, None, out=out, reps=3)
    med, _ = time_stream(lambda: M.eval_jacobian_conc(d_c, out=out), 5, torch)
    by = n * 8.0 * ((N + 1) + rows)
    idx = np.sort(np.random.default_rng(seed).choice(n, size=min(n_sample, n), replace=False))
    o = out.index_select(1, torch.from_numpy(idx).cuda()).cpu().numpy()
    J = np.zeros((N + 1, N + 1, idx.size))
    J[0, 0] = o[0]
    J[1:, 0] = o[1:N + 1]
    J[0, 1:] = o[N + 1:2 * N + 1]
    J[1:, 1:] = o[2 * N + 1:3 * N + 1][:, None, :]
    for j in range(N):
        for q in range(colptr[j], colptr[j + 1]):
            J[1 + rowidx[q], 1 + j] += o[3 * N + 1 + q]
    Jg = J.reshape((N + 1) ** 2, idx.size)
    Jr = RefMech(text=mech.to_text()).eval_jacobian_conc(np.ascontiguousarray(c[:, idx]))
    scale = np.max(np.abs(Jr), axis=0)
    scale[scale == 0] = 1.0
    e = np.linalg.norm((Jg - Jr) / scale, axis=0) / np.linalg.norm(Jr / scale, axis=0)
    ts, nt, lds = M.get_variant(2)
    del out, d_c
    return {"ms_per_launch": med, "evals_per_s": n / (med * 1e-3), "nnz_sparse_block": nnz,
            "dense_entries": (N + 1) ** 2, "outputs_per_state": rows,
            "algorithmic_bytes_per_state": by / n, "hbm_frac": by / (med * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "shape": {"tile_states": ts, "threads": nt, "lds_bytes": lds},
            "autotune_ms": [{"tile_states": sh[0], "threads": sh[1], "ms": t} for sh, t in tuned],
            "sample_max_enorm": float(e.max()), "sample_states": int(idx.size)}


def cs_leg(M, d_phi, d_p, n_cs, jac_ms, n, torch):
    """Complex-step Jacobian (the accuracy reference) on the first n_cs states."""
    N = M.n_species
    out = torch.empty((N * N, n_cs), dtype=torch.float64, device="cuda")
    ph, pp = d_phi[:, :n_cs].contiguous(), d_p[:n_cs].contiguous()
    M.eval_jacobian_cs(ph, pp, out=out)
    med, _ = time_stream(lambda: M.eval_jacobian_cs(ph, pp, out=out), 3, torch)
    per = med / n_cs
    return {"states": n_cs, "ms_per_launch": med, "evals_per_s": n_cs / (med * 1e-3),
            "cs_over_analytical_time_per_state": per / (jac_ms / n)}


def rates_leg(M, d_phi, d_p, n, N, torch):
    """Rates kernel: net production rates only, and every output (rop_f, rop_r,
    pres_mod, wdot, dphi)."""
    wd, _ = time_stream(lambda: M.eval_rates(d_phi, d_p, rop_f=False, rop_r=False, pres_mod=False,
                                             wdot=True, dphi=True), 5, torch)
    out = M.eval_rates(d_phi, d_p)
    full, _ = time_stream(lambda: M.eval_rates(d_phi, d_p), 5, torch)
    ts, nt, _ = M.get_variant(0)
    n_out = sum(v.shape[0] for v in out.values())
    return {"rhs_only_ms": wd, "rhs_evals_per_s": n / (wd * 1e-3),
            "all_outputs_ms": full, "all_outputs_rows": n_out,
            "all_outputs_hbm_frac": n * 8.0 * (N + 1 + n_out) / (full * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "shape": {"tile_states": ts, "threads": nt}}


def pasr_leg(mech, M, torch, n_reactors=100, n_res=0.2, seed=3262 + 52):
    """PaSR particle driver (App. C) on the benchmark mechanism: 100 reactors
    of 100 particles, T_in 600 K, 10 atm, tau_res 5 ms, tau_mix = tau_pair
    = 1 ms, advanced n_res residence times; then the Jacobian timed on the
    resulting particle states (the paper's own test distribution), with the
    E_norm of 32 sampled states against the oracle."""
    import numpy as np
    from oracle import RefMech
    from paper_1605_03262_amd.pasr import PaSR, burn
    from synth import ATM, pasr_fresh
    p_pa = 10 * ATM
    fresh = pasr_fresh(mech, 600.0, seed)
    hot = fresh.copy()
    hot[0] = 2000.0
    pilot = burn(M, hot, p_pa)
    reactor = PaSR(M, n_reactors=n_reactors, fresh=fresh, pilot=pilot, p_pa=p_pa, tau_res=5e-3, seed=seed)
    t0 = time.perf_counter()
    phi, p = reactor.run(n_res)
    wall = time.perf_counter() - t0
    n = phi.shape[1]
    steps = max(1, round(n_res * reactor.tau_res / reactor.dt))
    d_phi, d_p = torch.from_numpy(phi).cuda(), torch.from_numpy(p).cuda()
    N = mech.n_species
    jac = torch.empty((N * N, n), dtype=torch.float64, device="cuda")
    M.eval_jacobian(d_phi, d_p, out=jac)
    med, _ = time_stream(lambda: M.eval_jacobian(d_phi, d_p, out=jac), 5, torch)
    idx = np.sort(np.random.default_rng(seed).choice(n, size=32, replace=False))
    Jg = jac.index_select(1, torch.from_numpy(idx).cuda()).cpu().numpy()
    Jr = RefMech(text=mech.to_text()).eval_jacobian(np.ascontiguousarray(phi[:, idx]), p[idx])
    scale = np.max(np.abs(Jr), axis=0)
    scale[scale == 0] = 1.0
    e = np.linalg.norm((Jg - Jr) / scale, axis=0) / np.linalg.norm(Jr / scale, axis=0)
    return {"particles": n, "reactors": n_reactors, "time_steps": steps, "sub_steps_per_step": reactor.n_sub,
            "wall_s": wall, "particle_steps_per_s": n * steps / wall,
            "frozen_particle_steps": int(getattr(reactor, "frozen", 0)),
            "T_range_K": [float(phi[0].min()), float(phi[0].max())],
            "jacobian_ms_on_pasr_states": med, "jacobian_evals_per_s_on_pasr_states": n / (med * 1e-3),
            "sample_max_enorm": float(e.max())}


def serving_run(n_requests: int, seed: int = 7):
    """Poisson streams of Jacobian + mixed-Newton requests over the 13/53/111/
    360-species mechanisms (weights 0.4/0.3/0.2/0.1), n = floor(exp(U[0, ln 4097)))
    states each, served continuously at 50/80/95 % of the burst saturation rate;
    the 80 % trace also goes through the plain path (each request alone, in
    arrival order, FP64 LU, one stream)."""
    import numpy as np
    import torch
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED, Mechanism, Server
    from synth import conditioned_steps, config_mechanism, draw_newton_inputs, draw_states, NEWTON_GAMMA
    rng = np.random.default_rng(seed)
    mechs = [Mechanism(text=config_mechanism(c).to_text()) for c in range(4)]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    reqs = []
    for _ in range(n_requests):
        c = int(rng.choice(4, p=[0.4, 0.3, 0.2, 0.1]))
        n = min(4096, int(np.exp(rng.uniform(0.0, np.log(4097.0)))))
        N = mechs[c].n_species
        phi, p = draw_states(int(rng.integers(1 << 30)), N, n, T=(800.0, 2200.0), P_atm=(1.0, 50.0),
                             dirichlet=0.3)
        _, b = draw_newton_inputs(int(rng.integers(1 << 30)), N, n)
        # solvable steps, as an integrator's step control keeps them: h = c / (gamma ||J||_inf),
        # with ||J||_inf from the library's own Jacobian (set-up, outside every timed run)
        rows = torch.abs(mechs[c].eval_jacobian(dev(phi), dev(p)).view(N, N, n)).sum(dim=1).cpu().numpy()
        h = conditioned_steps(int(rng.integers(1 << 30)), rows)
        reqs.append((c, phi, p, h, b))
    torch.cuda.synchronize()
    total_states = sum(r[1].shape[1] for r in reqs)

    def run_server(gaps, mode):
        srv = Server(hbm_budget_bytes=64 << 30, max_batch_states=4096, n_streams=4, max_refine=4)
        ids = []
        t0 = time.perf_counter()
        tnext = t0
        for (c, phi, p, h, b), gap in zip(reqs, gaps):
            tnext += gap
            d = tnext - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ids.append(srv.submit(mechs[c], phi, p, h, b, NEWTON_GAMMA, mode=mode)[0])
        lat = [srv.wait(i) for i in ids]
        wall = time.perf_counter() - t0
        st = srv.stats()
        st.update(srv.graph_stats())
        srv.close()
        return np.array(lat), wall, st

    served = {}
    gaps80 = None
    for mode, name in ((NEWTON_MIXED, "mixed_fp32_lu_fp64_refine"), (NEWTON_FP64, "fp64_lu")):
        lat_b, wall_b, st_b = run_server(np.zeros(n_requests), mode)  # closed burst: saturation
        sat_rate = n_requests / wall_b
        loads = {}
        for frac in (0.5, 0.8, 0.95):
            gaps = rng.exponential(1.0 / (frac * sat_rate), size=n_requests)
            if frac == 0.8 and gaps80 is None:
                gaps80 = gaps
            lat, wall, st = run_server(gaps, mode)
            log(f"serving {name} at {int(frac * 100)}% load done")
            loads[f"{int(frac * 100)}%"] = {
                "arrival_rate_req_per_s": frac * sat_rate,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "states_per_s": total_states / wall, "rounds": st["batches"],
                "graph_replayed_rounds": st["replayed_rounds"]}
        served[name] = {"burst_saturation_req_per_s": sat_rate, "burst_states_per_s": total_states / wall_b,
                        "burst_rounds": st_b["batches"],
                        "burst_graphs": {k: st_b[k] for k in ("eager_rounds", "captured_rounds", "replayed_rounds",
                                                              "jacobian_launches", "multi_mechanism_launches")},
                        "offered_load": loads}

    arrivals = np.cumsum(gaps80)
    plain_lat = []
    t0 = time.perf_counter()
    for (c, phi, p, h, b), ta in zip(reqs, arrivals):
        d = t0 + ta - time.perf_counter()
        if d > 0:
            time.sleep(d)
        M = mechs[c]
        J = M.eval_jacobian(dev(phi), dev(p))
        x, info = M.newton_solve(J, dev(h), dev(b), NEWTON_GAMMA, mode=NEWTON_FP64)
        x.cpu()
        plain_lat.append(time.perf_counter() - (t0 + ta))
        del J, x, info
    plain_wall = time.perf_counter() - t0
    plain_lat = np.array(plain_lat)
    return {
        "requests": n_requests, "states": int(total_states),
        "newton_inputs": "b ~ N(0, 1); h = c / (gamma ||J||_inf), c log-uniform on [1, 3e3] (solvable systems)",
        "server": served,
        "plain_fp64_per_request_at_80%_of_mixed_saturation": {"p50_ms": float(np.percentile(plain_lat, 50) * 1e3),
                                          "p99_ms": float(np.percentile(plain_lat, 99) * 1e3),
                                          "states_per_s": total_states / plain_wall},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--states", type=int, default=None, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-pasr", action="store_true", help="skip the PaSR leg (its integrator launches the "
                    "Jacobian kernel on 10,000-state batches, which would mix into a profile's averages)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--variant", type=str, default=None, help="Jacobian launch shape TS,NT")
    ap.add_argument("--jacobian-only-config", type=int, default=None, metavar="ID",
                    help="only time the Jacobian kernel on workload ID (0-3) and print its roofline line")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="only run the program that the counter runs profile")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="store HBM bytes per launch from two rocprofv3 --pmc output folders")
    args = ap.parse_args()
    if args.write_traffic:
        return write_traffic(*args.write_traffic)
    if args.pmc_pass:
        return pmc_pass()
    if args.jacobian_only_config is not None:
        return jacobian_only(args.jacobian_only_config, args.steps)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); states are "
              "independent, so several GPUs would each run this same single-GPU path on their "
              "own shard.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1605_03262_amd import NEWTON_FP64, NEWTON_MIXED, Mechanism, _lib
    from synth import (WORKLOADS, NEWTON_GAMMA, conditioned_steps, config_mechanism, config_states,
                       draw_newton_inputs)

    c = WORKLOADS[CFG]
    mech = config_mechanism(CFG)
    phi, p = config_states(CFG, args.states)
    n, N = phi.shape[1], mech.n_species
    M = Mechanism(text=mech.to_text(), device=0)
    d_phi = torch.from_numpy(phi).cuda()
    d_p = torch.from_numpy(p).cuda()
    jac = torch.empty((N * N, n), dtype=torch.float64, device="cuda")
    if args.variant:
        ts, nt = (int(v) for v in args.variant.split(","))
        M.set_variant(1, ts, nt)
        tuned = None
    else:   # the library's autotuner picks the launch shape on this batch
        tuned = [{"tile_states": sh[0], "threads": sh[1], "ms": t}
                 for sh, t in M.autotune(1, d_phi, d_p, out=jac, reps=3)]
    h_cfg, rhs = draw_newton_inputs(3262 + 40, N, n)
    M.eval_jacobian(d_phi, d_p, out=jac)
    torch.cuda.synchronize()
    rows = torch.abs(jac.view(N, N, n)).sum(dim=1).cpu().numpy()
    h_cond = conditioned_steps(3262 + 41, rows)
    d_h = torch.from_numpy(h_cond).cuda()
    d_hcfg = torch.from_numpy(h_cfg).cuda()
    d_rhs = torch.from_numpy(rhs).cuda()
    ws = torch.empty((max(M.newton_workspace_bytes(n, 0), M.newton_workspace_bytes(n, 1)),),
                     dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}

    def newton(mode, hh):
        return M.newton_solve(jac, hh, d_rhs, NEWTON_GAMMA, mode=mode, max_refine=4, rtol=1e-14,
                              workspace=ws)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        M.eval_jacobian(d_phi, d_p, out=jac)
        if ev is not None:
            ev[1].record(stream)
        return newton(NEWTON_MIXED, d_h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x_last, info_last = step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps: {elapsed * 1e3 / args.steps:.3f} ms/step")
    # the last timed step's own outputs, checked against the oracle on sampled states
    parity = parity_sample(mech, phi, p, jac, x_last, h_cond, rhs, NEWTON_GAMMA)
    info_h = info_last[:n].cpu().numpy()
    parity["newton_fp64_fallbacks"] = int((info_h == -2).sum())
    parity["newton_singular"] = int((info_h == -1).sum())
    del x_last, info_last
    jac_ms = np.array([a.elapsed_time(b) for a, b in evs])
    jac_avg_ms = float(jac_ms.mean())
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed

    bytes_alg = n * (8.0 * N * N + 8.0 * (N + 1))
    achieved = bytes_alg / (jac_avg_ms * 1e-3) / 1e9
    # measured write peak: filling a buffer of the Jacobian's size (a device
    # fill kernel), the reference the nominal 8 TB/s is compared with
    fill_ms, _ = time_stream(lambda: jac.fill_(0.0), 5, torch)
    stream_write_gbs = jac.numel() * 8.0 / (fill_ms * 1e-3) / 1e9
    ts, nt, lds = M.get_variant(1)

    log(f"parity sample: max E_norm {parity['jacobian_max_enorm']:.2e}, Newton rel err {parity['newton_max_rel_err']:.2e}")
    # the paper's comparison method: forward-difference Jacobian on the same batch
    fd_out = torch.empty_like(jac)
    fd_ws = torch.empty((_lib.pyjac_fd_workspace_bytes(M.handle, 16384),), dtype=torch.uint8, device="cuda")
    fd_run = lambda: M.eval_jacobian_fd(d_phi, d_p, out=fd_out, workspace=fd_ws)  # noqa: E731
    fd_run()
    fd_med, _ = time_stream(fd_run, 3, torch)
    jac_med, _ = time_stream(lambda: M.eval_jacobian(d_phi, d_p, out=jac), 5, torch)
    fd_info = {"ms_per_launch": fd_med, "evals_per_s": n / (fd_med * 1e-3),
                          "analytical_ms_per_launch": jac_med,
                          "fd_over_analytical_time": fd_med / jac_med,
                          "method": "first-order forward differences of the GPU RHS, chunks of 16384 states"}
    del fd_out, fd_ws

    log("finite-difference Jacobian timed")
    # Newton alone, both modes, both step-size recipes
    newton_info = {}
    for label, hh in (("conditioned_h", d_h), ("configured_h", d_hcfg)):
        res = {}
        for mode, name in ((NEWTON_FP64, "fp64_lu"), (NEWTON_MIXED, "fp32_lu_fp64_refine")):
            med, mean = time_stream(lambda: newton(mode, hh), 3, torch)
            _, info = newton(mode, hh)
            torch.cuda.synchronize()
            info = info[:n].cpu().numpy()
            res[name] = {"ms_median": med, "states_per_s": n / (med * 1e-3),
                         "fp64_fallbacks": int((info == -2).sum()), "singular": int((info == -1).sum())}
            if mode == NEWTON_MIXED:
                sw = info[info > 0]
                res[name]["refine_sweeps_mean"] = float(sw.mean()) if sw.size else None
        res["mixed_speedup"] = res["fp64_lu"]["ms_median"] / res["fp32_lu_fp64_refine"]["ms_median"]
        # nominal LU flops (2/3 N^3) per state over the whole solve time (form, LU, solves, refinement)
        for name in ("fp64_lu", "fp32_lu_fp64_refine"):
            res[name]["lu_tflops_nominal"] = n * (2.0 / 3.0) * N ** 3 / (res[name]["ms_median"] * 1e-3) / 1e12
        newton_info[label] = res
    if N <= 64:
        newton_info["path"] = ("N <= 64, register-resident: FP64 LU one state per wavefront (row per lane, "
                               "v_readlane pivot rows); mixed mode FP32 LU with two states per wavefront "
                               "(rows spread over 32 lanes), FP64 residuals from the Jacobian restaged through "
                               "LDS each sweep, unconverged states re-solved in FP64")
    else:
        newton_info["path"] = ("N > 64, blocked: form A = I - h gamma J per state (LDS transpose), right-looking "
                               "LU with 16-column panels, trailing update on 16x16x4 MFMA (FP32 in mixed mode, "
                               "FP64 otherwise), triangular solves, FP64 residual refinement; non-converging "
                               "states re-solved in FP64")
    log("Newton timed")
    # the step's other kernel against the same HBM roofline: the mixed solve
    # reads J once for the FP32 factor and once per refinement sweep (it does
    # not fit on chip beside the factor), reads b and h, writes x and info
    mx = newton_info["conditioned_h"]["fp32_lu_fp64_refine"]
    sweeps = mx.get("refine_sweeps_mean") or 0.0
    nbytes = n * (8.0 * N * N * (1.0 + sweeps) + 16.0 * N + 12.0)
    newton_gbs = nbytes / (mx["ms_median"] * 1e-3) / 1e9
    roofline_newton = {"bound": "hbm", "achieved": newton_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": newton_gbs / HBM_PEAK_GBS,
                       "kernel": "mixed Newton solve call (conditioned h)", "avg_launch_ms": mx["ms_median"],
                       "algorithmic_bytes_per_launch": nbytes,
                       "bytes_per_state": "8 N^2 (1 + mean refinement sweeps) + 16 N + 12",
                       "refine_sweeps_mean": sweeps}
    rates_info = rates_leg(M, d_phi, d_p, n, N, torch)
    log("rates timed")
    conc_info = conc_leg(M, mech, phi, p, torch)
    log("concentration-form Jacobian timed")
    cs_info = cs_leg(M, d_phi, d_p, min(n, 8192), jac_med, n, torch)
    log("complex-step Jacobian timed")
    pasr_info = None if args.no_pasr else pasr_leg(mech, M, torch)
    if pasr_info is not None:
        log("PaSR driver and Jacobian on its states timed")

    out.update({
        "metric": "Jacobian evals/s (FP64, <=1e-10 rel err vs oracle) + p50/p99 request latency",
        "value": value, "unit": "Jacobian evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{c['name']}: {n} states, dense {N}x{N} FP64 Jacobian + "
                               f"mixed-precision Newton solve per step",
                   "n_species": N, "n_reactions": mech.n_reactions, "n_states": n,
                   "jacobian_variant": {"tile_states": ts, "threads": nt, "lds_bytes": lds},
                   "autotune_ms": tuned},
        "jacobian_only": {"ms_per_launch": jac_avg_ms, "evals_per_s": n / (jac_avg_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic((ts, nt)),
                     "kernel": "tile_kernel (Jacobian)", "avg_launch_ms": jac_avg_ms,
                     "algorithmic_bytes_per_launch": bytes_alg,
                     "traffic_source": "profiles/jacobian_c1_100k_traffic.json: rocprofv3 --pmc FETCH_SIZE and "
                                       "WRITE_SIZE runs of bench.py --pmc-pass, copy-calibrated; null unless the "
                                       "kernel source hash and launch shape match this run",
                     "target_frac": 0.60,
                     "measured_write_peak_GBps": stream_write_gbs,
                     "frac_of_measured_write_peak": achieved / stream_write_gbs},
        "roofline_newton": roofline_newton,
        "parity_sample": parity,
        "newton": newton_info,
        "rates": rates_info,
        "conc_jacobian": conc_info,
        "complex_step_jacobian": cs_info,
        "pasr": pasr_info,
        "fd_jacobian": fd_info,
    })
    if not args.no_serving:
        out["serving"] = serving_run(args.serving_requests)
    if not args.no_cpu_baseline:
        log("CPU oracle legs")
        out["cpu_baseline"] = cpu_baseline(mech, phi, p)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
