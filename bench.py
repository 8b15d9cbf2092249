#!/usr/bin/env python3
"""Benchmark: sigma = H C builds per second at CAS(16,16) on one MI355X.

One step = one full sigma build (sigma_1 + sigma_2 + sigma_3 of Eq. 8, with the
layout conversions) through cisigma_apply on a device-resident CI vector.
Prints one JSON line with
  * value: sigma builds/s of the FP32 path (FP32 MFMA, FP32 accumulation);
  * roofline: the alpha-beta contraction kernel (the dominant one) against the
    FP32 matrix-core peak, its duration measured with HIP events on its own
    stream over the timed region; its numerator is the method's own work, the
    sparse minimum 2 * sum over determinants of (alpha single excitations) x
    (beta single excitations) whose source determinant is in the space
    (2 [n_a (n - n_a + 1)]^2 N_det for a CAS), not the products the kernel
    issues (those are reported beside it as issued_flops);
  * cpu_baseline: the CPU oracle (plain Slater-Condon sigma) on a bounded
    random sample of output determinants of the same workload, scaled to
    sigma builds/s;
  * extra: the FP64 sigma rate, per-pass times, the FP32 sigma rate inside
    the even M_S = 0 sector (Sec. 3.3: no beta-beta pass), and the time to
    converge the Davidson energies (3 roots) in FP64 and in mixed precision
    (FP32 sigma and basis, FP64 projected problem and final refinement), with
    the largest energy difference between the two, plus mixed precision in the
    even sector; every Davidson eigenvector is checked against the oracle's
    sigma on sampled rows (energy_check_vs_oracle: sampled residual norm scaled
    to the whole vector and the energy error bound it implies);
  * extra.workloads: the GAS(20,20) space (FP32 and FP64 sigma, per pass) and
    the CAS(18,18) space (FP32 sigma), each with its sigma_3 fraction of peak on
    the same sparse-minimum numerator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cas16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6}     # MI355X dense matrix-core TFLOP/s
HBM_PEAK = 8000.0                         # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sigma3_min_products(spec):
    """(alpha excitation, beta excitation) products per sigma_3: for every
    determinant (I_a, I_b) of the space, the number of pairs (single excitation
    of I_a incl. E_kk, single excitation of I_b incl. E_kk) whose source
    determinant is in the space (Sec. 3.1: blocks of occupation types).  Counted
    per block from the occupation types alone; returns (products, ndet)."""
    import math
    n, na, nb = spec["norb"], spec["nalpha"], spec["nbeta"]
    if spec.get("orbsym") is not None:
        return _sigma3_min_products_sym(spec)
    gn, mn, mx = spec["gas"] if spec["gas"] else ([n], [na + nb], [na + nb])
    G = len(gn)

    def tuples(ne):
        out = []

        def rec(g, left, cur):
            if g == G:
                if left == 0:
                    out.append(tuple(cur))
                return
            for k in range(min(gn[g], left) + 1):
                rec(g + 1, left - k, cur + [k])
        rec(0, ne, [])
        return out

    def allowed(ta, tb):
        c = 0
        for g in range(G):
            c += ta[g] + tb[g]
            if c < mn[g] or c > mx[g]:
                return False
        return True

    def moves(t):
        # single excitations of a string of type t, grouped by source type:
        # electron from space gi to space gj (gi == gj includes the k == l terms)
        res = []
        for gi in range(G):
            for gj in range(G):
                c = t[gi] * (gn[gi] - t[gi] + 1) if gi == gj else t[gi] * (gn[gj] - t[gj])
                if c:
                    s = list(t)
                    s[gi] -= 1
                    s[gj] += 1
                    res.append((tuple(s), c))
        return res

    count = lambda t: math.prod(math.comb(gn[g], t[g]) for g in range(G))
    tot = ndet = 0
    for ta in tuples(na):
        for tb in tuples(nb):
            if not allowed(ta, tb):
                continue
            nd = count(ta) * count(tb)
            ndet += nd
            tot += nd * sum(ca * cb for sa, ca in moves(ta) for sb, cb in moves(tb) if allowed(sa, sb))
    return tot, ndet


def _sigma3_min_products_sym(spec):
    """sigma3_min_products for a CAS with orbital irreps (D2h products = XOR):
    an (alpha excitation i <- j, beta excitation k <- l) product of a
    determinant of the space has its source in the space exactly when the
    irreps of i, j, k, l multiply to the totally symmetric one (the same rule
    that leaves (ij|kl) nonzero).  With h(I, g) the single excitations of
    string I (E_kk included) whose two orbitals multiply to g, the count is
    sum over irreps a, g of H_alpha[a][g] H_beta[a ^ target][g], H[a][g] the sum
    of h over the strings of irrep a."""
    import itertools
    n, na, nb = spec["norb"], spec["nalpha"], spec["nbeta"]
    sym, tgt = spec["orbsym"], spec.get("target", 0)

    def hist(ne):
        H = [[0] * 8 for _ in range(8)]
        cnt = [0] * 8
        for occ in itertools.combinations(range(n), ne):
            irr = 0
            for p in occ:
                irr ^= sym[p]
            cnt[irr] += 1
            occ_set = set(occ)
            for j in occ:
                for i in range(n):
                    if i == j or i not in occ_set:
                        H[irr][sym[i] ^ sym[j]] += 1
        return H, cnt

    Ha, ca = hist(na)
    Hb, cb = hist(nb)
    prod = sum(Ha[a][g] * Hb[a ^ tgt][g] for a in range(8) for g in range(8))
    ndet = sum(ca[a] * cb[a ^ tgt] for a in range(8))
    return prod, ndet


def same_spin_floors(spec, ndet, w):
    """Floors of one same-spin pass of a one-block space (spin alpha; the beta
    pass is the same with the spins exchanged for n_a = n_b): compulsory HBM
    bytes (C read + sigma read-modify-write, 3 N_det w) at 8 TB/s, and the
    VALU flops of the sparse string Hamiltonian (2 N_a nnz N_b, nnz = 1 +
    n_a (n - n_a) + C(n_a, 2) C(n - n_a, 2) per row) at the FP32 or FP64 peak."""
    import math
    n, na, nb = spec["norb"], spec["nalpha"], spec["nbeta"]
    nnz = 1 + na * (n - na) + math.comb(na, 2) * math.comb(n - na, 2)
    nstr_a = math.comb(n, na)
    flops = 2.0 * nstr_a * nnz * (ndet // nstr_a)
    byt = 3.0 * ndet * w
    return {"compulsory_bytes": byt, "hbm_floor_ms": byt / (HBM_PEAK * 1e9) * 1e3, "valu_flops": flops,
            "valu_floor_ms": flops / ((PEAK["fp32"] if w == 4 else PEAK["fp64"]) * 1e12) * 1e3}


def time_sigma(ctx, cis, torch, dtype, steps, warmup, seed=0, parity=0):
    tdt = torch.float32 if dtype == "fp32" else torch.float64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1000 + seed)
    C = torch.randn(ctx.ndet, dtype=tdt, device="cuda", generator=gen)
    n = int(round(ctx.ndet ** 0.5))
    if parity and n * n == ctx.ndet:
        # a vector of the M_S = 0 sector: C(Ib, Ia) = parity * C(Ia, Ib)
        M = C.view(n, n)
        C = (0.5 * (M + parity * M.t())).reshape(-1).contiguous()
    # (spaces with several blocks: the vector is not projected onto the sector;
    # the cost of a sigma does not depend on the values, and this is timing only)
    C /= torch.linalg.vector_norm(C)
    S = torch.empty_like(C)
    ctx.set_option(cis.OPT_SPIN_PARITY, parity)
    for _ in range(warmup):
        ctx.apply(C, S)
    torch.cuda.synchronize()
    ctx.set_option(cis.OPT_PROFILE, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.apply(C, S)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    passes, ncalls = ctx.pass_times()
    ctx.set_option(cis.OPT_PROFILE, 0)
    assert ncalls == steps
    per_pass = {k: v / ncalls for k, v in passes.items()}
    # the same number of steps once more, each between two events on the stream it runs on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        ctx.apply(C, S)
        ev[k + 1].record()
    torch.cuda.synchronize()
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    per_pass["step_median"] = step_ms[len(step_ms) // 2]
    per_pass["step_min"] = step_ms[0]
    ctx.set_option(cis.OPT_SPIN_PARITY, 0)
    return dt, per_pass, C, S


def cpu_baseline(spec, h, g, C_dev, target_s, gpu_sigmas):
    """The oracle's row-sampled sigma of the benchmark vector, timed on all its
    threads and, for a few seconds, on one; the same rows also give the GPU
    sigma errors against the oracle (gpu_sigmas: name -> device sigma of the
    same vector).  Returns (baseline, errors, one-thread sigma builds/s)."""
    import numpy as np
    import oracle
    sp = oracle.Space(spec["norb"], spec["nalpha"], spec["nbeta"], h, g, gas=spec["gas"], orbsym=spec.get("orbsym"),
                      target=spec.get("target", 0))
    c = C_dev.double().cpu().numpy()
    rng = np.random.default_rng(7)
    nrows, done, t_used = 64, 0, 0.0
    all_rows, all_ref = [], []
    while t_used < target_s:
        rows = rng.integers(0, sp.ndet, nrows)
        t0 = time.perf_counter()
        ref = sp.sigma_rows(rows, c)
        t_used += time.perf_counter() - t0
        all_rows.append(rows)
        all_ref.append(ref)
        done += nrows
        nrows = min(nrows * 2, 1 << 16)
    rows_per_s = done / t_used
    rows = np.concatenate(all_rows)
    ref = np.concatenate(all_ref)
    import torch
    idx = torch.tensor(rows, device=C_dev.device)
    errs = {"rows": int(rows.size)}
    for name, S in gpu_sigmas.items():
        got = S[idx].double().cpu().numpy()
        errs[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    # the same sampling on one thread, for a few seconds
    nthreads = oracle.max_threads()
    oracle.set_threads(1)
    try:
        rows1 = rng.integers(0, sp.ndet, 256)
        t0 = time.perf_counter()
        n1 = 0
        while time.perf_counter() - t0 < min(3.0, target_s):
            sp.sigma_rows(rows1, c)
            n1 += rows1.size
        rate1 = n1 / (time.perf_counter() - t0)
    finally:
        oracle.set_threads(nthreads)
    one_thread = rate1 / sp.ndet
    model = "unknown CPU"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": rows_per_s / sp.ndet, "unit": "sigma builds/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{done} random output determinants of the same {sp.ndet}-determinant vector through "
                      f"the oracle's row-sampled Slater-Condon sigma ({t_used:.1f} s, {rows_per_s:.0f} rows/s "
                      f"on {nthreads} threads of {model}), scaled to the {sp.ndet} rows of one sigma build"}, errs, one_thread


def copy_calibration(torch, mib):
    """A plain streaming kernel of known size (read mib MiB, write mib MiB),
    launched so that a counter run (FETCH_SIZE / WRITE_SIZE) over this program
    also measures what those counters read for a known number of bytes."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def stored_traffic(kernel_tag):
    """HBM bytes per launch of the alpha-beta kernel from the committed counter
    summary, or None when the kernel source changed after the counters were
    taken (the summary records the source's SHA-256)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1707_04346_amd", "csrc")
    one_block = kernel_tag in ("k_sigma_ab_ws", "k_sigma_ab_x")
    srcs = [os.path.join(csrc, f) for f in (("sigma_abx.hip", "abx.h") if one_block else ("sigma_ab.hip",))]
    prof = os.path.join(ROOT, "profiles", f"{kernel_tag}_cas16_fp32_traffic.txt")
    if not (all(os.path.exists(f) for f in srcs) and os.path.exists(prof)):
        return None
    sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()
    fields = {}
    for ln in open(prof):
        if ":" in ln:
            k, v = ln.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_rdm(ctx, torch, n, na, nb, ndet):
    """Density matrices of a random vector, FP32 and FP64: milliseconds per call
    (HIP events, 3 calls after one warm-up) and the matrix-core rate of the
    products issued (upper triangle of 16x16 blocks of the (n^2+1)-row M)."""
    out = {}
    nbk = (n * n + 1 + 15) // 16
    npb = nbk * (nbk + 1) // 2
    lay = ctx.layout()
    nstr_a = int(lay["nalpha_str"][0])
    lda = -(-int(lay["nbeta_str"][0]) // 64) * 64          # beta columns, padded to 64
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        C = torch.randn(ndet, dtype=dt, device="cuda")
        g1 = torch.empty(n * n, dtype=torch.float64, device="cuda")
        g2 = torch.empty(n ** 4, dtype=torch.float64, device="cuda")
        ctx.rdm(C, g1, g2)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            ctx.rdm(C, g1, g2)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        flops = 2.0 * 16 * 16 * npb * lda * nstr_a
        out[name] = {"ms": ms, "issued_tflops": flops / (ms / 1e3) / 1e12, "trace_rdm1": float(g1.view(n, n).trace())}
        del C, g1, g2
    out["note"] = "spin-summed rdm1 + rdm2 of a random vector, device FP64 outputs"
    return out


def stored_same_spin_bytes():
    """HBM bytes of one same-spin pass (pair products + gather) from the committed
    counter summary, or None when those kernels, or the host code that sets
    their column chunks, changed after the counters were taken."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1707_04346_amd", "csrc")
    prof = os.path.join(ROOT, "profiles", "k_sigma_ab_x_cas16_fp32_traffic.txt")
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("sigma_ss.hip", "bufio.h", "api.hip"))).hexdigest()
    fields = {}
    for ln in open(prof):
        if ":" in ln:
            k, v = ln.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("same_spin_source_sha256") != sha:
        return None
    try:
        return float(fields["same_spin_hbm_bytes_per_pass"])
    except (KeyError, ValueError):
        return None


def cpu_leg_energy_check(spec, h, g, vecs, energies, nrows, seed, full_space=True):
    """Part of the CPU-oracle leg: the oracle's sigma (plain Slater-Condon, FP64)
    of each returned eigenvector x on nrows random determinants.  Per root the
    residual r = H x - E x on those rows, scaled to the whole vector,
    ||r|| ~ sqrt(N_det / nrows * sum_rows r_i^2) for normalised x, and the
    bound it implies on |E - lambda| for the nearest exact eigenvalue lambda of
    the symmetric H: ||r||.  For a full-space run, where the computed roots are
    the lowest eigenvalues, also ||r||^2 / gap with gap the distance to the
    nearest other computed root (Kato-Temple; an estimate, since the gap itself
    is computed).  A sector run has no such estimate: eigenvalues of the other
    sector may lie between its roots."""
    import numpy as np
    import oracle
    sp = oracle.Space(spec["norb"], spec["nalpha"], spec["nbeta"], h, g, gas=spec["gas"], orbsym=spec.get("orbsym"),
                      target=spec.get("target", 0))
    rng = np.random.default_rng(seed)
    rows = np.unique(rng.integers(0, sp.ndet, nrows))
    out = []
    t0 = time.perf_counter()
    for r, e in enumerate(energies):
        x = vecs[r].double().cpu().numpy()
        x /= np.linalg.norm(x)
        res = sp.sigma_rows(rows, x) - e * x[rows]
        rn = float(np.sqrt(sp.ndet / rows.size * np.sum(res ** 2)))
        others = [abs(e - f) for k, f in enumerate(energies) if k != r]
        gap = min(others) if others else None
        out.append({"root": r, "energy": float(e), "sampled_residual_norm": rn, "bound_residual": rn,
                    "kato_temple_estimate": (rn * rn / gap) if (gap and full_space) else None})
    return {"rows": int(rows.size), "seconds": time.perf_counter() - t0, "roots": out,
            "note": "oracle sigma of the returned eigenvectors on random rows; |E - exact| <= bound_residual"}


def davidson_runs(ctx, cis, torch, nroots, tol, max_iter, verbose, sector, modes, max_space, check=None):
    """Davidson to convergence in each mode; with check = (spec, h, g, nrows)
    every run's eigenvectors are certified against the oracle on sampled rows
    (the CPU-oracle leg)."""
    out = {}
    ctx.set_option(cis.OPT_MAX_ITER, max_iter)
    ctx.set_option(cis.OPT_VERBOSE, 1 if verbose else 0)
    if max_space:
        ctx.set_option(cis.OPT_MAX_SPACE, max_space)
    runs = [("fp64", cis.FP64, 0), ("mixed_fp32", cis.FP32, 0)]
    if sector:
        # lowest roots of the even-spin M_S = 0 sector (singlets first)
        runs.append(("mixed_fp32_even_sector", cis.FP32, 1))
    runs = [r for r in runs if r[0] in modes]
    for mode, prec, parity in runs:
        ctx.set_option(cis.OPT_PRECISION, prec)
        ctx.set_option(cis.OPT_SPIN_PARITY, parity)
        vecs = None
        if check is not None:
            vecs = torch.empty(nroots, ctx.ndet, dtype=torch.float64 if prec == cis.FP64 else torch.float32,
                               device="cuda")
        t0 = time.perf_counter()
        e, st, status = ctx.davidson(nroots, tol, vecs=vecs, allow_noconv=True)
        secs = time.perf_counter() - t0
        ctx.set_option(cis.OPT_SPIN_PARITY, 0)
        out[mode] = {"seconds": secs, "energies": [float(x) for x in e], "status": status,
                     "iterations": st["iterations"], "sigma_fp32": st["sigma_fp32"], "sigma_fp64": st["sigma_fp64"],
                     "refinements": st["refinements"], "residual": st["residual"]}
        if vecs is not None:
            spec, h, g, nrows = check
            out[mode]["energy_check_vs_oracle"] = cpu_leg_energy_check(spec, h, g, vecs, out[mode]["energies"],
                                                                       nrows, 31, full_space=parity == 0)
            del vecs
            torch.cuda.empty_cache()
        log(f"davidson {mode}: {out[mode]}")
    ctx.set_option(cis.OPT_PRECISION, cis.FP64)
    if "fp64" in out and "mixed_fp32" in out:
        d = [abs(a - b) for a, b in zip(out["fp64"]["energies"], out["mixed_fp32"]["energies"])]
        out["max_abs_energy_diff_mixed_vs_fp64"] = max(d)
    if "fp64" in out and "mixed_fp32_even_sector" in out:
        out["even_sector_E0_minus_full_E0"] = out["mixed_fp32_even_sector"]["energies"][0] - out["fp64"]["energies"][0]
    return out


def extra_workload(name, cis, torch, si, steps, warmup, fp64):
    """sigma timing of another configuration (per pass, HIP events), with the
    sigma_3 kernel's fraction of the matrix-core peak on the method's own work
    (the sparse minimum of sigma3_min_products)."""
    spec = si.WORKLOADS[name]
    h, g = si.integrals(spec["norb"], spec["nchol"], 0, orbsym=spec.get("orbsym"))
    t0 = time.perf_counter()
    ctx = cis.Context(spec["norb"], spec["nalpha"], spec["nbeta"], h, g, gas=spec["gas"],
                      orbsym=spec.get("orbsym"), target=spec.get("target", 0))
    out = {"ndet": ctx.ndet, "init_seconds": time.perf_counter() - t0, "gas": spec["gas"],
           "orbsym": spec.get("orbsym"), "target": spec.get("target")}
    prod, nd = sigma3_min_products(spec)
    assert nd == ctx.ndet
    out["sigma3_min_flops"] = 2.0 * prod
    for dt in (("fp32", "fp64") if fp64 else ("fp32",)):
        d, pp, C, S = time_sigma(ctx, cis, torch, dt, steps, warmup)
        del C, S
        torch.cuda.empty_cache()
        ms = 1e3 * d / steps
        flags = ctx.last_path(cis.FP32 if dt == "fp32" else cis.FP64)
        out[dt] = {"ms_per_sigma": ms, "sigma_per_s": 1e3 / ms, "pass_ms": pp,
                   "sigma3_tflops": 2.0 * prod / (pp["sigma_ab"] / 1e3) / 1e12,
                   "sigma3_frac_of_peak": 2.0 * prod / (pp["sigma_ab"] / 1e3) / 1e12 / PEAK[dt],
                   "path": {"ab_owner_computes": bool(flags & cis.PATH_AB_OWNER),
                            "same_spin_materialised": bool(flags & cis.PATH_SS_MATERIALISED)},
                   "sigma3_shape": ctx.last_shape(cis.FP32 if dt == "fp32" else cis.FP64)}
        log(f"{name} {dt}: {out[dt]}")
    if spec["gas"] is not None or spec.get("orbsym") is not None:
        # the per-block launch baseline: one launch per owner-computes unit instead of one over all
        ctx.set_option(cis.OPT_UNIT_LAUNCH, 1)
        d, pp, C, S = time_sigma(ctx, cis, torch, "fp32", steps, warmup)
        del C, S
        ctx.set_option(cis.OPT_UNIT_LAUNCH, 0)
        out["fp32_one_launch_per_unit"] = {"ms_per_sigma": 1e3 * d / steps, "pass_ms": pp}
        log(f"{name} fp32 one launch per unit: {out['fp32_one_launch_per_unit']}")
    if spec["nalpha"] == spec["nbeta"]:
        # the even M_S = 0 sector: the beta-beta pass replaced by the mirrored alpha-alpha part
        d, pp, C, S = time_sigma(ctx, cis, torch, "fp32", steps, warmup, parity=1)
        del C, S
        out["fp32_even_sector"] = {"ms_per_sigma": 1e3 * d / steps, "sigma_per_s": steps / d, "pass_ms": pp}
        log(f"{name} fp32 even sector: {out['fp32_even_sector']}")
    ctx.close()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cas16")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-davidson", action="store_true", help="skip timing Davidson to convergence (FP64 vs mixed)")
    ap.add_argument("--no-rdm", action="store_true", help="skip timing the density matrices")
    ap.add_argument("--nroots", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=300)
    ap.add_argument("--verbose", action="store_true", help="one line per Davidson iteration on stderr")
    ap.add_argument("--davidson-modes", default="fp64,mixed_fp32,mixed_fp32_even_sector",
                    help="comma list of the Davidson runs: fp64, mixed_fp32, mixed_fp32_even_sector")
    ap.add_argument("--max-space", type=int, default=0, help="Davidson subspace cap (0: the library's default)")
    ap.add_argument("--autotune", action="store_true",
                    help="let cisigma_autotune pick the launch parameters before timing (its report goes to extra)")
    ap.add_argument("--check-rows", type=int, default=10000,
                    help="random rows of the oracle's sigma per Davidson eigenvector (energy check)")
    ap.add_argument("--extra-workloads", default="gas20,cas18,cas16_d2h",
                    help="comma list of other configurations whose sigma is timed into extra.workloads ('' for none)")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed sigma builds per extra workload")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain copy kernel of this many MiB (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth_inputs as si
    import paper_1707_04346_amd as cis

    spec = si.WORKLOADS[args.workload]
    n, na, nb = spec["norb"], spec["nalpha"], spec["nbeta"]
    h, g = si.integrals(n, spec["nchol"], 0, orbsym=spec.get("orbsym"))
    t0 = time.perf_counter()
    ctx = cis.Context(n, na, nb, h, g, gas=spec["gas"], orbsym=spec.get("orbsym"), target=spec.get("target", 0))
    init_s = time.perf_counter() - t0
    log(f"init {args.workload}: ndet={ctx.ndet} in {init_s:.2f} s")

    tune = {}
    if args.autotune:
        t0 = time.perf_counter()
        for name, prec in (("fp32", cis.FP32), ("fp64", cis.FP64)):
            if name == "fp64" and args.no_fp64:
                continue
            tune[name] = ctx.autotune(prec, 3).strip().splitlines()
            log(f"autotune {name}: {tune[name]}")
        tune["seconds"] = time.perf_counter() - t0

    dt32, pp32, C32, S32 = time_sigma(ctx, cis, torch, "fp32", args.steps, args.warmup)
    ms32 = 1e3 * dt32 / args.steps
    path32 = ctx.last_path(cis.FP32)
    log(f"fp32 sigma: {ms32:.2f} ms/step, passes {pp32}, path flags {path32}")
    extra = {"init_seconds": init_s, "fp32_pass_ms": pp32, **({"autotune": tune} if tune else {}),
             "fp32_path": {"ab_owner_computes": bool(path32 & cis.PATH_AB_OWNER),
                           "same_spin_materialised": bool(path32 & cis.PATH_SS_MATERIALISED)}}
    # M_S = 0 sector (n_alpha = n_beta): the beta-beta pass is replaced by a transpose
    sector = na == nb
    if sector:
        dtp, ppp, _, _ = time_sigma(ctx, cis, torch, "fp32", args.steps, 1, parity=1)
        extra.update({"fp32_even_sector_sigma_per_s": args.steps / dtp,
                      "fp32_even_sector_ms_per_step": 1e3 * dtp / args.steps, "fp32_even_sector_pass_ms": ppp})
        log(f"fp32 sigma, even M_S=0 sector: {1e3 * dtp / args.steps:.2f} ms/step, passes {ppp}")
    if not args.no_fp64:
        dt64, pp64, _, _ = time_sigma(ctx, cis, torch, "fp64", max(2, args.steps // 2), 1)
        ms64 = 1e3 * dt64 / max(2, args.steps // 2)
        extra.update({"fp64_sigma_per_s": 1e3 / ms64, "fp64_ms_per_step": ms64, "fp64_pass_ms": pp64,
                      "speedup_fp32_vs_fp64": ms64 / ms32})
        log(f"fp64 sigma: {ms64:.2f} ms/step, passes {pp64}, path flags {ctx.last_path(cis.FP64)}")

    # alpha-beta contraction (sigma_3), on the method's own work: the sparse minimum
    # of (alpha excitation, beta excitation) products, 2 [n_a (n - n_a + 1)]^2 N_det
    # for a CAS.  The owner-computes kernel issues more: M = n_a (n - n_a) gathered
    # alpha rows x K = n(n+1)/2 orbital pairs per determinant (issued_flops).
    prod, nd = sigma3_min_products(spec)
    assert nd == ctx.ndet
    flops = 2.0 * prod
    issued = 2.0 * na * (n - na) * (n * (n + 1) // 2) * ctx.ndet
    ab_s = pp32["sigma_ab"] / 1e3
    achieved = flops / ab_s / 1e12
    owner = bool(path32 & cis.PATH_AB_OWNER)
    shared = bool(path32 & cis.PATH_AB_SHARED_CU)
    tag = ("k_sigma_ab_x" if shared else "k_sigma_ab_ws") if owner else "k_sigma_ab"
    kdesc = {"k_sigma_ab_x": "k_sigma_ab_x (owner-computes sigma_3, one-W-tile form, two workgroups per CU: "
                             "gathered C rows -> FP32 MFMA on six waves over three SIMDs, LDS scatter on two "
                             "waves on the fourth)",
             "k_sigma_ab_ws": "k_sigma_ab_ws (owner-computes sigma_3: gathered C rows -> FP32 MFMA on six waves "
                              "over three SIMDs, LDS scatter on two waves on the fourth)",
             "k_sigma_ab": "k_sigma_ab (sigma_3 gather -> FP32 MFMA -> atomic scatter)"}
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"],
                "traffic": stored_traffic(tag) if args.workload == "cas16" else None,
                "kernel": kdesc[tag],
                "flops_per_launch": flops,
                "flops_definition": "sparse minimum: 2 x sum over determinants of (alpha single excitations incl. "
                                    "E_kk) x (beta single excitations incl. E_kk) with the source determinant in "
                                    "the space",
                "issued_flops": issued, "issued_frac": issued / ab_s / 1e12 / PEAK["fp32"],
                "avg_launch_ms": pp32["sigma_ab"]}
    extra["sigma_ab_tflops_fp32"] = achieved
    if spec["gas"] is None and spec.get("orbsym") is None:
        # same-spin passes against their floors: t / max(HBM floor, VALU floor); the
        # counter bytes (when the committed summary matches the kernel source) beside them
        ss = same_spin_floors(spec, ctx.ndet, 4)
        t_ss = pp32["sigma_aa"]
        ss.update({"pass_ms": t_ss, "frac_of_floor": max(ss["hbm_floor_ms"], ss["valu_floor_ms"]) / t_ss,
                   "compulsory_GBps": ss["compulsory_bytes"] / (t_ss / 1e3) / 1e9,
                   "note": "frac_of_floor = max(compulsory-bytes time at 8 TB/s, VALU time of the sparse string "
                           "Hamiltonian at the FP32 peak) / pass time; the 60% HBM target is judged on it"})
        ssb = stored_same_spin_bytes() if args.workload == "cas16" else None
        if ssb is not None:
            ss["counter_bytes_per_pass"] = ssb
            ss["counter_GBps"] = ssb / (t_ss / 1e3) / 1e9
        extra["same_spin_pass"] = ss
    if not args.no_fp64:
        extra["sigma_ab_tflops_fp64"] = flops / (pp64["sigma_ab"] / 1e3) / 1e12
        extra["sigma_ab_frac_fp64"] = extra["sigma_ab_tflops_fp64"] / PEAK["fp64"]

    # NEXT: spin-summed 1- and 2-particle density matrices (one-block spaces, n <= 16)
    if spec["gas"] is None and spec.get("orbsym") is None and n <= 16 and not args.no_rdm:
        extra["rdm"] = time_rdm(ctx, torch, n, na, nb, ctx.ndet)
        log(f"rdm: {extra['rdm']}")

    if args.copy_calibration_mib > 0:
        copy_calibration(torch, args.copy_calibration_mib)

    cpu = None
    if not args.no_cpu:
        # sigma of the benchmark vector in both precisions, checked against the oracle on its sampled rows
        sig = {"fp32": S32}
        if not args.no_fp64:
            C64 = C32.double()
            S64 = torch.empty_like(C64)
            ctx.apply(C64, S64)
            torch.cuda.synchronize()
            sig["fp64"] = S64
        cpu, errs, one_thread = cpu_baseline(spec, h, g, C32, args.cpu_seconds, sig)
        extra["sigma_rel_error_vs_oracle_sampled_rows"] = errs
        extra["oracle_one_thread_sigma_builds_per_s"] = one_thread
        log(f"cpu baseline: {cpu}; sigma errors vs oracle: {errs}")
        del sig
        C64 = S64 = None

    if not args.no_davidson:
        # the Davidson basis lives in the library's own allocations: hand back what torch holds
        del C32, S32
        torch.cuda.empty_cache()
        extra["davidson"] = davidson_runs(ctx, cis, torch, args.nroots, args.tol, args.max_iter, args.verbose,
                                          sector, args.davidson_modes.split(","), args.max_space,
                                          None if args.no_cpu else (spec, h, g, args.check_rows))

    ndet = ctx.ndet
    C32 = S32 = None
    ctx.close()
    torch.cuda.empty_cache()
    if args.extra_workloads:
        # the other configurations of the metric: sigma timing per pass and sigma_3's fraction of peak
        extra["workloads"] = {}
        for name in args.extra_workloads.split(","):
            if name and name != args.workload:
                extra["workloads"][name] = extra_workload(name, cis, torch, si, args.extra_steps, 1,
                                                          name != "cas18")

    cfg = {"workload": f"{args.workload}: {n} orbitals, {na} alpha + {nb} beta electrons"
                       + (f", GAS {spec['gas']}" if spec["gas"] else " (CAS)")
                       + (f", orbital irreps {spec['orbsym']} target {spec['target']}" if spec.get("orbsym") else "")
                       + f", {ndet} determinants, seeded synthetic integrals (P={spec['nchol']})",
           "ndet": ndet, "norb": n, "nalpha": na, "nbeta": nb}
    line = {
        "metric": "sigma builds/s + sigma_ab TFLOP/s at CAS(16,16); Davidson time to 1e-6 Eh, FP32 vs FP64",
        "value": args.steps / dt32,
        "unit": "sigma builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
