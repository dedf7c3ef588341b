"""Learned warm start and low-rank preconditioner for band-limited Gauss-Newton-Krylov.

A small 3D convolutional encoder (WarmStartNet, bf16 matrix-core kernels in the HIP
library) maps the image pair, box-averaged to in_size^3 voxels, to grid samples of the
velocity on a coarse s^3 grid; their band-limited projection is the low-frequency block
(|m| <= s/2 - 1 per axis) of the velocity coefficients.  The committed network has four
levels (16 -> 128 channels) of strides 2, 2, 1, 1 on 64^3 inputs: s = 16, |m| <= 7.  It is trained on registrations
the method itself computes: image pair -> converged band-limited velocity of plain
Gauss-Newton-Krylov.  At registration time its prediction v0 is

* the initial guess of Gauss-Newton-Krylov (Section 2.3.1 starts from any v~; plain runs
  start from zero), with plain Gauss-Newton as the fallback when E(v0) > E(0), and
* optionally the source of r = 3 directions (the three velocity components of v0) for
  the two-level PCG preconditioner L~^{-1} + Z (Z^T H Z)^{-1} Z^T.

Plain and learned runs stop at the same absolute gradient: both normalise by the
gradient sup-norm at v = 0.

Every step runs in the library: pooling, the network, the coefficient map, the loss and
its gradient, Adam, and the registrations.  Python only draws the seeded phantom pairs
(paper_2006_06823_amd.synthetic) and schedules the calls.

Command line (runs on one ROCm device):
  python -m paper_2006_06823_amd.learned generate --seeds 10000:11000 --block 32 --out data0.npz
  python -m paper_2006_06823_amd.learned train --data data0.npz data1.npz --out-size 16 \\
         --eval-seeds 20000:20200 --weights net.npz --report report.json
(--variant 1 or 3 selects the image-transport or the deformation-state formulation, default 3;
--block the band of the stored targets, --out-size the network's output grid, to which the
targets are cropped.)
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import synthetic

SHAPE = (128, 128, 128)
BAND = (32, 32, 32)
NT = 10
IN_SIZE = 64
CHANNELS = (16, 32, 64, 128)
MAX_DISP_VOX = 8.0
BLOCK = 8  # coarse grid of the default network output = K of the predicted block


@dataclass
class SolveOpts:
    max_gn: int = 20
    max_pcg: int = 10
    grad_rtol: float = 1e-3


# Pairs of the learned path: "smooth" (the analytic low-frequency displacements of synthetic.phantom_pair_3d;
# the committed network's training and held-out pairs) or "prior" (the target is the template moved by a
# band-limited velocity drawn from the regulariser's prior, through the deformation-state solve; at 8 voxels
# these warps carry frequencies up to the band edge, plain Gauss-Newton leaves mse_rel ~0.54 on them, and
# the network trained on them predicts nothing: its loss stays at the targets' energy).
PAIRS = "smooth"


class PriorWarper:
    """I1 = m(1) of the deformation-state solve (Section 2.3.3) for the template and a velocity v* drawn from
    the prior: iid N(0, 1) band coefficients with the envelope 1 / (1 + 0.1 |k|^2) (synthetic.random_bl_
    coefficients), scaled so that its grid samples move at most max_disp_vox voxels over unit time."""

    def __init__(self, shape=SHAPE, band=BAND, nt=NT, device="cuda:0"):
        import torch
        from . import lddmm_bl as L
        self.torch = torch
        self.shape, self.band = tuple(shape), tuple(band)
        self.ctx = L.Context(L.Problem(n=self.shape, k=self.band, nt=nt, variant=3, precision=L.FP32),
                             device=torch.device(device))

    def velocity(self, seed, max_disp_vox=MAX_DISP_VOX):
        t = self.torch
        v = t.tensor(synthetic.random_bl_coefficients(3, self.band, seed + 104729), dtype=t.float32,
                     device=self.ctx.device)
        g = self.ctx.include(v, 3)
        n = t.tensor(self.shape, dtype=t.float32, device=self.ctx.device).reshape(3, 1, 1, 1)
        return (v * (max_disp_vox / float((g.abs() * n).max()))).contiguous()

    def __call__(self, P, seed, max_disp_vox=MAX_DISP_VOX):
        t = self.torch
        I = t.from_numpy(np.ascontiguousarray(P)).to(self.ctx.device)
        self.ctx.set_images(I, I)
        _, m1 = self.ctx.state_solve(self.velocity(seed, max_disp_vox), want_m1=True)
        return m1.cpu().numpy()


_warpers = {}


def _warper(shape):
    if tuple(shape) not in _warpers:
        _warpers[tuple(shape)] = PriorWarper(shape)
    return _warpers[tuple(shape)]


def render_pair(seed: int, shape=SHAPE, max_disp_vox=MAX_DISP_VOX, mode=None):
    """Seeded phantom pair (I0 template, I1 warped target), float32 [N1][N2][N3]; the "prior" mode runs the
    warp on the GPU in this process."""
    mode = mode or PAIRS
    if mode == "smooth":
        return synthetic.phantom_pair_3d(shape, seed, max_disp_vox=max_disp_vox)
    P, n0, n1 = synthetic.phantom_with_noise_3d(shape, seed)
    return P + n0, _warper(shape)(P, seed, max_disp_vox) + n1


def _render_job(args):
    seed, shape, disp, mode = args
    if mode == "smooth":
        I0, I1 = synthetic.phantom_pair_3d(shape, seed, max_disp_vox=disp)
        return seed, I0, I1, None
    P, n0, n1 = synthetic.phantom_with_noise_3d(shape, seed)
    return seed, P, n0, n1


class PairStream:
    """Renders phantom pairs in worker processes, in seed order (the "prior" targets' warps then run on the
    GPU in this process).

    Create it before the first GPU call of the process: the workers are forked.
    """

    def __init__(self, workers: int = 0, mode=None):
        if workers <= 0:
            workers = max(1, min(16, (os.cpu_count() or 2) - 1))
        self.mode = mode or PAIRS
        self.pool = mp.get_context("fork").Pool(workers)

    def pairs(self, seeds: Sequence[int], shape=SHAPE, max_disp_vox=MAX_DISP_VOX):
        jobs = [(int(s), tuple(shape), float(max_disp_vox), self.mode) for s in seeds]
        for seed, a, b, c in self.pool.imap(_render_job, jobs, chunksize=1):
            if self.mode == "smooth":
                yield seed, a, b
            else:
                yield seed, a + b, _warper(shape)(a, seed, max_disp_vox) + c

    def close(self):
        self.pool.close()
        self.pool.join()


def parse_range(spec: str) -> List[int]:
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


class Registrar:
    """One band-limited registration context plus the helpers of the learned path."""

    def __init__(self, shape=SHAPE, band=BAND, nt=NT, alpha=0.0025, s=2, device="cuda:0", variant=3):
        import torch
        from . import lddmm_bl as L
        self.torch = torch
        self.L = L
        self.device = torch.device(device)
        self.alpha, self.s = alpha, s
        self.band = tuple(band)
        self.variant = variant
        self.ctx = L.Context(L.Problem(n=tuple(shape), k=tuple(band), nt=nt, variant=variant,
                                       alpha=alpha, s=s, precision=L.FP32), device=self.device)

    def set_pair(self, I0, I1):
        t = self.torch
        self.I0 = t.from_numpy(np.ascontiguousarray(I0)).to(self.device)
        self.I1 = t.from_numpy(np.ascontiguousarray(I1)).to(self.device)
        self.ctx.set_images(self.I0, self.I1)

    def zero_velocity(self):
        return self.torch.zeros((3,) + self.band, dtype=self.torch.float32, device=self.device)

    def energy(self, v) -> float:
        E, _ = self.ctx.state_solve(v)
        return E[0]

    def grad_ref(self):
        """Gradient sup-norm and objective at v = 0: the common normalisation of plain and learned
        runs, and the reference of the warm start's fallback test."""
        E, _ = self.ctx.state_solve(self.zero_velocity())
        _, ginf = self.ctx.adjoint_solve()
        return ginf, E[0]

    def solve(self, v, opts: SolveOpts, gref: float, Z=None, energy_target=0.0, ml_inner=0):
        st, rep = self.ctx.gn_solve(v, max_gn=opts.max_gn, max_pcg=opts.max_pcg, grad_rtol=opts.grad_rtol,
                                    grad_ref_inf=gref, Z=Z, energy_target=energy_target, ml_inner=ml_inner)
        rep["status"] = int(st)
        return rep


def target_block(v, block=BLOCK):
    """The low block of velocities [..][3][K..] as a K = block band (pad slots zero): [..][3][b][b][b]."""
    t = v[..., :block, :block, :block].clone()
    t[..., block - 1, :, :] = 0
    t[..., :, block - 1, :] = 0
    t[..., :, :, block - 1] = 0
    return t


def generate(seeds: Sequence[int], opts: SolveOpts, stream: PairStream, log=print, variant=3,
             block=BLOCK) -> Dict[str, np.ndarray]:
    """Plain Gauss-Newton-Krylov on each seeded pair; keeps the converged velocity's low block (block = the
    band of the velocity: every coefficient).

    Returns arrays: seeds, blocks [n][3][b][b][b], energy_full / energy_block (squared V-norms
    of v* and of its block), and per-run statistics of the plain solver.
    """
    from .lddmm_bl import WarmStartNet
    torch = None
    reg = None
    net = None
    out = {k: [] for k in ("seeds", "blocks", "energy_full", "energy_block", "gn_iters", "pcg_iters",
                           "hess_matvecs", "seconds", "grad_inf_rel", "mse_rel", "status", "E0", "E")}
    t0 = time.time()
    for i, (seed, I0, I1) in enumerate(stream.pairs(seeds)):
        if reg is None:
            reg = Registrar(variant=variant)
            torch = reg.torch
            net = WarmStartNet(channels=CHANNELS, in_size=IN_SIZE, seed=0, device=reg.device)
        reg.set_pair(I0, I1)
        gref, _ = reg.grad_ref()
        v = reg.zero_velocity()
        rep = reg.solve(v, opts, gref)
        blk = target_block(v, block)
        zero = torch.zeros(net.out_shape(1), dtype=torch.float32, device=reg.device)
        efull, _ = net.loss(zero, v[None].contiguous(), reg.alpha, reg.s, want_grad=False)
        eblk, _ = net.loss(zero, blk[None].contiguous(), reg.alpha, reg.s, want_grad=False)
        out["seeds"].append(seed)
        out["blocks"].append(blk.cpu().numpy())
        out["energy_full"].append(efull)
        out["energy_block"].append(eblk)
        for k_out, k_rep in (("gn_iters", "gn_iters"), ("pcg_iters", "pcg_iters_total"),
                             ("hess_matvecs", "hess_matvecs"), ("seconds", "seconds"),
                             ("grad_inf_rel", "grad_inf_rel"), ("mse_rel", "mse_rel"), ("status", "status"),
                             ("E0", "E0"), ("E", "E")):
            out[k_out].append(rep[k_rep])
        if i % 25 == 0 or i == len(seeds) - 1:
            log(f"generate {i + 1}/{len(seeds)} seed {seed}: gn {rep['gn_iters']} pcg {rep['pcg_iters_total']} "
                f"grad {rep['grad_inf_rel']:.2e} mse {rep['mse_rel']:.3f} {rep['seconds']:.2f}s "
                f"block/full V-energy {eblk / max(efull, 1e-30):.3f} elapsed {time.time() - t0:.0f}s", flush=True)
    return {k: np.asarray(v) for k, v in out.items()}


def _pool_inputs(net, reg_device, pairs, torch):
    X = torch.empty((len(pairs), 2, IN_SIZE, IN_SIZE, IN_SIZE), dtype=torch.float32, device=reg_device)
    for j, (I0, I1) in enumerate(pairs):
        a = torch.from_numpy(I0).to(reg_device)
        b = torch.from_numpy(I1).to(reg_device)
        net.pool_pair(a, b, X[j])
    return X


def train(net, X, T, epochs: int, batch: int, lr: float, alpha=0.0025, s=2, Xval=None, Tval=None, seed=0,
          log=print):
    """Adam on the mean squared V-norm error of the predicted block (cosine learning-rate decay)."""
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    steps = epochs * max(1, n // batch)
    it = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = torch.from_numpy(perm[b0:b0 + batch]).to(X.device)
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            out = net.forward(xb)
            l, dout = net.loss(out, tb, alpha, s)
            net.zero_grad()
            net.backward(dout)
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * it / steps))
            net.step(lr_t)
            it += 1
            tot += l * batch
            cnt += batch
        rec = {"epoch": ep, "train_loss": tot / max(cnt, 1)}
        if Xval is not None:
            rec["val_loss"] = evaluate_loss(net, Xval, Tval, alpha, s)
        hist.append(rec)
        log(json.dumps(rec), flush=True)
    return hist


def evaluate_loss(net, X, T, alpha=0.0025, s=2, batch=16):
    tot = 0.0
    n = X.shape[0]
    for b0 in range(0, n, batch):
        xb = X[b0:b0 + batch].contiguous()
        tb = T[b0:b0 + batch].contiguous()
        out = net.forward(xb)
        l, _ = net.loss(out, tb, alpha, s, want_grad=False)
        tot += l * xb.shape[0]
    return tot / n


def predict(net, reg: Registrar, x1):
    """Velocity coefficients [3][K..] predicted for one pooled pair x1 [1][2][S^3]."""
    out = net.forward(x1)
    return net.velocity(out, reg.band)[0].contiguous()


def compare(net, reg: Registrar, seeds, stream: PairStream, opts: SolveOpts, log=print, with_Z=True, ml_inner=0):
    """Plain vs learned warm start (and warm start + low-rank preconditioner) on held-out pairs; with
    ml_inner > 0 also the plain start with the two-level spectral preconditioner ("plain_ml")."""
    torch = reg.torch
    rows = []
    for i, (seed, I0, I1) in enumerate(stream.pairs(seeds)):
        reg.set_pair(I0, I1)
        gref, Ez = reg.grad_ref()
        row = {"seed": seed}
        # plain
        v = reg.zero_velocity()
        rep = reg.solve(v, opts, gref)
        row["plain"] = rep
        vstar = v.clone()
        if ml_inner > 0:
            vm = reg.zero_velocity()
            rep = reg.solve(vm, opts, gref, ml_inner=ml_inner)
            rep["seconds_total"] = rep["seconds"]
            rep["reached_plain_E"] = bool(rep["E"] <= row["plain"]["E"])
            row["plain_ml"] = rep
        zero = torch.zeros(net.out_shape(1), dtype=torch.float32, device=reg.device)
        efull, _ = net.loss(zero, vstar[None].contiguous(), reg.alpha, reg.s, want_grad=False)
        # learned
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # timed: the prediction and the fallback test against the objective at v = 0 (known from the
        # normalisation above, which plain and learned runs share)
        x1 = torch.empty((1, 2, IN_SIZE, IN_SIZE, IN_SIZE), dtype=torch.float32, device=reg.device)
        net.pool_pair(reg.I0, reg.I1, x1[0])
        out = net.forward(x1)
        v0 = net.velocity(out, reg.band)[0].contiguous()
        E0 = reg.energy(v0)
        fallback = E0 > Ez
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        # untimed diagnostic: the prediction's V-norm error against the plain solution
        e_pred, _ = net.loss(out, vstar[None].contiguous(), reg.alpha, reg.s, want_grad=False)
        row["pred_vnorm_rel"] = float(np.sqrt(e_pred / max(efull, 1e-30)))
        row["fallback"] = bool(fallback)
        row["t_predict"] = t_pred
        # learned: same gradient tolerance; learned_E: stops at the plain run's final objective as well;
        # learned_Z: gradient tolerance with the two-level preconditioner
        variants = [("learned", None, 0.0), ("learned_E", None, row["plain"]["E"])]
        if with_Z:
            variants.append(("learned_Z", "Z", 0.0))
        for name, zmode, etarget in variants:
            v = reg.zero_velocity() if fallback else v0.clone()
            # each run starts as a deployment would: right after the fallback test, whose state solve at
            # v (already counted in t_pred) the Gauss-Newton solve then reuses instead of repeating
            reg.energy(v)
            Z = None
            if zmode and not fallback:
                Z = torch.zeros((3, 3) + reg.band, dtype=torch.float32, device=reg.device)
                for c in range(3):
                    Z[c, c] = v0[c]
            rep = reg.solve(v, opts, gref, Z=Z, energy_target=etarget)
            rep["reached_plain_E"] = bool(rep["E"] <= row["plain"]["E"])
            rep["seconds_total"] = rep["seconds"] + t_pred
            rep["vnorm_rel_to_plain"] = float(np.sqrt(
                net.loss(zero, (v - vstar)[None].contiguous(), reg.alpha, reg.s, want_grad=False)[0]
                / max(efull, 1e-30)))
            row[name] = rep
        rows.append(row)
        if i % 10 == 0 or i == len(seeds) - 1:
            msg = f"eval {i + 1}/{len(seeds)} seed {seed}: plain gn {row['plain']['gn_iters']} " \
                  f"mv {row['plain']['hess_matvecs']} {row['plain']['seconds']:.2f}s | learned gn " \
                  f"{row['learned']['gn_iters']} mv {row['learned']['hess_matvecs']} " \
                  f"{row['learned']['seconds_total']:.2f}s pred_err {row['pred_vnorm_rel']:.3f} | to plain E gn " \
                  f"{row['learned_E']['gn_iters']} {row['learned_E']['seconds_total']:.2f}s"
            if with_Z:
                msg += f" | +Z gn {row['learned_Z']['gn_iters']} {row['learned_Z']['seconds_total']:.2f}s"
            log(msg, flush=True)
    return rows


def summarize(rows, with_Z=True):
    def agg(name, key):
        return float(np.mean([r[name][key] for r in rows]))
    s = {"pairs": len(rows), "fallbacks": int(sum(r["fallback"] for r in rows)),
         "pred_vnorm_rel_mean": float(np.mean([r["pred_vnorm_rel"] for r in rows]))}
    names = ["plain", "learned", "learned_E"] + (["learned_Z"] if with_Z else []) + \
        (["plain_ml"] if rows and "plain_ml" in rows[0] else [])
    for nme in names:
        key_t = "seconds" if nme == "plain" else "seconds_total"
        tot_t = float(np.sum([r[nme][key_t] for r in rows]))
        s[nme] = {"gn_iters_mean": agg(nme, "gn_iters"), "hess_matvecs_mean": agg(nme, "hess_matvecs"),
                  "pcg_iters_mean": agg(nme, "pcg_iters_total"), "seconds_mean": tot_t / len(rows),
                  "registrations_per_s": len(rows) / tot_t,
                  "grad_inf_rel_max": float(np.max([r[nme]["grad_inf_rel"] for r in rows])),
                  "reached_tol": int(sum(r[nme]["grad_inf_rel"] <= 1e-3 for r in rows)),
                  "reached_plain_E": int(sum(r[nme]["E"] <= r["plain"]["E"] for r in rows)),
                  "E_mean": agg(nme, "E"),
                  "mse_rel_mean": agg(nme, "mse_rel")}
    for nme in names[1:]:
        s[nme]["gn_iter_ratio"] = s["plain"]["gn_iters_mean"] / max(s[nme]["gn_iters_mean"], 1e-9)
        s[nme]["time_ratio"] = s["plain"]["seconds_mean"] / max(s[nme]["seconds_mean"], 1e-9)
        # over the pairs where both runs reached the tolerance
        both = [r for r in rows if r["plain"]["grad_inf_rel"] <= 1e-3 and r[nme]["grad_inf_rel"] <= 1e-3]
        if both:
            key_t = "seconds_total"
            s[nme]["both_reached"] = len(both)
            s[nme]["gn_iter_ratio_both"] = (float(np.mean([r["plain"]["gn_iters"] for r in both]))
                                           / max(float(np.mean([r[nme]["gn_iters"] for r in both])), 1e-9))
            s[nme]["time_ratio_both"] = (float(np.mean([r["plain"]["seconds"] for r in both]))
                                        / max(float(np.mean([r[nme][key_t] for r in both])), 1e-9))
    return s


def save_weights(net, path):
    np.savez(path, params=net.get(0), channels=np.asarray(net.channels), in_size=net.in_size, out_size=net.req_out)


def load_weights(path, device="cuda:0"):
    from .lddmm_bl import WarmStartNet
    z = np.load(path, allow_pickle=False)
    out_size = int(z["out_size"]) if "out_size" in z.files else 0
    net = WarmStartNet(channels=tuple(int(c) for c in z["channels"]), in_size=int(z["in_size"]), device=device,
                       out_size=out_size)
    net.set(z["params"])
    return net


def _main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--seeds", required=True)
    g.add_argument("--out", required=True)
    g.add_argument("--workers", type=int, default=10)
    g.add_argument("--max-gn", type=int, default=20)
    g.add_argument("--max-pcg", type=int, default=10)
    g.add_argument("--variant", type=int, default=3, choices=(1, 3))
    g.add_argument("--pairs", default=PAIRS, choices=("prior", "smooth"))
    g.add_argument("--block", type=int, default=BLOCK, help="band of the stored targets (32: the whole band)")
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--eval-seeds", default="")
    t.add_argument("--weights", required=True)
    t.add_argument("--report", required=True)
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--val-frac", type=float, default=0.05)
    t.add_argument("--workers", type=int, default=0)
    t.add_argument("--max-gn", type=int, default=20)
    t.add_argument("--max-pcg", type=int, default=10)
    t.add_argument("--no-Z", action="store_true")
    t.add_argument("--variant", type=int, default=3, choices=(1, 3))
    t.add_argument("--pairs", default=PAIRS, choices=("prior", "smooth"))
    t.add_argument("--out-size", type=int, default=0,
                   help="output grid of the network (0: in_size / 2^(levels-1)); the targets are cropped to it")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--eval-seeds", required=True)
    e.add_argument("--report", required=True)
    e.add_argument("--workers", type=int, default=0)
    e.add_argument("--max-gn", type=int, default=20)
    e.add_argument("--max-pcg", type=int, default=10)
    e.add_argument("--no-Z", action="store_true")
    e.add_argument("--variant", type=int, default=3, choices=(1, 3))
    e.add_argument("--pairs", default=PAIRS, choices=("prior", "smooth"))
    a = ap.parse_args(argv)
    stream = PairStream(a.workers, a.pairs)  # fork the renderers before the GPU is touched
    opts = SolveOpts(a.max_gn, a.max_pcg)
    try:
        if a.cmd == "generate":
            d = generate(parse_range(a.seeds), opts, stream, variant=a.variant, block=a.block)
            np.savez(a.out, **d)
            print(json.dumps({"pairs": int(d["seeds"].size), "gn_iters_mean": float(d["gn_iters"].mean()),
                              "seconds_mean": float(d["seconds"].mean()),
                              "block_energy_frac": float((d["energy_block"] / d["energy_full"]).mean())}))
            return 0
        import torch
        from .lddmm_bl import WarmStartNet
        if a.cmd == "evaluate":
            reg = Registrar(variant=a.variant)
            net = load_weights(a.weights, device=reg.device)
            rows = compare(net, reg, parse_range(a.eval_seeds), stream, opts, with_Z=not a.no_Z)
            report = {"weights": a.weights, "eval": summarize(rows, with_Z=not a.no_Z), "eval_rows": rows}
            with open(a.report, "w") as f:
                json.dump(report, f, indent=1)
            print(json.dumps(report["eval"], indent=1))
            return 0
        data = [np.load(p, allow_pickle=False) for p in a.data]
        seeds = np.concatenate([d["seeds"] for d in data])
        blocks = np.concatenate([d["blocks"] for d in data]).astype(np.float32)
        ok = np.concatenate([d["status"] for d in data]) >= 0
        seeds, blocks = seeds[ok], blocks[ok]
        reg = Registrar(variant=a.variant)
        net = WarmStartNet(channels=CHANNELS, in_size=IN_SIZE, seed=1234, device=reg.device, out_size=a.out_size)
        if blocks.shape[-1] < net.out_size:
            raise SystemExit(f"targets of band {blocks.shape[-1]} are narrower than the network output {net.out_size}")
        t0 = time.time()
        pairs = []
        X = torch.empty((len(seeds), 2, IN_SIZE, IN_SIZE, IN_SIZE), dtype=torch.float32, device=reg.device)
        for j, (seed, I0, I1) in enumerate(stream.pairs(seeds)):
            net.pool_pair(torch.from_numpy(I0).to(reg.device), torch.from_numpy(I1).to(reg.device), X[j])
            if j % 250 == 0:
                print(f"inputs {j + 1}/{len(seeds)} {time.time() - t0:.0f}s", flush=True)
        T = target_block(torch.from_numpy(blocks).to(reg.device), net.out_size).contiguous()
        nval = max(1, int(a.val_frac * len(seeds)))
        Xtr, Ttr, Xva, Tva = X[nval:], T[nval:], X[:nval], T[:nval]
        t1 = time.time()
        hist = train(net, Xtr, Ttr, a.epochs, a.batch, a.lr, Xval=Xva, Tval=Tva)
        t_train = time.time() - t1
        save_weights(net, a.weights)
        report = {"train_pairs": int(Xtr.shape[0]), "val_pairs": nval, "epochs": a.epochs, "batch": a.batch,
                  "lr": a.lr, "out_size": net.out_size, "train_seconds": t_train, "history": hist}
        del X
        if a.eval_seeds:
            rows = compare(net, reg, parse_range(a.eval_seeds), stream, opts, with_Z=not a.no_Z)
            report["eval"] = summarize(rows, with_Z=not a.no_Z)
            report["eval_rows"] = rows
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)
        print(json.dumps(report.get("eval", {}), indent=1))
        return 0
    finally:
        stream.close()


if __name__ == "__main__":
    sys.exit(_main())
