"""Training and evaluation driver of the CNN surrogate.

Host-side sequencing only: every arithmetic step runs in the library's kernels (field synthesis,
the plain variable-coefficient stencil that generates the targets, crops, the MFMA forward and
backward passes, Adam).  The host draws the random numbers -- field coefficients and crop
offsets -- and passes them in.

One training step on a batch of B trajectories:
  1. synthesise (u0, kappa) on the full grid from per-trajectory coefficient rows;
  2. target u_K = K plain steps of the varcoef stencil (the generator is the method itself);
  3. crop a random window of each field (u0, kappa, u_K);
  4. masked MSE of u_hat = surrogate(u0, kappa) against u_K, full backward pass;
  5. Adam step with a cosine learning-rate schedule.
Cells closer than the receptive-field radius (6) to a crop edge that is not a grid edge are left
out of the loss: their true inputs lie outside the crop.

The plain stencil stays the judge: ``evaluate`` reports the held-out rel-L2 of the surrogate
against K plain steps, and ``surrogate_infer_checked`` (C ABI) falls back to the plain result.
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

from . import (SG_PARAM_COUNT, ST_FLAG_GRAPH, stencil_destroy, stencil_plan_varcoef, stencil_run_varcoef,
               stencil_set_blocking, stencil_workspace_bytes, surrogate_adam, surrogate_create, surrogate_crop,
               surrogate_destroy, surrogate_forward, surrogate_loss_grad, surrogate_synth_fields,
               surrogate_workspace_bytes)

CHANNELS = (2, 32, 32, 32, 32, 32, 1)
RF = 6  # receptive-field radius of six 3x3 layers


def init_params(seed: int) -> np.ndarray:
    """He-normal weights N(0, 2 / (9 C_in)) in the library layout ([ky][kx][ci][co] then bias), zero
    biases; the last layer is scaled by 0.1 so the untrained surrogate starts near u_hat = u0."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(6):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == 5 else 1.0)
        out.append(rng.normal(0.0, std, size=(3, 3, ci, co)).reshape(-1))
        out.append(np.zeros(co))
    v = np.concatenate(out).astype(np.float32)
    assert v.size == SG_PARAM_COUNT
    return v


def crop_lohi(y0: int, x0: int, crop: int, grid: int) -> list[int]:
    return [RF if y0 > 0 else 0, crop - (RF if y0 + crop < grid else 0),
            RF if x0 > 0 else 0, crop - (RF if x0 + crop < grid else 0)]


class Trainer:
    def __init__(self, grid: int = 1024, crop: int = 256, batch: int = 8, K: int = 16, seed: int = 0,
                 device: str = "cuda"):
        import torch
        self.torch = torch
        self.grid, self.crop, self.batch, self.K, self.seed = grid, crop, batch, K, seed
        dev = self.dev = device
        f32 = torch.float32
        self.model = surrogate_create()
        self.judge = stencil_plan_varcoef(grid, grid, 0.0, ST_FLAG_GRAPH)
        for tb in (8, 4, 2, 1):
            try:
                stencil_set_blocking(self.judge, tb)
                break
            except Exception:  # noqa: BLE001 - deeper blocks may not fit this device's LDS
                continue
        self.U0 = torch.empty((batch, grid, grid), dtype=f32, device=dev)
        self.KP = torch.empty_like(self.U0)
        self.UK = torch.empty_like(self.U0)
        self.jws = torch.empty(max(stencil_workspace_bytes(self.judge, K), 4), dtype=torch.uint8, device=dev)
        self.cu0 = torch.empty((batch, crop, crop), dtype=f32, device=dev)
        self.ckp = torch.empty_like(self.cu0)
        self.cuk = torch.empty_like(self.cu0)
        self.ws = torch.empty(surrogate_workspace_bytes(self.model, batch, crop, crop), dtype=torch.uint8,
                              device=dev)
        self.params = torch.from_numpy(init_params(seed)).to(dev)
        self.grad = torch.zeros(SG_PARAM_COUNT, dtype=f32, device=dev)
        self.optim = torch.zeros(2 * SG_PARAM_COUNT, dtype=f32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.t = 0

    def close(self):
        stencil_destroy(self.judge)
        surrogate_destroy(self.model)

    def make_targets(self, coef: np.ndarray):
        """Synthesise B trajectories' (u0, kappa) on the full grid and advance them K plain steps."""
        torch = self.torch
        n = coef.shape[0]
        surrogate_synth_fields(torch.from_numpy(np.ascontiguousarray(coef, np.float32)).to(self.dev), n,
                               self.grid, self.grid, self.U0, self.KP)
        for b in range(n):
            stencil_run_varcoef(self.judge, self.U0[b], self.KP[b], self.UK[b], self.K, self.jws)

    def step(self, coef: np.ndarray, offsets: np.ndarray, lr: float) -> None:
        torch = self.torch
        self.make_targets(coef)
        yx = torch.from_numpy(np.ascontiguousarray(offsets, np.int32)).to(self.dev)
        B, G, C = self.batch, self.grid, self.crop
        for src, dst in ((self.U0, self.cu0), (self.KP, self.ckp), (self.UK, self.cuk)):
            surrogate_crop(src, dst, yx, B, G, G, C, C)
        lohi = [v for (y0, x0) in offsets for v in crop_lohi(int(y0), int(x0), C, G)]
        surrogate_loss_grad(self.model, self.params, self.cu0, self.ckp, self.cuk, lohi, B, C, C, self.grad,
                            self.loss, self.ws)
        self.t += 1
        surrogate_adam(self.model, self.params, self.grad, self.optim, self.t, lr)

    def train(self, n_traj: int, lr: float = 1e-3, log_every: int = 50, log=print):
        steps = max(1, n_traj // self.batch)
        rng = np.random.default_rng(self.seed + 12345)
        losses = []
        t0 = time.perf_counter()
        for k in range(steps):
            coef = _coefficients(self.batch, 100_000 + self.seed * 1_000_003 + k)
            offs = rng.integers(0, self.grid - self.crop + 1, size=(self.batch, 2))
            lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))
            self.step(coef, offs, lr_k)
            if (k + 1) % log_every == 0 or k == steps - 1:
                lv = float(self.loss.cpu()[0])
                losses.append((k + 1, lv))
                log(f"step {k + 1}/{steps}  trajectories {(k + 1) * self.batch}  loss {lv:.4e}  "
                    f"{time.perf_counter() - t0:.1f} s", flush=True) if log is print else log(k + 1, lv)
        return losses

    def evaluate(self, params, n: int, seed: int = 7):
        """Held-out rel-L2 of the surrogate, of the identity predictor (u_hat = u0), against K plain steps."""
        torch = self.torch
        G = self.grid
        fws = torch.empty(surrogate_workspace_bytes(self.model, 1, G, G), dtype=torch.uint8, device=self.dev)
        uh = torch.empty((1, G, G), dtype=torch.float32, device=self.dev)
        errs, ident = [], []
        coef_all = _coefficients(n, seed)
        for k in range(0, n, self.batch):
            coef = coef_all[k:k + self.batch]
            self.make_targets(coef)
            for b in range(coef.shape[0]):
                surrogate_forward(self.model, params, self.U0[b], self.KP[b], uh, 1, G, G, fws)
                d = (uh[0].double() - self.UK[b].double()).norm() / self.UK[b].double().norm()
                i = (self.U0[b].double() - self.UK[b].double()).norm() / self.UK[b].double().norm()
                errs.append(float(d))
                ident.append(float(i))
        return np.array(errs), np.array(ident)


def _coefficients(n: int, seed: int) -> np.ndarray:
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    return workloads.field_coefficients(n, seed)


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the CNN surrogate on GPU-generated trajectories")
    ap.add_argument("--trajectories", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--heldout", type=int, default=1000)
    ap.add_argument("--out", default=None, help="write the trained parameters (.npy) and a JSON summary here")
    args = ap.parse_args(argv)
    tr = Trainer(grid=args.grid, crop=args.crop, batch=args.batch)
    try:
        p0 = tr.params.clone()
        t0 = time.perf_counter()
        losses = tr.train(args.trajectories, lr=args.lr)
        train_s = time.perf_counter() - t0
        e_tr, e_id = tr.evaluate(tr.params, args.heldout)
        e_un, _ = tr.evaluate(p0, min(args.heldout, 64))
        summary = {"trajectories": args.trajectories, "batch": args.batch, "grid": args.grid, "crop": args.crop,
                   "train_s": train_s, "final_loss": losses[-1][1],
                   "heldout": args.heldout, "rel_l2_trained_mean": float(e_tr.mean()),
                   "rel_l2_trained_max": float(e_tr.max()), "rel_l2_identity_mean": float(e_id.mean()),
                   "rel_l2_untrained_mean": float(e_un.mean())}
        print(json.dumps(summary), flush=True)
        if args.out:
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            np.save(args.out + ".npy", tr.params.cpu().numpy())
            with open(args.out + ".json", "w") as f:
                json.dump({"summary": summary, "losses": losses}, f)
    finally:
        tr.close()


if __name__ == "__main__":
    main()
