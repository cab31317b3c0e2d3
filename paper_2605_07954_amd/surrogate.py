"""Training and evaluation driver of the CNN surrogate.

Host-side sequencing only: training is one C-ABI call per chunk of optimiser steps
(``surrogate_train``: field synthesis, the plain variable-coefficient stencil that generates the
targets, crops, the MFMA forward and backward passes and Adam all run in the library's kernels),
and evaluation is ``surrogate_infer_checked``, whose judge is the plain stencil.  The host draws
the random numbers -- field coefficients and crop offsets -- and passes them in.

One optimiser step on a batch of B trajectories:
  1. synthesise (u0, kappa) on the full grid from per-trajectory coefficient rows;
  2. target u_K = K plain steps of the varcoef stencil (the generator is the method itself);
  3. crop a random window of each field (u0, kappa, u_K);
  4. masked MSE of u_hat = surrogate(u0, kappa) against u_K, full backward pass;
  5. Adam step with a cosine learning-rate schedule.
Cells closer than the receptive-field radius (6) to a crop edge that is not a grid edge are left
out of the loss: their true inputs lie outside the crop.
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

from . import (SG_JUDGE_FULL, SG_PARAM_COUNT, stencil_destroy, stencil_plan_varcoef, stencil_set_blocking,
               surrogate_checked_ws_bytes, surrogate_create, surrogate_destroy, surrogate_infer_checked,
               surrogate_init, surrogate_synth_fields, surrogate_train, surrogate_train_ws_bytes)


class Trainer:
    def __init__(self, grid: int = 1024, crop: int = 256, batch: int = 8, K: int = 16, seed: int = 0,
                 device: str = "cuda", chunk: int = 50):
        import torch
        self.torch = torch
        self.grid, self.crop, self.batch, self.K, self.seed, self.chunk = grid, crop, batch, K, seed, chunk
        self.dev = device
        self.model = surrogate_create()
        self.params = torch.empty(SG_PARAM_COUNT, dtype=torch.float32, device=device)
        self.optim = torch.empty(2 * SG_PARAM_COUNT, dtype=torch.float32, device=device)
        surrogate_init(self.model, self.params, self.optim, seed)  # seeded He-normal weights, zero Adam state
        self.ws = torch.empty(surrogate_train_ws_bytes(self.model, grid, grid, crop, batch, K, chunk),
                              dtype=torch.uint8, device=device)
        self.rng = np.random.default_rng(seed + 12345)
        self.judge = None

    def close(self):
        if self.judge is not None:
            stencil_destroy(self.judge)
        surrogate_destroy(self.model)

    def draws(self, k0: int, n: int):
        """Coefficient rows and crop offsets of optimiser steps k0 .. k0+n-1 (host random numbers)."""
        coef = np.concatenate([_coefficients(self.batch, 100_000 + self.seed * 1_000_003 + k) for k in range(k0, k0 + n)])
        yx = self.rng.integers(0, self.grid - self.crop + 1, size=(n * self.batch, 2)).astype(np.int32)
        return coef, yx

    def train(self, n_traj: int, lr: float = 1e-3, log_every: int | None = None, log=print):
        torch = self.torch
        steps = max(1, n_traj // self.batch)
        chunk = min(self.chunk, log_every or self.chunk)
        history = []
        t0 = time.perf_counter()
        for k0 in range(0, steps, chunk):
            n = min(chunk, steps - k0)
            coef, yx = self.draws(k0, n)
            losses = torch.zeros(n, dtype=torch.float64, device=self.dev)
            surrogate_train(self.model, self.params, self.optim, torch.from_numpy(coef).to(self.dev), yx, losses, self.ws,
                            self.grid, self.grid, self.crop, self.batch, self.K, n, k0, steps, lr)
            lv = float(losses[-1].cpu())
            history.append((k0 + n, lv))
            if log is print:
                print(f"step {k0 + n}/{steps}  trajectories {(k0 + n) * self.batch}  loss {lv:.4e}  "
                      f"{time.perf_counter() - t0:.1f} s", flush=True)
            elif log is not None:
                log(k0 + n, lv)
        return history

    def evaluate(self, params, n: int, seed: int = 7, judge_mode: int = SG_JUDGE_FULL):
        """Held-out rel-L2 against K plain steps (from the library's judged entry point, whole field
        by default) of the surrogate with `params` and of the identity predictor u_hat = u0
        (all-zero parameters)."""
        torch = self.torch
        G = self.grid
        if self.judge is None:
            self.judge = stencil_plan_varcoef(G, G, 0.0, 0)
            for tb in (8, 4, 2, 1):
                try:
                    stencil_set_blocking(self.judge, tb)
                    break
                except Exception:  # noqa: BLE001 - deeper blocks may not fit this device's LDS
                    continue
        cws = torch.empty(surrogate_checked_ws_bytes(self.model, G, G), dtype=torch.uint8, device=self.dev)
        zero = torch.zeros(SG_PARAM_COUNT, dtype=torch.float32, device=self.dev)
        U0 = torch.empty((self.batch, G, G), dtype=torch.float32, device=self.dev)
        KP = torch.empty_like(U0)
        out = torch.empty((G, G), dtype=torch.float32, device=self.dev)
        errs, ident = [], []
        coef_all = _coefficients(n, seed)
        for k in range(0, n, self.batch):
            coef = coef_all[k:k + self.batch]
            surrogate_synth_fields(torch.from_numpy(np.ascontiguousarray(coef, np.float32)).to(self.dev), coef.shape[0],
                                   G, G, U0, KP)
            for b in range(coef.shape[0]):
                _, e = surrogate_infer_checked(self.model, params, U0[b], KP[b], out, G, G, self.judge, self.K,
                                               float("inf"), cws, judge_mode)
                _, i = surrogate_infer_checked(self.model, zero, U0[b], KP[b], out, G, G, self.judge, self.K,
                                               float("inf"), cws, judge_mode)
                errs.append(e)
                ident.append(i)
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
    tr = Trainer(grid=args.grid, crop=args.crop, batch=args.batch, chunk=50)
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
