"""Host orchestration for learning the swept-volume network (paper Sec. IV-C, Sec. V).

The arithmetic runs in libsv's kernels: sv_make_samples draws and labels the
training rows with the exact check, sv_train_step does forward, loss, backward and
Adam on the GPU, sv_nn_predict evaluates the network on held-out rows.  This
module only sequences those calls: motion batches for data generation, a seeded
shuffle per epoch, batch slicing, and bookkeeping.

Recipe (synthetic stand-in for the paper's datasets): motions with q0, q1 uniform
within the joint limits; per motion n_uniform points uniform in the 1.2 m cube and
n_near points within `band` of the swept surface; labels are exact swept
distances at T samples; held-out motions give the validation rows (the paper
splits its data by motion, Sec. V-A).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import svgen
from paper_2402_15281_amd import _binding as sv


@dataclass
class DataRecipe:
    n_motions: int = 20000
    n_uniform: int = 250
    n_near: int = 250
    n_cand: int = 1000
    band: float = 0.05
    cube_half: float = 0.6
    T: int = 256
    chunk: int = 2000


@dataclass
class TrainRecipe:
    epochs: int = 20
    batch: int = 65536
    lr: float = 1e-3
    clamp_sigma: float = 0.1
    seed: int = 7


@dataclass
class TrainLog:
    epoch_loss: list = field(default_factory=list)
    val_mae: list = field(default_factory=list)
    steps: int = 0
    seconds: float = 0.0
    n_short: int = 0


def make_dataset(arm, recipe: DataRecipe, seed: int, device="cuda"):
    """Training rows [S][in_dim + 1] on the device, S = n_motions (n_uniform + n_near)."""
    robot = sv.make_robot(arm)
    per = recipe.n_uniform + recipe.n_near
    width = 3 + 2 * arm.dof + 1
    out = torch.empty(recipe.n_motions * per, width, dtype=torch.float32, device=device)
    n_short = torch.zeros(1, dtype=torch.int32, device=device)
    motions = svgen.make_motions(arm, recipe.n_motions, recipe.T, seed)
    cols = 3 * recipe.n_uniform + 6 * recipe.n_cand
    ws = None
    for c0 in range(0, recipe.n_motions, recipe.chunk):
        c1 = min(recipe.n_motions, c0 + recipe.chunk)
        sub = svgen.Motions(motions.q0[c0:c1], motions.q1[c0:c1], recipe.T)
        dm = sv.DeviceMotions(sub, device)
        rnd = torch.as_tensor(svgen.uniforms(seed * 1000003 + c0, c1 - c0, cols), device=device)
        # chunks only shrink, so the first chunk's workspace serves all of them
        ws = sv.sv_make_samples(robot, dm, recipe.cube_half, recipe.n_uniform, recipe.n_near, recipe.n_cand,
                                recipe.band, rnd, out[c0 * per:c1 * per], n_short, ws=ws)
    torch.cuda.synchronize()
    return out, int(n_short.item())


def init_params(spec: svgen.MLPSpec, seed: int) -> np.ndarray:
    """Seeded initialisation for training: the uniform(+-1/sqrt(fan_in)) init with the
    output layer scaled by 0.1, so that initial predictions fall inside the loss clamp
    [-sigma, sigma] (outside it the clamped loss passes no gradient)."""
    flat = svgen.mlp_init(spec, seed)
    flat[-(spec.width + 1):] *= np.float32(0.1)
    return flat


def predict(mlp, rows, precision=sv.SV_BF16):
    out = torch.empty(rows.shape[0], dtype=torch.float32, device=rows.device)
    sv.sv_nn_predict(mlp, precision, rows, out)
    return out


def evaluate(mlp, val_rows, sigma=0.1, precision=sv.SV_BF16) -> dict:
    """Held-out errors: clamped MAE (the training loss), MAE on rows with |delta| <=
    sigma (near the swept surface), and MAE over all rows."""
    in_dim = val_rows.shape[1] - 1
    pred = predict(mlp, val_rows, precision)
    d = val_rows[:, in_dim]
    err = torch.abs(pred - d)
    near = torch.abs(d) <= sigma
    clamped = torch.abs(torch.clamp(pred, -sigma, sigma) - torch.clamp(d, -sigma, sigma))
    return {"mae_clamped": float(clamped.mean().item()), "mae_near": float(err[near].mean().item()),
            "mae_all": float(err.mean().item()), "near_fraction": float(near.float().mean().item())}


def val_mae(mlp, val_rows, sigma=0.1, precision=sv.SV_BF16) -> float:
    return evaluate(mlp, val_rows, sigma, precision)["mae_clamped"]


def train(mlp, samples, recipe: TrainRecipe, val_rows=None, log=None, device="cuda") -> TrainLog:
    """Adam on the FP32 masters of `mlp` (updated in place) over `samples`."""
    n = samples.shape[0]
    n_params = mlp.params.numel()
    m = torch.zeros(n_params, dtype=torch.float32, device=device)
    v = torch.zeros(n_params, dtype=torch.float32, device=device)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    ws = sv.workspace(sv.sv_train_workspace_size(mlp, recipe.batch))
    steps_per_epoch = math.ceil(n / recipe.batch)
    tl = TrainLog()
    step = 0
    t0 = time.perf_counter()

    def epoch_order(ep):
        # the seeded sample order of one epoch, staged in pinned memory so that its copy
        # to the device is queued behind the running steps instead of waiting for them
        return torch.from_numpy(svgen.permutation(recipe.seed * 7919 + ep, n)).pin_memory()

    order = epoch_order(0)
    for ep in range(recipe.epochs):
        perm = order.to(device, non_blocking=True)
        ep_loss = torch.zeros(1, dtype=torch.float32, device=device)
        for s in range(steps_per_epoch):
            idx = perm[s * recipe.batch:(s + 1) * recipe.batch]
            step += 1
            sv.sv_train_step(mlp, m, v, step, samples, idx, lr=recipe.lr, clamp_sigma=recipe.clamp_sigma,
                             loss_out=loss, ws=ws)
            ep_loss += loss * idx.shape[0]
        if ep + 1 < recipe.epochs:
            order = epoch_order(ep + 1)       # on the host while the GPU runs this epoch
        tl.epoch_loss.append(float(ep_loss.item()) / n)
        if val_rows is not None:
            tl.val_mae.append(val_mae(mlp, val_rows, recipe.clamp_sigma))
        if log:
            log(f"epoch {ep + 1}/{recipe.epochs}: loss {tl.epoch_loss[-1]:.5f}"
                + (f", val clamped MAE {tl.val_mae[-1] * 1e3:.2f} mm" if val_rows is not None else ""))
    torch.cuda.synchronize()
    tl.steps = step
    tl.seconds = time.perf_counter() - t0
    return tl
