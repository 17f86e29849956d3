"""Host orchestration for learning the swept-volume network (paper Sec. IV-C, Sec. V).

The arithmetic runs in libsv's kernels: sv_make_samples draws and labels the
training rows with the exact check, sv_train_step does forward, loss, backward and
Adam on the GPU, sv_nn_predict evaluates the network on held-out rows.  This
module only sequences those calls: motion batches for data generation, a seeded
shuffle per epoch, batch slicing, and bookkeeping.

Recipes (synthetic stand-ins for the paper's datasets): motions with q0, q1 uniform
within the joint limits; labels are exact swept distances at T samples; held-out
motions give the validation rows (the paper splits its data by motion, Sec. V-A).
  DataRecipe: per motion n_uniform points uniform in the 1.2 m cube and n_near points
    within `band` of the swept surface (the 50/50 scheme);
  PaperRecipe: the paper's own proportions (Sec. IV-C): uniform box points, swept-
    surface points, two Gaussian points and one chord point per surface point.
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
    """Adam at lr (Sec. V: PyTorch's defaults) for `epochs` passes over the rows.

    schedule: "constant"; "plateau": the learning rate is multiplied by
    plateau_factor after plateau_patience epochs without a new best held-out loss
    (the paper's ReduceLROnPlateau with factor 0.1 and patience 10 over 200 epochs,
    Sec. V; needs validation rows); "cosine": lr (1 + cos(pi s / S)) / 2 at step s of
    S.  keep_best: end with the weights of the epoch
    with the best held-out loss (the paper tests the checkpoint with the best
    validation loss).  clamp_pred: clamp the predictions in the loss as well as the
    targets (sv_train_hparams.clamp_pred)."""
    epochs: int = 20
    batch: int = 65536
    lr: float = 1e-3
    clamp_sigma: float = 0.1
    seed: int = 7
    schedule: str = "constant"
    plateau_factor: float = 0.1
    plateau_patience: int = 10
    keep_best: bool = False
    clamp_pred: bool = False


@dataclass
class TrainLog:
    epoch_loss: list = field(default_factory=list)
    val_mae: list = field(default_factory=list)
    lr: list = field(default_factory=list)
    best_epoch: int = -1
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


@dataclass
class PaperRecipe:
    """The paper's training distribution (Sec. IV-C) at a fixed row budget per motion.

    The paper draws 0.25 points per dm^3 uniformly in a box covering every motion and
    0.2 points per cm^2 on the swept surface, each with 2 Gaussian points (sigma 3 mm)
    and 1 chord point.  Here the box is the training cube and the per-motion counts keep
    those densities' proportions for the mean swept-surface area of the motions
    (estimated on a pilot batch), scaled to rows_per_motion."""
    n_motions: int = 20000
    rows_per_motion: int = 500
    cube_half: float = 0.6
    sigma: float = 0.003
    T: int = 256
    cand_per_surface: int = 60
    uniform_per_m3: float = 250.0      # 0.25 per dm^3
    surface_per_m2: float = 2000.0     # 0.2 per cm^2
    chunk: int = 1000


def capsule_area_total(arm, device="cuda") -> float:
    """Sum of the capsules' surface areas (rigid, so any configuration; from sv_fk)."""
    robot = sv.make_robot(arm)
    q = torch.zeros(1, arm.dof, dtype=torch.float32, device=device)
    caps = torch.empty(1, arm.n_caps, 8, dtype=torch.float32, device=device)
    sv.sv_fk(robot, q, caps)
    c = caps[0].double().cpu().numpy()
    L = np.linalg.norm(c[:, 3:6] - c[:, 0:3], axis=1)
    r = c[:, 6]
    return float(np.sum(2 * math.pi * r * L + 4 * math.pi * r * r))


def swept_area_estimate(arm, recipe: PaperRecipe, seed: int, n: int = 200, n_cand: int = 4000, device="cuda") -> float:
    """Mean swept-surface area (m^2) of n motions: the accepted share of surface
    candidates times the total area of the T capsule instances."""
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, n, recipe.T, seed)
    dm = sv.DeviceMotions(mo, device)
    rnd = torch.as_tensor(svgen.uniforms(seed * 7919 + 1, n, 5 * n_cand + 8), device=device)
    out = torch.empty(n, 4, 3 + 2 * arm.dof + 1, dtype=torch.float32, device=device)
    acc = torch.zeros(n, dtype=torch.int32, device=device)
    sv.sv_make_samples_paper(robot, dm, recipe.cube_half, 0, 1, n_cand, recipe.sigma, rnd, out, acc)
    frac = acc.double().mean().item() / n_cand
    return frac * recipe.T * capsule_area_total(arm, device)


def paper_counts(recipe: PaperRecipe, area_m2: float):
    """(n_uniform, n_surface) with the paper's density proportions within rows_per_motion."""
    nu0 = recipe.uniform_per_m3 * (2 * recipe.cube_half) ** 3
    ns0 = recipe.surface_per_m2 * area_m2
    ns = max(1, int(round(recipe.rows_per_motion * ns0 / (nu0 + 4 * ns0))))
    return recipe.rows_per_motion - 4 * ns, ns


def make_dataset_paper(arm, recipe: PaperRecipe, seed: int, area_m2: float = None, device="cuda"):
    """Training rows in the paper's proportions: (rows [S][in_dim + 1], n_short, info)."""
    if area_m2 is None:
        area_m2 = swept_area_estimate(arm, recipe, seed + 17, device=device)
    nu, ns = paper_counts(recipe, area_m2)
    nc = recipe.cand_per_surface * ns
    robot = sv.make_robot(arm)
    per = nu + 4 * ns
    width = 3 + 2 * arm.dof + 1
    out = torch.empty(recipe.n_motions * per, width, dtype=torch.float32, device=device)
    n_short = torch.zeros(1, dtype=torch.int32, device=device)
    motions = svgen.make_motions(arm, recipe.n_motions, recipe.T, seed)
    cols = 3 * nu + 5 * nc + 8 * ns
    ws = None
    for c0 in range(0, recipe.n_motions, recipe.chunk):
        c1 = min(recipe.n_motions, c0 + recipe.chunk)
        sub = svgen.Motions(motions.q0[c0:c1], motions.q1[c0:c1], recipe.T)
        dm = sv.DeviceMotions(sub, device)
        if ws is None:   # chunks only shrink, so the first chunk's workspace serves all of them
            ws = sv.workspace(sv_paper_ws(robot, dm, nu, ns, nc))
        rnd = torch.as_tensor(svgen.uniforms(seed * 1000003 + c0, c1 - c0, cols), device=device)
        sv.sv_make_samples_paper(robot, dm, recipe.cube_half, nu, ns, nc, recipe.sigma, rnd,
                                 out[c0 * per:c1 * per], None, n_short, ws=ws)
    torch.cuda.synchronize()
    return out, int(n_short.item()), {"area_m2": area_m2, "n_uniform": nu, "n_surface": ns, "n_cand": nc}


def sv_paper_ws(robot, dm, nu, ns, nc) -> int:
    import ctypes
    n = ctypes.c_size_t(0)
    d = dm.desc()
    sv._check(sv.lib.sv_make_samples_paper_workspace_size(ctypes.byref(robot), ctypes.byref(d), nu, ns, nc,
                                                          ctypes.byref(n)))
    return n.value


def init_params(spec: svgen.MLPSpec, seed: int) -> np.ndarray:
    """Seeded initialisation for training: the uniform(+-1/sqrt(fan_in)) init with the
    output layer scaled by 0.1, so that initial predictions fall inside the loss clamp
    [-sigma, sigma] (outside it the clamped loss passes no gradient)."""
    flat = svgen.mlp_init(spec, seed)
    flat[-(spec.width + 1):] *= np.float32(0.1)
    return flat


def init_params_res(spec: svgen.ResSpec, seed: int) -> np.ndarray:
    """Seeded initialisation of the residual network for training: linear layers
    uniform(+-1/sqrt(fan_in)) as svgen.res_init draws them, BatchNorm layers as PyTorch
    creates them (gamma 1, beta 0, running mean 0, running variance 1), the output layer
    scaled by 0.1 as in init_params."""
    flat = svgen.res_init(spec, seed)
    W, i = spec.width, spec.in_dim
    for b in range(spec.n_blocks):
        base = W * i + W + b * (W * W + W * i + 5 * W) + W * W + W * i
        flat[base + W:base + 2 * W] = 1.0        # gamma
        flat[base + 2 * W:base + 3 * W] = 0.0    # beta
        flat[base + 3 * W:base + 4 * W] = 0.0    # running mean
        flat[base + 4 * W:base + 5 * W] = 1.0    # running variance
    flat[-(W + 1):] *= np.float32(0.1)
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

    # The seeded sample order of each epoch, drawn on the device in stream order: a host
    # permutation of 10M rows (about 0.2 s) outlasts a whole epoch of steps (0.17 s at
    # 1.1 ms per step) and left the GPU waiting at every epoch boundary.
    gen = torch.Generator(device=device)
    gen.manual_seed(recipe.seed)

    def epoch_order(ep):
        return torch.randperm(n, generator=gen, device=device, dtype=torch.int32)

    if recipe.schedule not in ("constant", "plateau", "cosine"):
        raise ValueError(f"unknown schedule {recipe.schedule!r}")
    if (recipe.schedule == "plateau" or recipe.keep_best) and val_rows is None:
        raise ValueError("the plateau schedule and keep_best need validation rows")
    lr = recipe.lr
    best, since_best, best_params = math.inf, 0, None
    order = epoch_order(0)
    for ep in range(recipe.epochs):
        perm = order
        ep_loss = torch.zeros(1, dtype=torch.float32, device=device)
        tl.lr.append(lr)
        for s in range(steps_per_epoch):
            idx = perm[s * recipe.batch:(s + 1) * recipe.batch]
            step += 1
            if recipe.schedule == "cosine":
                lr = recipe.lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / (recipe.epochs * steps_per_epoch)))
            sv.sv_train_step(mlp, m, v, step, samples, idx, lr=lr, clamp_sigma=recipe.clamp_sigma,
                             loss_out=loss, ws=ws, clamp_pred=recipe.clamp_pred)
            ep_loss.add_(loss, alpha=idx.shape[0])
        if ep + 1 < recipe.epochs:
            order = epoch_order(ep + 1)
        tl.epoch_loss.append(float(ep_loss.item()) / n)
        if val_rows is not None:
            tl.val_mae.append(val_mae(mlp, val_rows, recipe.clamp_sigma))
            if tl.val_mae[-1] < best:
                best, since_best, tl.best_epoch = tl.val_mae[-1], 0, ep
                if recipe.keep_best:
                    best_params = mlp.params.clone()
            else:
                since_best += 1
                if recipe.schedule == "plateau" and since_best > recipe.plateau_patience:
                    lr *= recipe.plateau_factor
                    since_best = 0
        if log:
            log(f"epoch {ep + 1}/{recipe.epochs}: lr {tl.lr[-1]:.1e}, loss {tl.epoch_loss[-1]:.5f}"
                + (f", val clamped MAE {tl.val_mae[-1] * 1e3:.2f} mm" if val_rows is not None else ""))
    if best_params is not None:
        mlp.params.copy_(best_params)
    torch.cuda.synchronize()
    tl.steps = step
    tl.seconds = time.perf_counter() - t0
    return tl
