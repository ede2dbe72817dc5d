"""Training and use of the template-proposal network (orchestration only).

Every computation runs in the HIP library: labels come from the full FTK
search (ftk_align + ftk_best_template), features from ftk_features,
training from ftk_mlp_train_step, the search from ftk_align_proposed.  This
module sequences those calls; the few host-side numbers it forms (feature
mean and spread for the input standardisation, the confidence threshold)
are statistics of the training data, computed once before training.
"""
from __future__ import annotations

import numpy as np

from . import ftk as F


def shift_bins(shifts_px, spacing_px: float = 0.5) -> np.ndarray:
    """Radius bin of every shift: round(|delta| / spacing)."""
    sh = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2)
    return np.rint(np.hypot(sh[:, 0], sh[:, 1]) / spacing_px).astype(np.int32)


def ftk_labels(plan: F.Plan, images, templates, shift_bin: np.ndarray, chunk: int = 4096, stream=None):
    """Full-FTK labels of device images [nI][n][n] against device templates:
    (best template [nI], shift-radius bin of the best pose [nI], best pose
    [nI][3]) as device int32 tensors."""
    import torch
    nI = images.shape[0]
    tc = plan.transform(templates, stream=stream)
    lab_t = torch.empty(nI, dtype=torch.int32, device=images.device)
    pose = torch.empty((nI, 3), dtype=torch.int32, device=images.device)
    for i0 in range(0, nI, chunk):
        ic = plan.transform(images[i0:i0 + chunk], stream=stream)
        _, best = plan.align_coeffs(ic, tc, stream=stream)
        bt, bp = F.best_template(best, stream=stream)
        lab_t[i0:i0 + chunk] = bt
        pose[i0:i0 + chunk] = bp
    sb = torch.as_tensor(shift_bin, dtype=torch.int32, device=images.device)
    lab_s = sb[pose[:, 1].long()]
    return lab_t, lab_s, pose


def input_norm(feats: np.ndarray):
    """Per-feature mean and inverse spread of the training features."""
    f = np.asarray(feats, dtype=np.float64)
    mu = f.mean(axis=0)
    sd = f.std(axis=0)
    return mu.astype(np.float32), (1.0 / np.maximum(sd, 1e-12 * max(sd.max(), 1e-30))).astype(np.float32)


def train(net: F.MLP, feats, lab_t, lab_s, perms, batch: int, lr: float, wd: float = 1e-4,
          beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, lr_final: float | None = None, stream=None):
    """Epochs of minibatch AdamW; perms[e] is epoch e's row order (int32
    permutation of 0..n-1, drawn by the caller).  Returns the mean loss per
    epoch.  The learning rate decays linearly to lr_final (default lr/10)."""
    import torch
    n = feats.shape[0]
    steps_per_epoch = n // batch
    total = steps_per_epoch * len(perms)
    lr_final = lr / 10 if lr_final is None else lr_final
    losses = []
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    acc = torch.zeros(1, dtype=torch.float32, device=feats.device)
    step = 0
    for order in perms:
        perm = torch.as_tensor(np.asarray(order, dtype=np.int32), device=feats.device)
        acc.zero_()
        for s0 in range(steps_per_epoch):
            frac = step / max(total - 1, 1)
            rate = lr + (lr_final - lr) * frac
            net.train_step(feats, lab_t, lab_s, perm[s0 * batch:(s0 + 1) * batch], rate, beta1, beta2, eps, wd,
                           loss=loss, stream=stream)
            acc += loss
            step += 1
        losses.append(float(acc.item()) / steps_per_epoch)
    return losses


def full_search_labeler(plan: F.Plan, tmpl_coeffs, stream=None):
    """Labels by the plan's full search: coefficients -> (best template,
    best pose) device tensors."""
    def label(ic):
        _, best = plan.align_coeffs(ic, tmpl_coeffs, stream=stream)
        return F.best_template(best, stream=stream)
    return label


def refined_labeler(coarse: F.Plan, fine: F.Plan, tmpl_coeffs, k: int = 4, stream=None):
    """Labels by the two-pass search (ftk_align_refined: the coarse form over
    every template, the fine form on each image's k best)."""
    def label(ic):
        _, bt, bp = F.align_refined(coarse, fine, ic, tmpl_coeffs, k, stream=stream)
        return bt, bp
    return label


def train_online(net: F.MLP, plan: F.Plan, clean, tmpl_coeffs, shift_bin: np.ndarray, noise_fn, perms,
                 kind: str, n_r: int, n_q: int, batch: int, lr: float, wd: float = 1e-2, lr_final=None,
                 label_chunk: int = 4096, stream=None, labeler=None, log=None):
    """Training with fresh noise every epoch: epoch e re-noises the clean
    device images [nI][n][n] with noise_fn(e) (a device tensor of the same
    shape, drawn by the caller), labels them with the full FTK search
    against the template coefficients, takes their features and runs one
    epoch of minibatch AdamW in the order perms[e].  The input
    standardisation is set from the first epoch's features.  labeler:
    coefficients -> (best template, best pose), default the plan's full
    search; log(e, loss) is called after each epoch.  Returns the mean loss
    per epoch."""
    import torch
    nI = clean.shape[0]
    sb = torch.as_tensor(shift_bin, dtype=torch.int32, device=clean.device)
    steps = nI // batch
    total = steps * len(perms)
    lr_final = lr / 10 if lr_final is None else lr_final
    loss = torch.empty(1, dtype=torch.float32, device=clean.device)
    acc = torch.zeros(1, dtype=torch.float32, device=clean.device)
    lab_t = torch.empty(nI, dtype=torch.int32, device=clean.device)
    lab_s = torch.empty(nI, dtype=torch.int32, device=clean.device)
    feats = torch.empty((nI, F.feature_count(kind, n_r, n_q)), dtype=torch.float32, device=clean.device)
    losses = []
    step = 0
    labeler = labeler or full_search_labeler(plan, tmpl_coeffs, stream)
    for e, order in enumerate(perms):
        imgs = clean + noise_fn(e)
        for i0 in range(0, nI, label_chunk):
            ic = plan.transform(imgs[i0:i0 + label_chunk].contiguous(), stream=stream)
            bt, bp = labeler(ic)
            lab_t[i0:i0 + label_chunk] = bt
            lab_s[i0:i0 + label_chunk] = sb[bp[:, 1].long()]
            F.features(plan, ic, n_r, n_q, kind=kind, out=feats[i0:i0 + label_chunk], stream=stream)
        if e == 0:
            mu, isg = input_norm(feats.cpu().numpy())
            net.set_input_norm(mu, isg)
        perm = torch.as_tensor(np.asarray(order, dtype=np.int32), device=clean.device)
        acc.zero_()
        for s0 in range(steps):
            rate = lr + (lr_final - lr) * (step / max(total - 1, 1))
            net.train_step(feats, lab_t, lab_s, perm[s0 * batch:(s0 + 1) * batch], rate, wd=wd, loss=loss,
                           stream=stream)
            acc += loss
            step += 1
        losses.append(float(acc.item()) / steps)
        if log:
            log(e, losses[-1])
    return losses


def choose_tau(mass: np.ndarray, hit: np.ndarray, max_miss: float) -> float:
    """Smallest confidence threshold whose confident-and-missed fraction is
    at most max_miss (hit[i]: the label is among image i's proposals)."""
    mass = np.asarray(mass, dtype=np.float64)
    hit = np.asarray(hit, dtype=bool)
    n = mass.size
    for tau in np.unique(np.concatenate([mass, [np.inf]])):
        miss = np.count_nonzero((mass >= tau) & ~hit)
        if miss <= max_miss * n:
            return float(tau)
    return float("inf")
