"""Learned diagonal control variate: training and evaluation driver.

Orchestration only: features, the MLP forward and backward passes, Adam,
the LDOS targets and the variance estimates all run in libnd through its C
ABI; this module allocates device tensors and loops.

Estimator (the library's nd_ldos_moments with cv_g): for node i, moment m and
probe z,  g_im + z_i ((T_m(H) - diag g_m) z)_i,  unbiased for any g.  Its
per-probe variance is estimated from the same run as
    s^2 = k/(k-1) (ldos_sq - ldos^2),
and the number of probes needed for a target variance v* is mean(s^2) / v*,
averaged over nodes and the moments m = 1 .. M-1 (moment 0 is excluded: it has
no variance under +/-1 probes and a trivial one under the control variate).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import (ND_HUBPATHS, ND_PENDANTS, ND_PROBE_GAUSSIAN, ND_PROBE_RADEMACHER, ND_TWINS_CLOSED, ND_TWINS_OPEN,
               N_FEAT, n_params, nd_adam_step, nd_column_stats, nd_cv_exact_diag, nd_ldos_moments, nd_ldos_variance,
               nd_mlp_forward, nd_mlp_grad, nd_motif_diag, nd_motif_filter, nd_node_features)

ALL_MOTIFS = ND_TWINS_OPEN | ND_TWINS_CLOSED | ND_PENDANTS | ND_HUBPATHS

F32, F64 = torch.float32, torch.float64


@dataclass
class ControlVariate:
    params: torch.Tensor   # device float [n_params(n_out)]
    mean: torch.Tensor     # device float [5] feature means (training set)
    std: torch.Tensor      # device float [5]
    n_out: int


def raw_features(g) -> torch.Tensor:
    """log1p-scaled structural features [N][5] (unstandardised)."""
    f = torch.empty(g.n * N_FEAT, dtype=F32, device="cuda")
    nd_node_features(g, f)
    return f


def features(g, cv: ControlVariate) -> torch.Tensor:
    f = torch.empty(g.n * N_FEAT, dtype=F32, device="cuda")
    nd_node_features(g, f, cv.mean, cv.std)
    return f


def ldos_targets(g, n_probes: int, n_moments: int, seed: int) -> torch.Tensor:
    """First n_moments LDOS moments from an n_probes Rademacher run, as float [N][M]."""
    ld = torch.empty(g.n * n_moments, dtype=F64, device="cuda")
    nd_ldos_moments(g, None, n_probes, n_moments, seed, ND_PROBE_RADEMACHER, ld)
    return ld.to(F32)


def feature_stats(feats) -> tuple:
    """Column means and standard deviations over the concatenated training features."""
    x = torch.cat(feats)
    mean = torch.empty(N_FEAT, dtype=F32, device="cuda")
    std = torch.empty(N_FEAT, dtype=F32, device="cuda")
    nd_column_stats(x, x.numel() // N_FEAT, N_FEAT, mean, std)
    return mean, std


def train(graphs, targets, n_out: int, init: np.ndarray, steps: int = 2000, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, log_every: int = 0):
    """Fit the MLP to per-node targets by minibatch Adam on the GPU.

    graphs: built nd graphs; targets: matching float [N][n_out] device tensors.
    Returns (ControlVariate, loss history)."""
    mean, std = feature_stats([raw_features(g) for g in graphs])
    cv = ControlVariate(torch.from_numpy(np.ascontiguousarray(init, dtype=np.float32)).cuda(), mean, std, n_out)
    X = torch.cat([features(g, cv) for g in graphs])
    Y = torch.cat([t.reshape(-1) for t in targets])
    total = X.numel() // N_FEAT
    P = n_params(n_out)
    m = torch.zeros(P, dtype=F32, device="cuda")
    v = torch.zeros(P, dtype=F32, device="cuda")
    grad = torch.empty(P, dtype=F32, device="cuda")
    loss = torch.empty(1, dtype=F32, device="cuda")
    rng = np.random.default_rng(seed)
    idx_all = torch.from_numpy(rng.integers(0, total, size=(steps, batch), dtype=np.int64).astype(np.int32)).cuda()
    hist = []
    for t in range(1, steps + 1):
        idx = idx_all[t - 1]
        nd_mlp_grad(cv.params, X, Y, n_out, idx, batch, n_out, grad, loss)
        nd_adam_step(cv.params, m, v, grad, P, t, lr)
        if log_every and (t % log_every == 0 or t == 1):
            hist.append((t, float(loss.item())))
    return cv, hist


def motifs_of(g, seed: int = 1):
    """Motif classes of every kind the library detects (Sec. 3.4)."""
    return nd_motif_filter(g, seed, ALL_MOTIFS)


def smooth_targets(targets: torch.Tensor, motifs, n_out: int) -> torch.Tensor:
    """Training targets without the exactly known motif part of the
    diagonal: the MLP learns the remainder (in place)."""
    nd_motif_diag(motifs, targets, n_out, n_out, -1.0)
    return targets


def predict(g, cv: ControlVariate, motifs=None, exact_low: bool = True) -> torch.Tensor:
    """The control variate g [N][n_out]: the MLP's output, plus the exact
    motif part of the diagonal for class members (when the model was trained
    on smooth targets, give the same kinds of motifs), with the exactly known
    T_0..T_3(H)_ii in the first four columns (exact_low)."""
    out = torch.empty(g.n * cv.n_out, dtype=F32, device="cuda")
    nd_mlp_forward(cv.params, features(g, cv), g.n, cv.n_out, out)
    if motifs is not None:
        nd_motif_diag(motifs, out, cv.n_out, cv.n_out, 1.0)
    if exact_low:
        nd_cv_exact_diag(g, out, cv.n_out, min(4, cv.n_out))
    return out


def exact_known(g, n_out: int, motifs=None) -> torch.Tensor:
    """A control variate holding only what is known exactly: T_0..T_3(H)_ii
    and the motif part of every class member's diagonal (zero elsewhere);
    the baseline the learned part must improve on."""
    out = torch.zeros(g.n * n_out, dtype=F32, device="cuda")
    if motifs is not None:
        nd_motif_diag(motifs, out, n_out, n_out, 1.0)
    nd_cv_exact_diag(g, out, n_out, min(4, n_out))
    return out


def probe_variance(g, n_moments: int, n_probes: int, seed: int, gaussian: bool, cv_g=None) -> float:
    """Mean per-probe variance of the diagonal estimates over nodes and
    moments 1 .. M-1, from one n_probes run (unbiased sample variance)."""
    k = n_probes
    ld = torch.empty(g.n * n_moments, dtype=F64, device="cuda")
    sq = torch.empty(g.n * n_moments, dtype=F64, device="cuda")
    flags = ND_PROBE_GAUSSIAN if gaussian else ND_PROBE_RADEMACHER
    nd_ldos_moments(g, None, k, n_moments, seed, flags, ld, cv_g=cv_g, ldos_sq=sq)
    out = torch.empty(1, dtype=F64, device="cuda")
    nd_ldos_variance(ld, sq, g.n, n_moments, 1, k, out)
    return float(out.item())


def empirical_variance(g, n_moments: int, n_probes: int, reps: int, seed: int, gaussian: bool, cv_g=None) -> float:
    """Variance of the n_probes-probe LDOS estimate across `reps` reseeded
    runs, averaged over nodes and moments 1 .. M-1 (compare with
    probe_variance / n_probes)."""
    flags = ND_PROBE_GAUSSIAN if gaussian else ND_PROBE_RADEMACHER
    runs = []
    for r in range(reps):
        ld = torch.empty(g.n * n_moments, dtype=F64, device="cuda")
        nd_ldos_moments(g, None, n_probes, n_moments, seed + 7919 * r, flags, ld, cv_g=cv_g)
        runs.append(ld.reshape(g.n, n_moments)[:, 1:])
    stack = torch.stack(runs)
    return float(stack.var(dim=0, unbiased=True).mean().item())
