"""FP64 NumPy reference of the warm-start MLP and its window features.

TEST INFRASTRUCTURE ONLY (imported by tests/ and the benchmark's CPU leg).

The network (a learned initialisation for the fit of Sec. IV-A; the paper's
own fit starts from fixed values) is 150 -> 256 -> 256 -> 5 with ReLU, padded
to 160 inputs and 16 outputs.  ``mirror=True`` rounds to BF16 (round to
nearest even) exactly where the GPU kernels do: the features X, the weight
copies W1..W3, the hidden activations H1, H2 and the back-propagated
gradients dY, dH2, dH1; everything else is FP64.  ``mirror=False`` is the
plain FP64 network (used for the finite-difference pin).
"""
from __future__ import annotations

import numpy as np

IN, IN_PAD, HID, OUT, OUT_PAD = 150, 160, 256, 5, 16
SHAPES = (("W1", (IN_PAD, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, OUT_PAD)), ("b3", (OUT_PAD,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via FP32; returns float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X, mirror: bool = True):
    r = bf16 if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta)
    Xr = r(X)
    H1 = r(np.maximum(Xr @ r(p["W1"]) + p["b1"], 0.0))
    H2 = r(np.maximum(H1 @ r(p["W2"]) + p["b2"], 0.0))
    Y = H2 @ r(p["W3"]) + p["b3"]
    return Y, (Xr, H1, H2)


def loss_and_grad(theta, X, U, mirror: bool = True):
    """L = mean over the batch and the 5 outputs of (Y - U)^2; returns (L, dL/dtheta)."""
    r = bf16 if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta)
    Y, (Xr, H1, H2) = forward(theta, X, mirror)
    B = X.shape[0]
    R = Y[:, :OUT] - U
    L = float(np.mean(R * R))
    dY = np.zeros((B, OUT_PAD))
    dY[:, :OUT] = 2.0 * R / (B * OUT)
    dY = r(dY)
    g = {"W3": H2.T @ dY, "b3": dY.sum(0)}
    dH2 = r((dY @ r(p["W3"]).T) * (H2 > 0))
    g["W2"] = H1.T @ dH2
    g["b2"] = dH2.sum(0)
    dH1 = r((dH2 @ r(p["W2"]).T) * (H1 > 0))
    g["W1"] = Xr.T @ dH1
    g["b1"] = dH1.sum(0)
    return L, pack(g)


def features(target, obs_first: int, obs_stride: int, dt: float, p0, length, lane_offsets):
    """Window features [N, IN_PAD] (values before BF16 rounding, FP64), from the
    observed absolute positions target [n_obs, N]: per observation j at time
    t_j = (obs_first + j obs_stride) dt
      (p_j - p0) / 1000,
      (p_j - p_{j-1}) / (t_j - t_{j-1}) / 30 with p_{-1} = p0 at t_{-1} = 0,
      (p_{h,j} - p_j - length_h) / 50 for the leader h (the vehicle ahead in
      the lane), 200 / 50 for a lane head,
    laid out as [offsets of all observations | speeds | gaps | zero padding].
    Plain loops over vehicles and observations in FP64."""
    target = np.asarray(target, dtype=np.float64)
    n_obs, N = target.shape
    p0 = np.asarray(p0, dtype=np.float64)
    length = np.asarray(length, dtype=np.float64)
    lane_offsets = np.asarray(lane_offsets)
    F = np.zeros((N, IN_PAD))
    for lane in range(len(lane_offsets) - 1):
        for i in range(int(lane_offsets[lane]), int(lane_offsets[lane + 1])):
            head = i == int(lane_offsets[lane])
            prev, tprev = p0[i], 0.0
            for j in range(n_obs):
                tj = (obs_first + j * obs_stride) * float(dt)
                pj = target[j, i]
                F[i, j] = (pj - p0[i]) / 1000.0
                F[i, n_obs + j] = (pj - prev) / (tj - tprev) / 30.0
                gap = 200.0 if head else target[j, i - 1] - pj - length[i - 1]
                F[i, 2 * n_obs + j] = gap / 50.0
                prev, tprev = pj, tj
    return F
