"""Coefficients of the FP32 arctangent of eval.hip (bem_atan2): atan(t) ~
t * P(t^2) on [0, 1], P of degree 8, fitted by least squares on Chebyshev
nodes with Lawson reweighting (an iteration towards the minimax fit), then
rounded to FP32. Prints the coefficients (lowest degree first) and the
largest error of the FP32 Horner evaluation on a dense grid (about 9e-8)."""
import numpy as np


def fit(deg=8, n=4000, iters=60):
    t = np.cos(np.pi * (np.arange(n) + 0.5) / n) * 0.5 + 0.5
    t = np.concatenate([t, np.linspace(0, 1, 2001)])
    t = t[t > 1e-6]
    A = np.vstack([(t * t) ** k for k in range(deg + 1)]).T * t[:, None]
    w = np.ones_like(t)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], np.arctan(t) * sw, rcond=None)
        err = np.abs(A @ c - np.arctan(t))
        w = w * (err / err.max() + 1e-3)
        w /= w.sum()
    return c.astype(np.float32)


def fp32_error(cf):
    t = np.linspace(0, 1, 200001).astype(np.float32)
    s = t * t
    p = np.float32(cf[-1])
    for k in range(len(cf) - 2, -1, -1):
        p = (p * s + cf[k]).astype(np.float32)
    return float(np.abs((t * p).astype(np.float64) - np.arctan(t.astype(np.float64))).max())


if __name__ == "__main__":
    cf = fit()
    print([float(x) for x in cf])
    print("max abs error of the FP32 evaluation: %.2e" % fp32_error(cf))
