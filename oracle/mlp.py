"""FP64 reference of the opening-rule network and its training gradient.

TEST INFRASTRUCTURE ONLY.  Plain numpy, written from the definitions: a
4-32-32-1 ReLU network on normalised inputs, x_n = (x - mean) * inv_std,
output in normalised label units; the loss of a batch is the mean over the
batch of (output - (y - y_mean) / y_std)^2; gradients by the chain rule.
Parameter layout (1249 trained + 10 normalisation floats): W1[32][4],
b1[32], W2[32][32], b2[32], W3[32], b3, x_mean[4], x_inv_std[4], y_mean,
y_std.
"""
import numpy as np

NH, NIN = 32, 4
W1, B1, W2, B2, W3, B3 = 0, 128, 160, 1184, 1216, 1248
NTRAIN = 1249
XMEAN, XISTD, YMEAN, YSTD = 1249, 1253, 1257, 1258


def unpack(w):
    w = np.asarray(w, np.float64)
    return (w[W1:B1].reshape(NH, NIN), w[B1:W2], w[W2:B2].reshape(NH, NH), w[B2:W3], w[W3:B3], w[B3],
            w[XMEAN:XISTD], w[XISTD:YMEAN], w[YMEAN], w[YSTD])


def loss_and_grad(w, X, Y):
    """Batch loss and its gradient with respect to the 1249 trained weights."""
    a1, c1, a2, c2, a3, c3, xm, xi, ym, ys = unpack(w)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    B = X.shape[0]
    x = (X - xm) * xi
    z1 = x @ a1.T + c1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ a2.T + c2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ a3 + c3
    r = out - (Y - ym) / ys
    loss = np.mean(r * r)
    go = 2.0 * r / B
    g2 = (go[:, None] * a3[None, :]) * (z2 > 0)
    g1 = (g2 @ a2) * (z1 > 0)
    grad = np.zeros(NTRAIN)
    grad[W1:B1] = (g1.T @ x).ravel()
    grad[B1:W2] = g1.sum(0)
    grad[W2:B2] = (g2.T @ h1).ravel()
    grad[B2:W3] = g2.sum(0)
    grad[W3:B3] = h2.T @ go
    grad[B3] = go.sum()
    return loss, grad


def forward(w, X):
    """FP64 network output in label units."""
    a1, c1, a2, c2, a3, c3, xm, xi, ym, ys = unpack(w)
    x = (np.asarray(X, np.float64) - xm) * xi
    h1 = np.maximum(x @ a1.T + c1, 0.0)
    h2 = np.maximum(h1 @ a2.T + c2, 0.0)
    return (h2 @ a3 + c3) * ys + ym
