"""Pure-Python, per-pixel implementation of the EDGE stages for tiny inputs.

Written independently of oracle/edge_oracle.c (no shared code) so that an
indexing, sign or transposition slip in either one shows up as a mismatch.
Stage definitions follow the reading stated in oracle/hxo.h (O1..O8).
"""
import math


def clamp(v, lo, hi):
    return lo if v < lo else hi if v > hi else v


def weights(k, sigma):
    r = k // 2
    raw = [math.exp(-(d * d) / (2.0 * sigma * sigma)) for d in range(-r, r + 1)]
    s = sum(raw)
    return [v / s for v in raw]


def get(img, y, x):
    H, W = len(img), len(img[0])
    return img[clamp(y, 0, H - 1)][clamp(x, 0, W - 1)]


def blur(img, k, sigma):
    g = weights(k, sigma)
    r = k // 2
    H, W = len(img), len(img[0])
    out = [[0.0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            acc = 0.0
            for a in range(k):
                for b in range(k):
                    acc += g[a] * g[b] * float(get(img, y + a - r, x + b - r))
            out[y][x] = acc
    return out


def laplacian(B):
    H, W = len(B), len(B[0])
    return [[(get(B, y - 1, x) + get(B, y + 1, x)) +
             (get(B, y, x - 1) + get(B, y, x + 1)) - 4.0 * get(B, y, x)
             for x in range(W)] for y in range(H)]


def zero_crossing(L):
    H, W = len(L), len(L[0])
    Z = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            signs = {1 if get(L, y + dy, x + dx) > 0 else 0
                     for dy in (-1, 0, 1) for dx in (-1, 0, 1)}
            Z[y][x] = 1 if len(signs) == 2 else 0
    return Z


def sobel(B):
    H, W = len(B), len(B[0])
    G = [[0.0] * W for _ in range(H)]
    kx = [[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]]
    for y in range(H):
        for x in range(W):
            gx = gy = 0.0
            for a in range(3):
                for b in range(3):
                    v = get(B, y + a - 1, x + b - 1)
                    gx += kx[a][b] * v
                    gy += kx[b][a] * v
            G[y][x] = math.sqrt(gx * gx + gy * gy)
    return G


def edge_detect(img, k=5, sigma=1.0, theta=0.1):
    B = blur(img, k, sigma)
    L = laplacian(B)
    Z = zero_crossing(L)
    G = sobel(B)
    M = max(max(row) for row in G)
    tau = theta * M
    H, W = len(img), len(img[0])
    mask = [[1 if (Z[y][x] == 1 and G[y][x] > tau) else 0 for x in range(W)]
            for y in range(H)]
    return dict(B=B, L=L, Z=Z, G=G, M=M, mask=mask)
