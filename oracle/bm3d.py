"""BM3D denoiser (oracle), the third plug-in prior of the u-step.

The paper cites BM3D (Dabov et al., IEEE TIP 2007) for the denoising step
(Sec. III-B) and treats its strength as a noise level (Sec. IV-B); it gives no
further detail, so the settings below are this implementation's choices:

* grey-scale, per slice; 8x8 blocks; reference blocks on a step-3 grid plus
  the last row/column position; search window +-19 pixels (39x39) around the
  reference, clipped to the image;
* block distance = mean squared difference over the 64 pixels, evaluated in
  float64 in a fixed order: for each block column c (0..7) the column sum
  over rows r (0..7) of (a - b)^2, then the sum of the eight column sums
  (plain products and sums, no fused multiply-add), divided by 64;
* a group is the reference block followed by the other candidates with
  distance <= tau (3000/255^2 in the hard-threshold stage, 400/255^2 in the
  Wiener stage), ordered by (distance, raster index of the block), at most 16
  blocks, truncated to the largest power of two;
* 3D transform = orthonormal 8x8 DCT-II of every block, then the orthonormal
  Haar transform along the group;
* stage 1 keeps coefficients with |c| >= 2.7 sigma, weight 1/(sigma^2 max(1, kept));
  stage 2 (on the basic estimate) shrinks the noisy group's coefficients by
  W = B^2/(B^2 + sigma^2) (B: the basic estimate's coefficients), weight
  1/(sigma^2 ||W||^2) (1/sigma^2 for a group whose W is all zero);
* aggregation: weighted sum of every filtered block into a numerator and the
  weights into a denominator per pixel; estimate = numerator / denominator.
"""
import numpy as np

P = 8
STEP = 3
RADIUS = 19
NMAX = 16
TAU_HT = 3000.0 / (255.0 * 255.0)
TAU_WIE = 400.0 / (255.0 * 255.0)
LAMBDA_3D = 2.7


def ref_positions(n):
    pos = list(range(0, n - P + 1, STEP))
    if pos[-1] != n - P:
        pos.append(n - P)
    return pos


def dct_matrix():
    """Orthonormal DCT-II matrix C[k, j] = a_k cos(pi (2j+1) k / 16)."""
    C = np.zeros((P, P))
    for k in range(P):
        a = np.sqrt(1.0 / P) if k == 0 else np.sqrt(2.0 / P)
        for j in range(P):
            C[k, j] = a * np.cos(np.pi * (2 * j + 1) * k / (2 * P))
    return C


def haar_matrix(n):
    """Orthonormal Haar transform of length n (a power of two), full decomposition."""
    if n == 1:
        return np.ones((1, 1))
    h = haar_matrix(n // 2)
    top = np.kron(h, [1.0, 1.0]) / np.sqrt(2.0)
    bot = np.kron(np.eye(n // 2), [1.0, -1.0]) / np.sqrt(2.0)
    return np.vstack([top, bot])


def block_distance(img, ry, rx, cys, cxs):
    """Distances from the reference block at (ry, rx) to the blocks at (cys[i], cxs[i])."""
    img = np.asarray(img, dtype=np.float64)
    acc = np.zeros(len(cys))
    for c in range(P):
        col = np.zeros(len(cys))
        for r in range(P):
            t = img[ry + r, rx + c] - img[cys + r, cxs + c]
            col = col + t * t
        acc = acc + col
    return acc / (P * P)


def match(img, ry, rx, tau):
    """Group of the reference (ry, rx): list of block positions, reference first."""
    H, W = img.shape
    ys = np.arange(max(0, ry - RADIUS), min(H - P, ry + RADIUS) + 1)
    xs = np.arange(max(0, rx - RADIUS), min(W - P, rx + RADIUS) + 1)
    cy, cx = np.meshgrid(ys, xs, indexing="ij")
    cy, cx = cy.ravel(), cx.ravel()
    keep = ~((cy == ry) & (cx == rx))
    cy, cx = cy[keep], cx[keep]
    d = block_distance(img, ry, rx, cy, cx)
    ok = d <= tau
    cy, cx, d = cy[ok], cx[ok], d[ok]
    order = np.lexsort((cy * W + cx, d))[: NMAX - 1]
    group = [(ry, rx)] + [(int(cy[i]), int(cx[i])) for i in order]
    n = 1
    while n * 2 <= len(group):
        n *= 2
    return group[:n]


def match_all(img, tau):
    """Groups of every reference position of one slice, in raster order of the references."""
    H, W = img.shape
    return [match(img, ry, rx, tau) for ry in ref_positions(H) for rx in ref_positions(W)]


def _blocks(img, group):
    return np.stack([img[y:y + P, x:x + P] for (y, x) in group])


def transform3d(blocks, C):
    n = blocks.shape[0]
    t = np.einsum("kj,bjl,ml->bkm", C, blocks, C)  # C X C^T per block
    return np.einsum("ab,bkm->akm", haar_matrix(n), t)


def itransform3d(coef, C):
    n = coef.shape[0]
    t = np.einsum("ba,bkm->akm", haar_matrix(n), coef)
    return np.einsum("kj,bkm,ml->bjl", C, t, C)


def stage_ht(img, sigma, groups):
    """Hard-threshold stage: basic estimate of one slice from its groups."""
    img = np.asarray(img, dtype=np.float64)
    C = dct_matrix()
    num = np.zeros_like(img)
    den = np.zeros_like(img)
    thr = LAMBDA_3D * sigma
    for g in groups:
        coef = transform3d(_blocks(img, g), C)
        keep = np.abs(coef) >= thr
        kept = int(keep.sum())
        est = itransform3d(np.where(keep, coef, 0.0), C)
        w = 1.0 / (sigma * sigma * max(1, kept))
        for b, (y, x) in enumerate(g):
            num[y:y + P, x:x + P] += w * est[b]
            den[y:y + P, x:x + P] += w
    return num / den


def stage_wiener(img, basic, sigma, groups):
    """Wiener stage: final estimate of one slice from the noisy slice and the basic estimate."""
    img = np.asarray(img, dtype=np.float64)
    basic = np.asarray(basic, dtype=np.float64)
    C = dct_matrix()
    num = np.zeros_like(img)
    den = np.zeros_like(img)
    for g in groups:
        cb = transform3d(_blocks(basic, g), C)
        cn = transform3d(_blocks(img, g), C)
        Wc = cb * cb / (cb * cb + sigma * sigma)
        est = itransform3d(Wc * cn, C)
        wn = np.sum(Wc * Wc)
        w = 1.0 / (sigma * sigma * (wn if wn > 0 else 1.0))  # an all-zero group keeps weight 1/sigma^2
        for b, (y, x) in enumerate(g):
            num[y:y + P, x:x + P] += w * est[b]
            den[y:y + P, x:x + P] += w
    return num / den


def bm3d_slice(img, sigma, return_basic=False):
    img = np.asarray(img, dtype=np.float64)
    g1 = match_all(img, TAU_HT)
    basic = stage_ht(img, sigma, g1)
    g2 = match_all(basic, TAU_WIE)
    out = stage_wiener(img, basic, sigma, g2)
    return (out, basic) if return_basic else out


def bm3d(f, sigma):
    """BM3D of every slice of f [..., H, W] at noise level sigma."""
    f = np.asarray(f, dtype=np.float64)
    out = np.empty_like(f)
    flat = f.reshape(-1, *f.shape[-2:])
    o = out.reshape(-1, *f.shape[-2:])
    for i in range(flat.shape[0]):
        o[i] = bm3d_slice(flat[i], sigma)
    return out
