"""CPU statement of the leaf binning (test helper, not part of the library).

Written from the definition of the leaf tiling (exact cube tiling of
Sec. 4.1.1 at the leaf level, periodic images of eq. (periodic-images)):
  periodic axis i < D : y = x - L floor(x / L)     (IEEE ops, no FMA)
  free axis           : 0 <= x < L required, y = x
  b_i = min(n_i - 1, max(0, floor(y * (n_i / L_i))))
  key = (b0 n1 + b1) n2 + b2
  perm = stable sort of the keys, box_start[b] = first sorted index with key >= b.
numpy element-wise ufuncs round every operation, so this is bit-comparable
with the device code.
"""
import numpy as np


def bin_spec(x, L, D, n):
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    Lv = np.asarray(L, dtype=np.float64)
    nv = np.asarray(n, dtype=np.int64)
    y = np.empty_like(x)
    ok = np.isfinite(x).all(axis=1)
    for ax in range(3):
        if ax < D:
            with np.errstate(invalid="ignore"):
                y[:, ax] = x[:, ax] - Lv[ax] * np.floor(x[:, ax] / Lv[ax])
        else:
            with np.errstate(invalid="ignore"):
                ok &= (x[:, ax] >= 0.0) & (x[:, ax] < Lv[ax])
            y[:, ax] = x[:, ax]
    inv = nv.astype(np.float64) / Lv
    with np.errstate(invalid="ignore"):
        f = np.floor(y * inv)
    b = np.zeros((N, 3), dtype=np.int64)
    for ax in range(3):
        fa = np.where(np.isfinite(f[:, ax]), f[:, ax], 0.0)
        b[:, ax] = np.clip(fa, 0, nv[ax] - 1).astype(np.int64)
    key = (b[:, 0] * nv[1] + b[:, 1]) * nv[2] + b[:, 2]
    key = np.where(ok, key, 0).astype(np.int32)
    perm = np.argsort(key, kind="stable").astype(np.int32)
    skey = key[perm]
    nbox = int(nv.prod())
    box_start = np.searchsorted(skey, np.arange(nbox + 1), side="left").astype(np.int32)
    ys = y[perm].T.copy()
    return dict(ok=bool(ok.all()), key=key, perm=perm, skey=skey, box_start=box_start, ys=ys)


def axis_tables_spec(D, n):
    rows = []
    imgs = []
    for ax in range(3):
        for b in range(n[ax]):
            r, s = [], []
            for off in (-1, 0, 1):
                nb = b + off
                im = 0
                if ax < D:
                    if nb < 0:
                        nb += n[ax]
                        im = -1
                    elif nb >= n[ax]:
                        nb -= n[ax]
                        im = 1
                elif nb < 0 or nb >= n[ax]:
                    nb = -1
                r.append(nb)
                s.append(im)
            rows.append(r)
            imgs.append(s)
    return np.asarray(rows, dtype=np.int32), np.asarray(imgs, dtype=np.int8)
