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


def tiles_spec(box_start, D, n, T=64, CAP=512, ZMAX=46):
    """Target tiles as the library forms them, heavy-first.

    Per leaf column (b0, b1), walking z upwards: a box with more than T
    targets, or whose three neighbour slabs hold more than CAP sources, gets
    tiles of its own (col, z, -(z+1), first) of at most T targets each;
    otherwise a tile grows over z0..z1 while its targets stay <= T, the slabs
    z0-1 .. z1+1 (sources in the 9 stencil columns) stay <= CAP and
    z1 - z0 + 1 <= ZMAX.  A slab is counted once per stencil column it is
    reached through, and a slab beyond a free z face is empty.  The tiles,
    listed column by column, are then stably sorted by the key
    64 - bit_length(cost + 1), cost = sum over the tile's targets of the
    sources in their 3 slabs.  Finally, within each bucket (run of equal
    keys) of B tiles at offset o, the positions o + k with k = q (mod 8) take,
    for q = 0, 1, ..., 7 in turn, the next ceil((B - q) / 8) tiles of the
    bucket in order (one contiguous run per XCD of the pair kernels).
    """
    tiles, keys = _tile_list(box_start, D, n, T, CAP, ZMAX)
    order = np.argsort(keys, kind="stable")
    srt, sk = tiles[order], keys[order]
    out = np.empty_like(srt)
    o = 0
    while o < len(srt):
        B = int(np.searchsorted(sk, sk[o], side="right")) - o
        pos = [k for q in range(8) for k in range(q, B, 8)]
        out[o + np.asarray(pos, dtype=np.int64)] = srt[o:o + B]
        o += B
    return out


def heavy_count_spec(box_start, D, n, heavy_log=16, T=64, CAP=512, ZMAX=46):
    """Number of tiles of cost 2^heavy_log - 1 or more (bit_length(cost + 1)
    above heavy_log): the leading tiles of the heavy-first order."""
    _, keys = _tile_list(box_start, D, n, T, CAP, ZMAX)
    return int((keys <= 63 - heavy_log).sum())


def _tile_list(box_start, D, n, T, CAP, ZMAX):
    """The tiles column by column, with their keys 64 - bit_length(cost + 1)."""
    n0, n1, n2 = (int(v) for v in n)
    nbr, _ = axis_tables_spec(D, n)
    bs = np.asarray(box_start, dtype=np.int64)
    cnt = (bs[1:] - bs[:-1]).reshape(n0 * n1, n2)
    tiles, keys = [], []
    for b0 in range(n0):
        for b1 in range(n1):
            col = b0 * n1 + b1
            ccol = []
            for k in range(9):
                nb0 = nbr[b0][k // 3]
                nb1 = nbr[n0 + b1][k % 3]
                if nb0 >= 0 and nb1 >= 0:
                    ccol.append(nb0 * n1 + nb1)
            slab = cnt[ccol].sum(axis=0) if ccol else np.zeros(n2, dtype=np.int64)

            def sl(zv):
                if 0 <= zv < n2:
                    return int(slab[zv])
                if D > 2:
                    return int(slab[zv % n2])
                return 0

            z = 0
            while z < n2:
                nt = int(cnt[col, z])
                if nt == 0:
                    z += 1
                    continue
                q1 = sl(z - 1) + sl(z) + sl(z + 1)
                first = int(bs[col * n2 + z])
                if nt > T or q1 > CAP:
                    for c in range(0, nt, T):
                        m = min(T, nt - c)
                        tiles.append((col, z, -(z + 1), first + c))
                        keys.append(64 - (m * q1 + 1).bit_length())
                    z += 1
                    continue
                z1, tacc, q, cost = z, nt, q1, nt * q1
                while z1 + 1 < n2 and z1 + 2 - z <= ZMAX:
                    nn = int(cnt[col, z1 + 1])
                    s2 = sl(z1 + 2)
                    if tacc + nn > T or q + s2 > CAP:
                        break
                    cost += nn * (sl(z1) + sl(z1 + 1) + s2)
                    z1 += 1
                    tacc += nn
                    q += s2
                tiles.append((col, z, z1, first))
                keys.append(64 - (cost + 1).bit_length())
                z = z1 + 1
    return np.asarray(tiles, dtype=np.int32).reshape(-1, 4), np.asarray(keys, dtype=np.int64)
