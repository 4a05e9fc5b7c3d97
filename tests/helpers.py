"""Shared test helpers: oracle comparison with exemptions, BVH structure checks."""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-4  # max abs per RGBA channel against the FP64 oracle


def compare(gpu_rgba, gpu_n, orc: dict, tol: float = TOL) -> dict:
    """Element-wise comparison of GPU output with the oracle on the same pixels.

    Exempt: a grazing sphere (|disc| <= 1e-6 r^2) before the end of the
    composited range, or more than one knife-edge.  A pixel with one
    knife-edge passes if it matches either branch.  Everything else must
    agree within `tol` per channel with an identical hit count.
    """
    g = np.asarray(gpu_rgba, dtype=np.float64).reshape(-1, 4)
    n = np.asarray(gpu_n).reshape(-1).astype(np.int64)
    flags = orc["flags"]
    exempt = (flags & (oracle.FLAG_GRAZE | oracle.FLAG_MULTI_KNIFE)) != 0
    err_main = np.abs(g - orc["rgba"]).max(axis=1)
    ok_main = (err_main <= tol) & (n == orc["n"])
    err_alt = np.abs(g - orc["alt_rgba"]).max(axis=1)
    ok_alt = (err_alt <= tol) & (n == orc["alt_n"]) & ((flags & oracle.FLAG_KNIFE) != 0)
    ok = ok_main | ok_alt | exempt
    bad = np.nonzero(~ok)[0]
    strict = ~exempt
    return {
        "pixels": g.shape[0],
        "exempt": int(exempt.sum()),
        "knife": int(((flags & oracle.FLAG_KNIFE) != 0).sum()),
        "bad": bad,
        "max_err": float(np.where(strict, np.minimum(err_main, np.where(ok_alt, err_alt, np.inf)), 0).max())
        if g.shape[0] else 0.0,
        "hits_checked": int(n[strict].sum()),
    }


def assert_parity(stats: dict, exempt_frac: float | None = 1e-4, context: str = ""):
    bad = stats["bad"]
    assert bad.size == 0, f"{context}: {bad.size} mismatching pixels, first {bad[:10].tolist()}"
    if exempt_frac is not None:
        assert stats["exempt"] <= max(1, exempt_frac * stats["pixels"]), f"{context}: too many exempt {stats}"


# ---------------------------------------------------------------- BVH layout

def _align(x):
    return (x + 255) & ~255


def bvh_layout(cap: int) -> dict:
    c = max(cap, 1)
    nodes = 256
    leaf_parent = _align(nodes + c * 64)
    node_parent = _align(leaf_parent + c * 4)
    leaf_ids = _align(node_parent + c * 4)
    flags = _align(leaf_ids + c * 4)
    ranges = _align(flags + c * 4)
    entries = _align(ranges + c * 8)
    wide = _align(entries + c * 8)
    return {"nodes": nodes, "leaf_parent": leaf_parent, "node_parent": node_parent, "leaf_ids": leaf_ids,
            "wide": wide}


LEAF = 0x80000000
EMPTY = 0xFFFFFFFF


def bvh_core(mem, cap: int):
    """The BVH bytes that define the hierarchy: everything except the refit's
    list of top-tree entries (appended in a nondeterministic order) and its count."""
    import torch
    c = max(cap, 1)
    lay = bvh_layout(cap)
    ranges = _align(lay["leaf_ids"] + c * 4)       # flags
    ranges = _align(ranges + c * 4)                # ranges
    entries = _align(ranges + c * 8)
    core = mem[:entries].clone() if isinstance(mem, torch.Tensor) else mem[:entries].copy()
    core[4:8] = 0
    return core


def check_bvh(mem: np.ndarray, cap: int, cr: np.ndarray, alpha: np.ndarray) -> dict:
    """Structure of a built BVH: every sphere in exactly one leaf slot with its exact data,
    every internal node reached once, boxes containing their children, sphere boxes
    containing the exact spheres, depth bounded."""
    mem = np.ascontiguousarray(mem).view(np.uint8)
    n = int(mem[:4].view(np.uint32)[0])
    assert n == cr.shape[0]
    scene = mem[8:32].view(np.float32).astype(np.float64)
    lay = bvh_layout(cap)
    n_nodes = max(n - 1, 1)
    f = mem[lay["nodes"]: lay["nodes"] + n_nodes * 64].view(np.float32).reshape(n_nodes, 16)
    refs = f[:, 12:14].copy().view(np.uint32)
    leaf_ids = mem[lay["leaf_ids"]: lay["leaf_ids"] + n * 4].view(np.uint32)
    assert np.array_equal(np.sort(leaf_ids), np.arange(n, dtype=np.uint32)), "leaf ids are not a permutation"
    seen_leaf = np.zeros(n, dtype=np.int64)
    seen_node = np.zeros(n_nodes, dtype=np.int64)
    c64 = cr.astype(np.float64)
    # iterative walk from the root with its box
    stack = [(0, scene[:3], scene[3:], 0)]
    max_depth = 0
    while stack:
        node, lo, hi, depth = stack.pop()
        max_depth = max(max_depth, depth)
        seen_node[node] += 1
        for side in range(2):
            ref = int(refs[node, side])
            s = f[node, 6 * side: 6 * side + 6].astype(np.float64)
            if ref == EMPTY:
                assert n == 1 and side == 1
                continue
            if ref & LEAF:
                sid = ref & ~LEAF
                seen_leaf[sid] += 1
                assert np.array_equal(f[node, 6 * side: 6 * side + 4], cr[sid]), "leaf sphere data differs"
                assert f[node, 6 * side + 4] == alpha[sid], "leaf alpha differs"
                clo, chi = c64[sid, :3] - c64[sid, 3], c64[sid, :3] + c64[sid, 3]
            else:
                clo, chi = s[:3], s[3:]
                stack.append((ref, clo, chi, depth + 1))
            assert np.all(clo >= lo) and np.all(chi <= hi), f"child box escapes node {node}"
    assert np.all(seen_leaf == 1), "a sphere is missing or duplicated"
    assert np.all(seen_node == 1), "an internal node is unreachable or shared"
    assert max_depth < 64
    check_wide(mem, cap, n, f)
    return {"n": n, "depth": max_depth, "leaf_ids": leaf_ids.copy()}


def check_wide(mem: np.ndarray, cap: int, n: int, f: np.ndarray):
    """The 4-wide node of every internal node X, bit for bit, rebuilt here from
    the binary nodes: per child c of X, an internal child C gives its two slots
    (words 12c..12c+11), its two refs (24+2c, 25+2c) and its split axis (29+c);
    a leaf or empty child keeps X's slot, zeros, its ref (an out-of-range
    internal ref becomes EMPTY), EMPTY and axis 3.  Word 28 is X's axis; word 31
    the slot kinds: bit s for a leaf ref below n, bit 4+s for an internal ref
    below the node count."""
    n_nodes = max(n - 1, 1)
    u = f.view(np.uint32)
    w = np.zeros((n_nodes, 32), dtype=np.uint32)
    w[:, 28] = u[:, 14]
    for c in range(2):
        ref = u[:, 12 + c]
        internal = (ref != EMPTY) & ((ref & LEAF) == 0) & (ref < n_nodes)
        C = u[np.where(internal, ref, 0)]
        own = np.concatenate([u[:, 6 * c: 6 * c + 6], np.zeros((n_nodes, 6), np.uint32)], axis=1)
        w[:, 12 * c: 12 * c + 12] = np.where(internal[:, None], C[:, :12], own)
        keep = (ref == EMPTY) | ((ref & LEAF) != 0)
        w[:, 24 + 2 * c] = np.where(internal, C[:, 12], np.where(keep, ref, EMPTY))
        w[:, 25 + 2 * c] = np.where(internal, C[:, 13], EMPTY)
        w[:, 29 + c] = np.where(internal, C[:, 14], 3)
    kinds = np.zeros(n_nodes, dtype=np.uint32)
    for sl in range(4):
        r = w[:, 24 + sl]
        leaf = (r != EMPTY) & ((r & LEAF) != 0)
        inner = (r != EMPTY) & ((r & LEAF) == 0)
        kinds |= np.where(leaf & ((r & ~np.uint32(LEAF)) < n), 1 << sl, 0).astype(np.uint32)
        kinds |= np.where(inner & (r < n_nodes), 1 << (4 + sl), 0).astype(np.uint32)
    w[:, 31] = kinds
    off = bvh_layout(cap)["wide"]
    got = mem[off: off + n_nodes * 128].view(np.uint32).reshape(n_nodes, 32)
    bad = np.nonzero((got != w).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} wide nodes differ from the gather of their binary nodes, first {bad[:8].tolist()}"


# ---------------------------------------------------------------- sampling

def tile_sample(width: int, height: int, tile: int, rng) -> np.ndarray:
    """One random pixel in every tile x tile block of the image (row-major indices)."""
    tx, ty = np.meshgrid(np.arange(0, width, tile), np.arange(0, height, tile))
    px = np.minimum(tx + rng.integers(0, tile, tx.shape), width - 1)
    py = np.minimum(ty + rng.integers(0, tile, ty.shape), height - 1)
    return (py * width + px).ravel()


def project_centres(cr: np.ndarray, cam) -> tuple[np.ndarray, np.ndarray]:
    """Continuous pixel coordinates (x, y) of the sphere centres in `cam` (pinhole, row 0 at the top);
    centres behind the camera get NaN.  Host geometry only: it picks which pixels to check."""
    c = cr[:, :3].astype(np.float64) - np.asarray(cam.eye, dtype=np.float64)
    z = c @ np.asarray(cam.forward, dtype=np.float64)
    x = c @ np.asarray(cam.right, dtype=np.float64)
    y = c @ np.asarray(cam.up, dtype=np.float64)
    aspect = cam.width / cam.height
    with np.errstate(divide="ignore", invalid="ignore"):
        sx = np.where(z > 0, x / (z * cam.tan_half_fov_y * aspect), np.nan)
        sy = np.where(z > 0, y / (z * cam.tan_half_fov_y), np.nan)
    return (sx + 1.0) * 0.5 * cam.width, (1.0 - sy) * 0.5 * cam.height


def silhouette_pixels(cr: np.ndarray, cam, rng, tile: int = 8, count: int = 16) -> np.ndarray:
    """Every pixel of 2 x `count` tiles where the exact tests are hardest: the tiles with the most
    projected sphere centres (the sheet of samples seen edge-on, where rays graze many spheres),
    and tiles on the edge of coverage (centres in the tile, none in a neighbour: silhouettes and
    disocclusion borders).  Chosen from the sphere set alone, never from a GPU result."""
    W, H = cam.width, cam.height
    tx_n, ty_n = (W + tile - 1) // tile, (H + tile - 1) // tile
    x, y = project_centres(cr, cam)
    ok = np.isfinite(x) & np.isfinite(y) & (x >= 0) & (y >= 0) & (x < W) & (y < H)
    t = (y[ok] // tile).astype(np.int64) * tx_n + (x[ok] // tile).astype(np.int64)
    cnt = np.bincount(t, minlength=tx_n * ty_n).reshape(ty_n, tx_n)
    heavy = np.argsort(cnt.ravel(), kind="stable")[::-1][:count]
    pad = np.pad(cnt, 1)
    nb_min = np.min([pad[1 + dy:1 + dy + ty_n, 1 + dx:1 + dx + tx_n]
                     for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx], axis=0)
    edge = np.nonzero(((cnt > 0) & (nb_min == 0)).ravel())[0]
    if edge.size > count:
        edge = rng.choice(edge, size=count, replace=False)
    tiles = np.unique(np.concatenate([heavy, edge]))
    ox, oy = np.meshgrid(np.arange(tile), np.arange(tile))
    px = (tiles % tx_n)[:, None] * tile + ox.ravel()[None, :]
    py = (tiles // tx_n)[:, None] * tile + oy.ravel()[None, :]
    keep = (px < W) & (py < H)
    return np.unique((py * W + px)[keep])


# ---------------------------------------------------------------- build pins

def morton30(cr: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """30-bit Morton codes of the centres in the box [lo, hi], float32 arithmetic: per axis
    u = (p - lo) / (hi - lo) (0 for a flat axis), q = clamp(trunc(1024 u), 0, 1023); bit 3k+2
    of the code is bit k of q_x, 3k+1 of q_y, 3k of q_z."""
    p = cr[:, :3].astype(np.float32)
    lo = np.asarray(lo, dtype=np.float32)
    ext = np.asarray(hi, dtype=np.float32) - lo
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.where(ext > 0, (p - lo) / np.where(ext > 0, ext, np.float32(1)), np.float32(0)).astype(np.float32)
    q = np.clip(np.trunc(u * np.float32(1024.0)), 0, 1023).astype(np.uint32)
    code = np.zeros(p.shape[0], dtype=np.uint32)
    for k in range(10):
        for a, off in ((0, 2), (1, 1), (2, 0)):
            code |= ((q[:, a] >> k) & 1) << (3 * k + off)
    return code


def karras_by_split(keys: np.ndarray, ids: np.ndarray) -> dict:
    """Binary radix tree over sorted keys by recursive splitting: a range [lo, hi] of sorted
    positions splits where the highest bit in which the (key, position) pairs of its two ends
    differ turns from 0 to 1.  Node numbering as in the linear construction: the root is 0, a child
    range [lo, g] is node g and [g + 1, hi] node g + 1, and a single position is a leaf
    (LEAF | sphere id).  Returns {node: (left ref, right ref, split axis)}."""
    n = keys.shape[0]
    aug = [(int(k) << 32) | i for i, k in enumerate(keys)]
    out = {}
    stack = [(0, 0, n - 1)]
    while stack:
        node, lo, hi = stack.pop()
        diff = aug[lo] ^ aug[hi]
        bit = diff.bit_length() - 1
        g = lo
        while g + 1 <= hi and not ((aug[g + 1] >> bit) & 1):
            g += 1
        prefix = 63 - bit  # common leading bits of the 64-bit pair
        axis = 2 - ((31 - prefix) % 3) if prefix < 32 else 3
        left = (LEAF | int(ids[g])) if g == lo else g
        right = (LEAF | int(ids[g + 1])) if g + 1 == hi else g + 1
        out[node] = (left, right, axis)
        if g != lo:
            stack.append((g, lo, g))
        if g + 1 != hi:
            stack.append((g + 1, g + 1, hi))
    return out
