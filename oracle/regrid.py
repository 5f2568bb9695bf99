"""Reference regrid of a Mesh -- TEST INFRASTRUCTURE ONLY.

Plan (Sec. 3.3 criteria drive the mesh; the 2:1 rule of Sec. 3): flags
+1/-1/0 per block give new octree leaves.  A refined block becomes its
eight children (same cell count, one level finer); eight flagged sibling
leaves merge into their parent.  The 2:1 rule is checked on a raster of
the whole domain at the finest level: the cells within the stencil reach
of a block (2g of the finer block's cells, periodic wrap or clipped at an
outflow boundary) may not belong to a block two or more levels coarser.

Transfer (Sec. 3.1, Eqs. 1-2, Lagrange interpolation with n = g+1 nodes per
axis, tensor product): a refined block's fine cells are interpolated from
the n coarse centres nearest to each fine centre, in the parent's
ghost-filled data; a merged block's coarse cells from the n fine centres
of the owning child nearest to the coarse centre (ties towards the child's
interior).  Node sets and weights are built per axis from these
definitions and applied as dense weight matrices.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle

NF = oracle.NF


# ------------------------------------------------------------------ plan

def _raster(mesh, levels, F):
    """Finest-level raster of per-block values `levels` (int array)."""
    N = [int(mesh.nroot[a]) << F for a in range(3)]
    R = np.full((N[2], N[1], N[0]), -1, dtype=np.int16)
    for b in range(mesh.nb):
        s = 1 << (F - int(mesh.level[b]))
        lo = [int(mesh.ilo[b, a]) * s for a in range(3)]
        hi = [(int(mesh.ilo[b, a]) + int(mesh.n[b])) * s for a in range(3)]
        R[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = levels[b]
    return R


def _dilate(mask, r, periodic):
    """Box dilation by r cells per axis (wrap if periodic, else clipped)."""
    out = mask.copy()
    for ax in range(3):
        cur = out.copy()
        for d in range(1, r + 1):
            for sgn in (1, -1):
                if periodic:
                    cur |= np.roll(out, sgn * d, axis=ax)
                else:
                    sh = np.zeros_like(out)
                    if sgn > 0:
                        sl_dst = [slice(None)] * 3
                        sl_src = [slice(None)] * 3
                        sl_dst[ax] = slice(d, None)
                        sl_src[ax] = slice(None, -d)
                    else:
                        sl_dst = [slice(None)] * 3
                        sl_src = [slice(None)] * 3
                        sl_dst[ax] = slice(None, -d)
                        sl_src[ax] = slice(d, None)
                    sh[tuple(sl_dst)] = out[tuple(sl_src)]
                    cur |= sh
        out = cur
    return out


def _box(mesh, b, F):
    s = 1 << (F - int(mesh.level[b]))
    return tuple(slice(int(mesh.ilo[b, a]) * s, (int(mesh.ilo[b, a]) + int(mesh.n[b])) * s)
                 for a in (2, 1, 0))


def _violations(mesh, t, F, periodic):
    """Per block: the largest target level within the reach of its cells
    among levels at least two above its own target (else -1)."""
    g = mesh.g
    R = _raster(mesh, t, F)
    worst = np.full(mesh.nb, -1)
    for lev in range(int(t.max()), 1, -1):
        reach = 2 * g * (1 << (F - lev))
        near = _dilate(R >= lev, reach, periodic)
        for b in range(mesh.nb):
            if t[b] <= lev - 2 and near[_box(mesh, b, F)].any():
                worst[b] = max(worst[b], lev)
    return worst


def plan(mesh, flags, level_max: int):
    """New block list (a Mesh) under the rules above, in the old order with
    children (z, y, x) in place of their parent and a merged parent in
    place of its first child."""
    flags = np.asarray(flags, dtype=int)
    lev = np.asarray(mesh.level, dtype=int)
    t = lev + ((flags > 0) & (lev < level_max)).astype(int)
    F = int(max(t.max(), lev.max()))
    periodic = mesh.bc == 0
    while True:
        w = _violations(mesh, t, F, periodic)
        bad = w >= 0
        if not bad.any():
            break
        t = np.where(bad, np.maximum(t, w - 1), t)
    # sibling groups of eight flagged leaves
    groups = {}
    for b in range(mesh.nb):
        n = int(mesh.n[b])
        ilo = tuple(int(v) for v in mesh.ilo[b])
        if flags[b] != -1 or t[b] != lev[b] or lev[b] < 1 or any(v % n for v in ilo):
            continue
        groups.setdefault((lev[b], n) + tuple(v // (2 * n) for v in ilo), []).append(b)
    groups = [m for m in groups.values() if len(m) == 8]
    live = [True] * len(groups)
    for m in groups:
        t[m] = lev[m] - 1
    # the merged parent is the union of its children: a child's box violating
    # the rule at the parent's level means the parent does
    while True:
        w = _violations(mesh, t, F, periodic)
        changed = False
        for i, m in enumerate(groups):
            if live[i] and (w[m] >= 0).any():
                live[i] = False
                t[m] = lev[m]
                changed = True
        if not changed:
            break
    first = {}
    for i, m in enumerate(groups):
        if live[i]:
            for b in m:
                first[b] = min(m)
    L, Nn, I = [], [], []
    for b in range(mesh.nb):
        n = int(mesh.n[b])
        if b in first:
            if first[b] == b:
                L.append(lev[b] - 1)
                Nn.append(n)
                I.append([int(v) // 2 // n * n for v in mesh.ilo[b]])
        elif t[b] > lev[b]:
            for cz in range(2):
                for cy in range(2):
                    for cx in range(2):
                        L.append(lev[b] + 1)
                        Nn.append(n)
                        I.append([2 * int(mesh.ilo[b, 0]) + cx * n, 2 * int(mesh.ilo[b, 1]) + cy * n,
                                  2 * int(mesh.ilo[b, 2]) + cz * n])
        else:
            L.append(lev[b])
            Nn.append(n)
            I.append([int(v) for v in mesh.ilo[b]])
    return dataclasses.replace(mesh, level=np.array(L, dtype=np.int32), n=np.array(Nn, dtype=np.int32),
                               ilo=np.array(I, dtype=np.int32).reshape(-1, 3))


def two_to_one_ok(mesh) -> bool:
    """The rule above on a given mesh (raster check)."""
    lev = np.asarray(mesh.level, dtype=int)
    return not (_violations(mesh, lev, int(lev.max()), mesh.bc == 0) >= 0).any()


# -------------------------------------------------------------- transfer

def lagrange(nodes, x):
    """Weights of the Lagrange polynomial through `nodes` evaluated at x."""
    nodes = np.asarray(nodes, dtype=float)
    w = np.ones(len(nodes))
    for i, xi in enumerate(nodes):
        for j, xj in enumerate(nodes):
            if i != j:
                w[i] *= (x - xj) / (xi - xj)
    return w


def _prolong_nodes(ilo_f, n, np_):
    """Per fine cell ilo_f .. ilo_f+n-1 (global, fine level): the global
    indices of the np coarse centres nearest its centre, and their weights."""
    rows = []
    for i in range(ilo_f, ilo_f + n):
        x = (i + 0.5) / 2.0                       # fine centre, coarse units
        J = i // 2
        cand = np.arange(J - np_, J + np_ + 1)
        d = np.abs(cand + 0.5 - x)
        nodes = np.sort(cand[np.argsort(d, kind="stable")[:np_]])
        rows.append((nodes, lagrange(nodes + 0.5, x)))
    return rows


def _restrict_nodes(K, c_lo, c_n, np_):
    """Fine indices (global) of the np fine centres of the child [c_lo,
    c_lo + c_n) nearest the centre of coarse cell K, ties to the interior."""
    x = 2.0 * K + 1.0                             # coarse centre, fine units
    cand = np.arange(c_lo, c_lo + c_n)
    d = np.abs(cand + 0.5 - x)
    dc = np.abs(cand + 0.5 - (c_lo + c_n / 2.0))
    order = np.lexsort((dc, d))
    return np.sort(cand[order[:np_]]), x


def transfer(old_mesh, old_u, new_mesh, fill: bool = True):
    """Per-block interiors (22, n, n, n) of new_mesh from the old register
    `old_u` (oracle layout); the old ghosts are filled first unless fill is
    False (then they must hold valid values)."""
    om = oracle.OracleMesh(old_mesh)
    u = old_u.copy()
    if fill:
        oracle.fill_ghosts(om, u)
    g = old_mesh.g
    np_ = g + 1
    key = {(int(old_mesh.level[b]), int(old_mesh.n[b])) + tuple(int(v) for v in old_mesh.ilo[b]): b
           for b in range(old_mesh.nb)}
    out = []
    for d in range(new_mesh.nb):
        l, n = int(new_mesh.level[d]), int(new_mesh.n[d])
        ilo = [int(v) for v in new_mesh.ilo[d]]
        b = key.get((l, n) + tuple(ilo))
        if b is not None:
            out.append(om.block_view(u, b)[:, g:g + n, g:g + n, g:g + n].copy())
            continue
        parent = None
        for c in range(old_mesh.nb):
            if int(old_mesh.level[c]) != l - 1:
                continue
            cl, cn = [int(v) for v in old_mesh.ilo[c]], int(old_mesh.n[c])
            if all(2 * cl[a] <= ilo[a] and ilo[a] + n <= 2 * (cl[a] + cn) for a in range(3)):
                parent = c
                break
        if parent is not None:
            P = om.block_view(u, parent)
            cl = [int(v) for v in old_mesh.ilo[parent]]
            EP = P.shape[1]
            W = []
            for a in range(3):
                M = np.zeros((n, EP))
                for r, (nodes, w) in enumerate(_prolong_nodes(ilo[a], n, np_)):
                    M[r, nodes - cl[a] + g] = w
                W.append(M)
            out.append(np.einsum("xi,yj,zk,fkji->fzyx", W[0], W[1], W[2], P, optimize=True))
            continue
        # restriction from the eight children
        res = np.empty((NF, n, n, n))
        kids = {}
        for c8 in range(8):
            cx, cy, cz = c8 & 1, (c8 >> 1) & 1, c8 >> 2
            kid = key.get((l + 1, n, 2 * ilo[0] + cx * n, 2 * ilo[1] + cy * n, 2 * ilo[2] + cz * n))
            if kid is None:
                raise ValueError(f"block {d} is neither kept, refined nor merged")
            kids[(cx, cy, cz)] = kid
        h = n // 2
        for (cx, cy, cz), kid in kids.items():
            Cb = om.block_view(u, kid)[:, g:g + n, g:g + n, g:g + n]
            kl = [int(v) for v in old_mesh.ilo[kid]]
            W = []
            for a, ca in enumerate((cx, cy, cz)):
                M = np.zeros((h, n))
                for r in range(h):
                    K = ilo[a] + ca * h + r
                    nodes, x = _restrict_nodes(K, kl[a], n, np_)
                    M[r, nodes - kl[a]] = lagrange(nodes + 0.5, x)
                W.append(M)
            res[:, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h] = np.einsum(
                "xi,yj,zk,fkji->fzyx", W[0], W[1], W[2], Cb, optimize=True)
        out.append(res)
    return out
