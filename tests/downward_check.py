"""Element-by-element check of a computed downward pass (M2F, M2L, F2L, L2L,
L2P and P2P), used at sizes where the oracle cannot run the whole matvec.

Sampled local expansions are rebuilt by the oracle's single-expansion
operators from the checked run's own multipoles (M2L in the circulant form
over the target's M2L list, Sec. 2.3) and its father's locals (L2L, Sec. 2.2);
sampled leaves' potentials are rebuilt by the oracle's L2P from the run's
locals plus the direct sum over every P2P pair whose target cell holds the
leaf (Alg. 1 keeps a non-leaf partner's whole point range).  Each result is
compared within `tol` of its largest magnitude.
"""
import numpy as np

import oracle


def downward_check(*, kappa, L, kernel, hf_threshold, dir_refine, D, origin, tree, m2l, p2p, mult, loc,
                   X, q, p, n_local, n_leaf, tol, seed):
    """tree: dict(level, ijk, first, count, is_leaf, perm) of the one tree (X = Y);
    m2l: dict(level, t, s, delta, dir); p2p: dict(t, s); mult / loc: (cell, dir,
    values [n x L^3]) of the multipole and local expansions; X, q, p in caller
    order.  Returns the numbers of locals and leaves checked."""
    screened = kernel == oracle.YUKAWA
    lev, ijk = np.asarray(tree["level"]), np.asarray(tree["ijk"]).astype(np.int64)
    cell_of = {(int(l), *map(int, c)): i for i, (l, c) in enumerate(zip(lev, ijk))}

    def parent(c):
        return cell_of[(int(lev[c]) - 1, *map(int, ijk[c] >> 1))] if lev[c] > 0 else -1

    def geom(c):
        h = D / 2.0 ** lev[c]
        return origin + h * ijk[c], h

    nlev = int(lev.max()) + 2
    hf = [not screened and kappa * D / 2.0 ** (l + 1) > hf_threshold for l in range(nlev)]
    lstar = max([l for l in range(nlev) if hf[l]], default=-1)
    dirs = {}

    def dset(E):
        if E not in dirs:
            dirs[E] = oracle.directions(E)
        return dirs[E]

    def direction(level, u):
        return None if u < 0 else dset(lstar - level + dir_refine)[0][u]

    mc, md, mv = mult
    lc, ld, lv = loc
    mv = np.asarray(mv).astype(np.complex128)
    lv = np.asarray(lv).astype(np.complex128)
    iM = {(int(c), int(u)): e for e, (c, u) in enumerate(zip(mc, md))}
    locs_of = {}
    for e, c in enumerate(lc):
        locs_of.setdefault(int(c), []).append(e)
    key = np.asarray(m2l["t"]).astype(np.int64) * 1_000_000 + (np.asarray(m2l["dir"]).astype(np.int64) + 1)
    order = np.argsort(key, kind="stable")
    skey = key[order]
    rng = np.random.default_rng(seed)

    checked_local = 0
    for e in rng.choice(len(lc), size=min(4 * n_local, len(lc)), replace=False):
        t, u = int(lc[e]), int(ld[e])
        l = int(lev[t])
        at, ht = geom(t)
        acc = np.zeros(L ** 3, dtype=complex)
        k = t * 1_000_000 + u + 1
        a, b = np.searchsorted(skey, k), np.searchsorted(skey, k, side="right")
        for j in order[a:b]:
            acc += oracle.m2l_fft(kappa, ht, L, m2l["delta"][j], mv[iM[(int(m2l["s"][j]), u)]], kernel=kernel)
        par = parent(t)
        if par >= 0:
            ap, hp = geom(par)
            for f in locs_of.get(par, []):
                v = int(ld[f])
                fv = int(dset(lstar - l + 1 + dir_refine)[1][v]) if hf[l] else -1
                if fv == u:
                    acc += oracle.l2l(kappa, L, ap, hp, direction(l - 1, v), at, ht, lv[f])
        if not np.abs(acc).max() > 0:
            continue
        err = np.abs(lv[e] - acc).max() / np.abs(acc).max()
        assert err <= tol, ("local expansion", t, u, err)
        checked_local += 1
        if checked_local >= n_local:
            break

    perm = np.asarray(tree["perm"])
    first, count = np.asarray(tree["first"]), np.asarray(tree["count"])
    pt = np.asarray(p2p["t"])
    po = np.argsort(pt, kind="stable")
    pts_t = pt[po]
    xs, qs, ps = X[perm], q[perm], np.asarray(p)[perm].astype(np.complex128)
    leaves = np.nonzero(np.asarray(tree["is_leaf"]))[0]
    checked_leaf = 0
    for t in rng.choice(leaves, size=min(n_leaf, len(leaves)), replace=False):
        t = int(t)
        sl = slice(int(first[t]), int(first[t] + count[t]))
        x = xs[sl]
        at, ht = geom(t)
        acc = np.zeros(len(x), dtype=complex)
        for f in locs_of.get(t, []):
            acc += oracle.l2p(kappa, L, at, ht, direction(int(lev[t]), int(ld[f])), lv[f], x)
        c = t
        while c >= 0:
            a, b = np.searchsorted(pts_t, c), np.searchsorted(pts_t, c, side="right")
            for j in po[a:b]:
                s = int(p2p["s"][j])
                ss = slice(int(first[s]), int(first[s] + count[s]))
                acc += oracle.direct_sum(x, xs[ss], qs[ss], kappa, 1e-12 * D, kernel=kernel)
            c = parent(c)
        err = np.abs(ps[sl] - acc).max() / np.abs(acc).max()
        assert err <= tol, ("leaf potentials", t, err)
        checked_leaf += 1
    return checked_local, checked_leaf
