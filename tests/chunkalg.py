"""NumPy model of the chunked (lane-parallel) solve used by the wave kernels (tests only).

A parity chain of nc elements is cut into G chunks of C elements, one chunk
per lane.  The LU factors are recomputed per chunk from the state of the two
(biharmonic) or one (Helmholtz) previous rows at the chunk start; the forward
and backward recurrences become affine maps per chunk, combined across
chunks by a Kogge-Stone scan in the same association order as the kernels.
Checked against the oracle to show the reordering keeps the 1e-12 bar.
"""
import numpy as np

import fastalg as fa


def ks_prefix(items, compose, G):
    """Inclusive Kogge-Stone scan: out[m] = items[m] o ... o items[0] (compose(later, earlier))."""
    cur = list(items)
    d = 1
    while d < G:
        nxt = list(cur)
        for m in range(G):
            if m - d >= 0:
                nxt[m] = compose(cur[m], cur[m - d])
        cur = nxt
        d *= 2
    return cur


def ks_suffix(items, compose, G):
    """Inclusive suffix scan: out[m] = items[m] o items[m+1] o ... (compose(lower, higher))."""
    cur = list(items)
    d = 1
    while d < G:
        nxt = list(cur)
        for m in range(G):
            if m + d < G:
                nxt[m] = compose(cur[m], cur[m + d])
        cur = nxt
        d *= 2
    return cur


def helm_chunked(alpha, f, N, C, G, gl=False):
    n = N - 2
    ns = alpha.shape[0]
    _, d, e, g, _ = fa.helm_factor_forward(alpha, np.zeros((ns, n), complex), N, gl)
    l = np.zeros((ns, n))
    l[:, 2:] = (-0.5 * np.pi * alpha)[:, None] / d[:, :-2]
    u = np.zeros((ns, N), complex)
    for p in (0, 1):
        ks = np.arange(p, n, 2)
        nc = ks.size
        assert nc <= C * G
        idx = np.full(C * G, -1)
        idx[:nc] = ks
        ok = idx >= 0
        ii = np.where(ok, idx, 0)
        L = np.where(ok, l[:, ii], 0.0)
        rd = np.where(ok, 1.0 / d[:, ii], 0.0)
        gg = np.where(ok, g[:, ii], 0.0)
        ee = gg + (-0.5 * np.pi * alpha)[:, None]
        x = np.where(ok, f[:, ii], 0.0)
        # forward: y_i = x_i - L_i y_{i-1}
        y0 = np.zeros_like(x)
        T = np.ones((ns, G))
        ylast = np.zeros((ns, G), complex)
        for m in range(G):
            prev = np.zeros(ns, complex)
            for j in range(C):
                i = m * C + j
                y0[:, i] = x[:, i] - L[:, i] * prev
                prev = y0[:, i]
                T[:, m] *= -L[:, i]
            ylast[:, m] = prev
        items = [(T[:, m], ylast[:, m]) for m in range(G)]
        comp = lambda b, a: (b[0] * a[0], b[0] * a[1] + b[1])  # b after a
        inc = ks_prefix(items, comp, G)
        y = y0.copy()
        for m in range(1, G):
            sin = inc[m - 1][1]
            h = sin
            for j in range(C):
                i = m * C + j
                h = -L[:, i] * h
                y[:, i] = y0[:, i] + h
        # backward: state (a=u_{i+1}, S=S_{i+2}); u_i = rd(y - e a - g S); new (u_i, S + a)
        yh = rd * y
        eh = rd * ee
        gh = rd * gg
        A = np.zeros((ns, G, 2, 2))
        cvec = np.zeros((ns, G, 2), complex)
        for m in range(G):
            Am = np.tile(np.eye(2), (ns, 1, 1))
            c = np.zeros((ns, 2), complex)
            for j in range(C - 1, -1, -1):
                i = m * C + j
                Mj = np.zeros((ns, 2, 2))
                Mj[:, 0, 0] = -eh[:, i]
                Mj[:, 0, 1] = -gh[:, i]
                Mj[:, 1, 0] = 1.0
                Mj[:, 1, 1] = 1.0
                Am = np.einsum("sab,sbc->sac", Mj, Am)
                c = np.einsum("sab,sb->sa", Mj, c) + np.stack([yh[:, i], np.zeros(ns)], 1)
            A[:, m] = Am
            cvec[:, m] = c
        items = [(A[:, m], cvec[:, m]) for m in range(G)]
        compb = lambda lo, hi: (np.einsum("sab,sbc->sac", lo[0], hi[0]), np.einsum("sab,sb->sa", lo[0], hi[1]) + lo[1])
        inc = ks_suffix(items, compb, G)
        out = np.zeros_like(x)
        for m in range(G):
            s = inc[m + 1][1] if m + 1 < G else np.zeros((ns, 2), complex)
            a, S = s[:, 0], s[:, 1]
            for j in range(C - 1, -1, -1):
                i = m * C + j
                ui = yh[:, i] - eh[:, i] * a - gh[:, i] * S
                out[:, i] = ui
                a, S = ui, S + a
        u[:, ks] = out[:, :nc]
    return u


def bih_chunked(a, b, f, N, C, G, gl=False):
    n = N - 4
    ns = a.shape[0]
    U0, U2, U4, P, R, L1, L2, _ = fa.bih_factor_forward(a, b, np.zeros((ns, n), complex), N, gl)
    u = np.zeros((ns, N), complex)
    for p in (0, 1):
        ks = np.arange(p, n, 2)
        nc = ks.size
        assert nc <= C * G
        idx = np.full(C * G, -1)
        idx[:nc] = ks
        ok = idx >= 0
        ii = np.where(ok, idx, 0)
        z = lambda arr: np.where(ok, arr[:, ii], 0.0)
        l1, l2 = z(L1), z(L2)
        r0 = np.where(ok, 1.0 / U0[:, ii], 0.0)
        u2h, u4h, ph, rh = r0 * z(U2), r0 * z(U4), r0 * z(P), r0 * z(R)
        kk = np.where(ok, idx, 0).astype(float)
        q4 = 1.0 / (kk + 7.0)
        s4 = (kk + 6.0) ** 2 / (kk + 7.0)
        x = np.where(ok, f[:, ii], 0.0)
        # forward: y_i = x_i - l1 y_{i-1} - l2 y_{i-2}; state (y_i, y_{i-1})
        y0 = np.zeros_like(x)
        items = []
        for m in range(G):
            T = np.tile(np.eye(2), (ns, 1, 1))
            s = np.zeros((ns, 2), complex)
            for j in range(C):
                i = m * C + j
                Mj = np.zeros((ns, 2, 2))
                Mj[:, 0, 0] = -l1[:, i]
                Mj[:, 0, 1] = -l2[:, i]
                Mj[:, 1, 0] = 1.0
                T = np.einsum("sab,sbc->sac", Mj, T)
                yi = x[:, i] - l1[:, i] * s[:, 0] - l2[:, i] * s[:, 1]
                y0[:, i] = yi
                s = np.stack([yi, s[:, 0]], 1)
            items.append((T, s))
        comp = lambda later, earlier: (np.einsum("sab,sbc->sac", later[0], earlier[0]),
                                       np.einsum("sab,sb->sa", later[0], earlier[1]) + later[1])
        inc = ks_prefix(items, comp, G)
        zero = np.zeros((ns, 2), complex)
        shat = [zero] + [inc[m - 1][1] for m in range(1, G)]
        # refinement sweep: rerun each chunk from f and its scanned state, scan the
        # defects e_m - shat_{m+1} with the same transfers, add the response
        y = np.zeros_like(x)
        defects = []
        for m in range(G):
            s = shat[m].copy()
            for j in range(C):
                i = m * C + j
                yi = x[:, i] - l1[:, i] * s[:, 0] - l2[:, i] * s[:, 1]
                y[:, i] = yi
                s = np.stack([yi, s[:, 0]], 1)
            defects.append(s - (shat[m + 1] if m + 1 < G else s))
        inc2 = ks_prefix([(items[m][0], defects[m]) for m in range(G)], comp, G)
        for m in range(1, G):
            h = inc2[m - 1][1].copy()
            for j in range(C):
                i = m * C + j
                hi = -l1[:, i] * h[:, 0] - l2[:, i] * h[:, 1]
                y[:, i] = y[:, i] + hi
                h = np.stack([hi, h[:, 0]], 1)
        yh = r0 * y
        items = []
        for m in range(G):
            A = np.tile(np.eye(4), (ns, 1, 1))
            c = np.zeros((ns, 4), complex)
            for j in range(C - 1, -1, -1):
                i = m * C + j
                Mj = np.zeros((ns, 4, 4))
                Mj[:, 0, 0], Mj[:, 0, 1], Mj[:, 0, 2], Mj[:, 0, 3] = -u2h[:, i], -u4h[:, i], -ph[:, i], -rh[:, i]
                Mj[:, 1, 0] = 1.0
                Mj[:, 2, 1], Mj[:, 2, 2] = q4[i], 1.0
                Mj[:, 3, 1], Mj[:, 3, 3] = s4[i], 1.0
                A = np.einsum("sab,sbc->sac", Mj, A)
                e = np.zeros((ns, 4), complex)
                e[:, 0] = yh[:, i]
                c = np.einsum("sab,sb->sa", Mj, c) + e
            items.append((A, c))
        compb = lambda lo, hi: (np.einsum("sab,sbc->sac", lo[0], hi[0]), np.einsum("sab,sb->sa", lo[0], hi[1]) + lo[1])
        inc = ks_suffix(items, compb, G)
        out = np.zeros_like(x)
        for m in range(G):
            s = inc[m + 1][1] if m + 1 < G else np.zeros((ns, 4), complex)
            aa, bb, cq, cs = s[:, 0], s[:, 1], s[:, 2], s[:, 3]
            for j in range(C - 1, -1, -1):
                i = m * C + j
                ui = yh[:, i] - u2h[:, i] * aa - u4h[:, i] * bb - ph[:, i] * cq - rh[:, i] * cs
                out[:, i] = ui
                aa, bb, cq, cs = ui, aa, cq + q4[i] * bb, cs + s4[i] * bb
        u[:, ks] = out[:, :nc]
    return u


def mass_chunked(family, f, N, C, G, gl=False):
    """u = B^{-1} f (Dirichlet or biharmonic mass matrix) by the chunked scheme of the
    mass-solve kernels: one shared LU per parity chain (no pivoting), then per chunk
    the forward and backward recurrences of bandwidth s = 1 or 2 as affine maps on
    the s-vector state, combined by Kogge-Stone scans, and each chunk rerun from its
    scanned incoming state."""
    from oracle import shen_oracle as so
    quad = so.GL if gl else so.GC
    B = so.mass_matrix(family, N, quad)
    n = B.shape[0]
    s = 1 if family == "helmholtz" else 2
    ns = f.shape[0]
    u = np.zeros((ns, N), complex)
    for p in (0, 1):
        ks = np.arange(p, n, 2)
        nc = ks.size
        assert nc <= C * G
        M = B[np.ix_(ks, ks)]
        # banded LU without pivoting: lo[i, t] = L_{i, i-1-t}, up[i, t] = U_{i, i+1+t}
        lo = np.zeros((C * G, s))
        up = np.zeros((C * G, s))
        rd = np.ones(C * G)
        Uf = M.copy()
        for i in range(nc):
            # eliminate row i by rows i-s .. i-1 (in order)
            for r in range(max(0, i - s), i):
                lo[i, i - 1 - r] = Uf[i, r] / Uf[r, r]
                Uf[i, r:r + s + 1] -= lo[i, i - 1 - r] * Uf[r, r:r + s + 1]
            rd[i] = 1.0 / Uf[i, i]
            for t in range(s):
                if i + 1 + t < nc:
                    up[i, t] = Uf[i, i + 1 + t]
        x = np.zeros((ns, C * G), complex)
        x[:, :nc] = f[:, ks]

        # forward: y_i = x_i - sum_t lo[i, t] y_{i-1-t}; chunk map on (y_{i-1}, ..., y_{i-s})
        def fwd_map(m):
            rows = range(m * C, m * C + C)
            A = np.eye(s)
            c = np.zeros((ns, s), complex)
            for i in rows:
                comp = np.zeros((s, s))
                comp[0, :] = -lo[i]
                comp[1:, :-1] = np.eye(s)[:-1, :-1] if s > 1 else comp[1:, :-1]
                A = comp @ A
                c = c @ comp.T
                c[:, 0] += x[:, i]
            return A, c

        items = [fwd_map(m) for m in range(G)]
        comp_f = lambda b, a: (b[0] @ a[0], a[1] @ b[0].T + b[1])
        inc = ks_prefix(items, comp_f, G)
        y = np.zeros_like(x)
        for m in range(G):
            st = inc[m - 1][1] if m > 0 else np.zeros((ns, s), complex)
            for i in range(m * C, m * C + C):
                v = x[:, i] - sum(lo[i, t] * st[:, t] for t in range(s))
                y[:, i] = v
                st = np.concatenate([v[:, None], st[:, :-1]], axis=1)
        # backward: u_i = rd_i (y_i - sum_t up[i, t] u_{i+1+t}); chunk map on (u_{i+1}, ..., u_{i+s})
        def bwd_map(m):
            A = np.eye(s)
            c = np.zeros((ns, s), complex)
            for i in range(m * C + C - 1, m * C - 1, -1):
                comp = np.zeros((s, s))
                comp[0, :] = -rd[i] * up[i]
                if s > 1:
                    comp[1, 0] = 1.0
                A = comp @ A
                c = c @ comp.T
                c[:, 0] += rd[i] * y[:, i]
            return A, c

        items = [bwd_map(m) for m in range(G)]
        comp_b = lambda lo_, hi: (lo_[0] @ hi[0], hi[1] @ lo_[0].T + lo_[1])
        inc = ks_suffix(items, comp_b, G)
        out = np.zeros_like(x)
        for m in range(G):
            st = inc[m + 1][1] if m + 1 < G else np.zeros((ns, s), complex)
            for i in range(m * C + C - 1, m * C - 1, -1):
                v = rd[i] * (y[:, i] - sum(up[i, t] * st[:, t] for t in range(s)))
                out[:, i] = v
                st = np.concatenate([v[:, None], st[:, :-1]], axis=1)
        u[:, ks] = out[:, :nc]
    return u
