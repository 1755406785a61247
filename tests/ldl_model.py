"""Host model of the blocked LDL^H factorisation of the shifted solves (the
GPU panel, lower-triangle trailing update and back-substitution): the same
slot layout (matrix, right-hand side, candidate column, look-ahead window,
W = L D), the same order of steps and the same pivot rule (Bunch and
Kaufman, Math. Comp. 31, 1977), in binary64 complex arithmetic.  Test
infrastructure: it checks the blocking scheme's bookkeeping (windows,
symmetric interchanges, panels that end before a 2x2 block, the per-panel
undo of interchanges) on the CPU; the GPU kernels are checked against the
oracle by the GPU tests.
"""
import numpy as np

NB, LA = 32, 4
ALPHA = 0.64038820320220756872767623199676
IP2 = -2147483648


def mag1(z):
    return abs(z.real) + abs(z.imag)


def panel(M, ipiv, n, k0, ptol, st):
    bc, xc, vc0, wb = n, n + 1, n + 2, n + 2 + LA
    kend = min(k0 + NB, n)
    wbase = wend = k0
    k = k0
    while k < kend:
        nk = k - k0
        if k >= wend:
            wbase, wend = k, min(k + LA, kend)
            nw = wend - wbase
            swt = np.zeros((LA, NB), complex)
            for j in range(nw):
                for c in range(nk):
                    swt[j, c] = np.conj(M[wbase + j, wb + c])
            for r in range(k, n):
                for j in range(nw):
                    col = wbase + j
                    z = M[r, col] if r >= col else np.conj(M[col, r])
                    for c in range(nk):
                        z -= M[r, k0 + c] * swt[j, c]
                    M[r, vc0 + j] = z
        vk = vc0 + (k - wbase)
        best, bi = -1.0, n
        for r in range(k + 1, n):
            m = mag1(M[r, vk])
            if m > best:
                best, bi = m, r
        colmax = max(best, 0.0)
        imax = bi
        absakk = abs(M[k, vk].real)
        cand = not (colmax < max(ptol, 1e-300) or absakk >= ALPHA * colmax)
        rowmax = absimax = 0.0
        xv = vc0 + (imax - wbase) if (cand and imax < wend) else xc
        if cand:
            if imax >= wend:
                s = [np.conj(M[imax, wb + c]) for c in range(nk)]
                for r in range(k, n):
                    z = M[r, imax] if r >= imax else np.conj(M[imax, r])
                    for c in range(nk):
                        z -= M[r, k0 + c] * s[c]
                    M[r, xc] = z
            rb = 0.0
            for r in range(k, n):
                if r != imax:
                    rb = max(rb, mag1(M[r, xv]))
            rowmax = rb
            absimax = abs(M[imax, xv].real)
        kstep, kp = 1, k
        if cand:
            if absakk >= ALPHA * colmax * (colmax / rowmax):
                kp = k
            elif absimax >= ALPHA * rowmax:
                kp = imax
            else:
                kstep, kp = 2, imax
        if kstep == 2 and k + 1 >= kend:
            break
        st['cand'] += cand
        st['swap'] += kp != k + kstep - 1
        st['2x2'] += kstep == 2
        st['kp_in'] += (kp != k + kstep - 1) and kp < wend
        kk = k + kstep - 1
        v0 = vk
        v1 = (vk + 1 if k + 1 < wend else xc) if kstep == 2 else vk
        if kp != kk:
            kp_in = kp < wend
            for c in range(nk):
                M[[kk, kp], k0 + c] = M[[kp, kk], k0 + c]
                M[[kk, kp], wb + c] = M[[kp, kk], wb + c]
            for r in range(kk + 1, n):
                if r < kp:
                    M[kp, r] = np.conj(M[r, kk])
                elif r > kp:
                    M[r, kp] = M[r, kk]
            vkk = vc0 + (kk - wbase)
            if kk < wend:
                if kp_in:
                    vkp = vc0 + (kp - wbase)
                    M[k:n, [vkk, vkp]] = M[k:n, [vkp, vkk]]
                else:
                    M[k:n, vkk] = M[k:n, xc]
            M[[kk, kp], bc] = M[[kp, kk], bc]
            M[kp, kp] = M[kk, kk]
            nlive = wend - k
            for t in range(nlive):
                M[[kk, kp], vk + t] = M[[kp, kk], vk + t]
            if v1 == xc and kstep == 2:
                M[[kk, kp], xc] = M[[kp, kk], xc]
        j1 = k + kstep
        if kstep == 1:
            d = M[k, v0].real
            if abs(d) < ptol:
                d = ptol if d >= 0 else -ptol
            inv = 1.0 / d
            M[k, k] = d
            ipiv[k] = kp
            y = M[k, bc]
        else:
            d11, d22, d21 = M[k, v0].real, M[k + 1, v1].real, M[k + 1, v0]
            det = d11 * d22 - abs(d21) ** 2
            idet = 1.0 / det
            M[k, k] = d11
            M[k + 1, k + 1] = d22
            M[k + 1, k] = d21
            ipiv[k] = -(kp + 1)
            ipiv[k + 1] = IP2
            y0, y1 = M[k, bc], M[k + 1, bc]
        for q in range(kstep):
            ipiv[n + k + q] = 1 if k + q == k0 else 0
        nl = max(0, wend - j1)
        spj0 = [np.conj(M[j1 + t, v0]) for t in range(nl)]
        spj1 = [np.conj(M[j1 + t, v1]) for t in range(nl)] if kstep == 2 else None
        vj1 = vc0 + (j1 - wbase)
        for r in range(j1, n):
            if kstep == 1:
                w = M[r, v0]
                l = w * inv
                M[r, k] = l
                M[r, wb + nk] = w
                M[r, bc] -= l * y
                for t in range(nl):
                    M[r, vj1 + t] -= l * spj0[t]
            else:
                a, b2 = M[r, v0], M[r, v1]
                l0 = (a * d22 - b2 * d21) * idet
                l1 = (b2 * d11 - a * np.conj(d21)) * idet
                M[r, k] = l0
                M[r, k + 1] = l1
                M[r, wb + nk] = a
                M[r, wb + nk + 1] = b2
                M[r, bc] -= l0 * y0 + l1 * y1
                for t in range(nl):
                    M[r, vj1 + t] -= l0 * spj0[t] + l1 * spj1[t]
        k += kstep
    return k0, k - k0


def update(M, n, k0, kb):
    r0 = k0 + kb
    wb = n + 2 + LA
    if r0 >= n:
        return
    W = M[r0:n, wb:wb + kb]
    Lm = M[r0:n, k0:k0 + kb]
    U = np.conj(W).T
    full = Lm @ U
    # lower triangle (and the whole diagonal-tile region is harmless)
    for j in range(r0, n):
        M[j:n, j] -= full[j - r0:, j - r0]


def backsolve(M, ipiv, n):
    yc = n
    x = M[:n, yc].copy()
    i = 0
    while i < n:
        p = ipiv[i]
        if p >= 0:
            x[i] = x[i] / M[i, i].real
            i += 1
        else:
            d11, d22, d21 = M[i, i].real, M[i + 1, i + 1].real, M[i + 1, i]
            idet = 1 / (d11 * d22 - abs(d21) ** 2)
            y0, y1 = x[i], x[i + 1]
            x[i] = (d22 * y0 - np.conj(d21) * y1) * idet
            x[i + 1] = (d11 * y1 - d21 * y0) * idet
            i += 2
    pend = n
    i = n - 1
    while i >= 0:
        two = ipiv[i] == IP2
        c0 = i - 1 if two else i
        s0 = np.conj(M[i + 1:n, i]) @ x[i + 1:n]
        x[i] -= s0
        if two:
            x[c0] -= np.conj(M[i + 1:n, c0]) @ x[i + 1:n]
        if ipiv[n + c0] == 1:
            j = pend - 1
            while j >= c0:
                p = ipiv[j]
                if p == IP2:
                    kpp = -ipiv[j - 1] - 1
                    x[[j, kpp]] = x[[kpp, j]]
                    j -= 1
                elif p >= 0 and p != j:
                    x[[j, p]] = x[[p, j]]
                j -= 1
            pend = c0
        i = c0 - 1
    return x


def solve(A, b, ptol=0.0, st=None, la=None):
    """x with (A) x = b through the blocked factorisation (A Hermitian; its
    lower triangle is read); st counts candidates, interchanges (inside the
    window too) and 2x2 blocks."""
    global LA
    if la is not None:
        LA = la
    n = A.shape[0]
    M = np.zeros((n, n + 2 + LA + NB), complex)
    M[:, :n] = A
    M[:, n] = b
    ipiv = np.zeros(2 * n, int)
    st = st if st is not None else dict(cand=0, swap=0, kp_in=0)
    st.setdefault('2x2', 0)
    lk0 = lkb = 0
    w = NB - 1
    for s in range((n + w - 1) // w):
        k0 = lk0 + lkb
        if k0 >= n:
            break
        lk0, lkb = panel(M, ipiv, n, k0, ptol, st)
        if lkb < NB and lk0 + lkb < n:
            st['short_panels'] = st.get('short_panels', 0) + 1
        update(M, n, lk0, lkb)
    return backsolve(M, ipiv, n), st


