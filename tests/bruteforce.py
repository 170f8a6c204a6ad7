"""Independent dense NumPy implementation of one SI / GSIS iteration.

Used only to pin the oracle on tiny grids. It is written from the paper in a
different shape from the oracle: an explicit face list, least squares by
``numpy.linalg.lstsq`` on each cell's displacement matrix, face fluxes
accumulated into both cells, and the increment system of every ordinate
assembled as a dense matrix and solved without any cell ordering.
"""
import math

import numpy as np


def _faces(nx, ny, dx, dy):
    """Interior faces (c, nb, nx_, ny_, area) with normal from c to nb, and
    boundary faces (c, nx_, ny_, area, side_index)."""
    interior, boundary = [], []
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            if i + 1 < nx:
                interior.append((c, c + 1, 1.0, 0.0, dy))
            if j + 1 < ny:
                interior.append((c, c + nx, 0.0, 1.0, dx))
            if i == 0:
                boundary.append((c, -1.0, 0.0, dy, j))
            if i == nx - 1:
                boundary.append((c, 1.0, 0.0, dy, ny + j))
            if j == 0:
                boundary.append((c, 0.0, -1.0, dx, 2 * ny + i))
            if j == ny - 1:
                boundary.append((c, 0.0, 1.0, dx, 2 * ny + nx + i))
    return interior, boundary


def _centres(nx, ny, dx, dy):
    X = np.array([(i + 0.5) * dx for j in range(ny) for i in range(nx)])
    Y = np.array([(j + 0.5) * dy for j in range(ny) for i in range(nx)])
    return X, Y


def gradient(p, U, alsm=True):
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    st = p["sigma_a"] + p["sigma_s"]
    X, Y = _centres(nx, ny, dx, dy)
    interior, _ = _faces(nx, ny, dx, dy)
    nbrs = [[] for _ in range(nx * ny)]
    for c, nb, _, _, _ in interior:
        nbrs[c].append(nb)
        nbrs[nb].append(c)
    G = np.zeros((nx * ny, 2))
    for c in range(nx * ny):
        rows, rhs = [], []
        for nb in nbrs[c]:
            xf = 0.5 * (X[c] + X[nb]), 0.5 * (Y[c] + Y[nb])
            if alsm:
                s = st[nb] / st[c]
                xs = xf[0] + s * (X[nb] - xf[0]), xf[1] + s * (Y[nb] - xf[1])
            else:
                xs = X[nb], Y[nb]
            rows.append([xs[0] - X[c], xs[1] - Y[c]])
            rhs.append(U[nb] - U[c])
        if rows:
            A = np.array(rows)
            # columns that are identically zero (no neighbour in that axis)
            keep = np.abs(A).sum(0) > 0
            g = np.zeros(2)
            g[keep] = np.linalg.lstsq(A[:, keep], np.array(rhs), rcond=None)[0]
            G[c] = g
    return G


def limiter(p, U, G):
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    interior, _ = _faces(nx, ny, dx, dy)
    umax, umin = U.copy(), U.copy()
    for c, nb, _, _, _ in interior:
        umax[c] = max(umax[c], U[nb]); umin[c] = min(umin[c], U[nb])
        umax[nb] = max(umax[nb], U[c]); umin[nb] = min(umin[nb], U[c])
    psi = np.ones(nx * ny)
    offs = [(0.5 * dx, 0), (-0.5 * dx, 0), (0, 0.5 * dy), (0, -0.5 * dy)]
    for c in range(nx * ny):
        for ox, oy in offs:
            d = G[c, 0] * ox + G[c, 1] * oy
            if d > 0:
                psi[c] = min(psi[c], min(1.0, (umax[c] - U[c]) / d))
            elif d < 0:
                psi[c] = min(psi[c], min(1.0, (umin[c] - U[c]) / d))
    return psi


def _recon(p, U, order, lim, alsm):
    if order < 2:
        return np.zeros((len(U), 2)), np.zeros(len(U))
    G = gradient(p, U, alsm)
    psi = limiter(p, U, G) if lim else np.ones(len(U))
    return G, psi


def face_values(p, U, k, order, lim, alsm, bnd):
    """Upwinded face values of ordinate k on interior and boundary faces."""
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    X, Y = _centres(nx, ny, dx, dy)
    interior, boundary = _faces(nx, ny, dx, dy)
    G, psi = _recon(p, U, order, lim, alsm)
    mu, eta = p["mu"][k], p["eta"][k]
    fi = []
    for c, nb, nxx, nyy, A in interior:
        xf, yf = 0.5 * (X[c] + X[nb]), 0.5 * (Y[c] + Y[nb])
        up = c if mu * nxx + eta * nyy >= 0 else nb
        fi.append(U[up] + psi[up] * (G[up, 0] * (xf - X[up]) + G[up, 1] * (yf - Y[up])))
    fb = []
    for c, nxx, nyy, A, b in boundary:
        if mu * nxx + eta * nyy >= 0:
            xf, yf = X[c] + 0.5 * dx * nxx, Y[c] + 0.5 * dy * nyy
            fb.append(U[c] + psi[c] * (G[c, 0] * (xf - X[c]) + G[c, 1] * (yf - Y[c])))
        else:
            fb.append(0.0 if bnd is None else bnd[b, k])
    return np.array(fi), np.array(fb)


def residual(p, I, order=2, lim=True, alsm=True):
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    N, K = nx * ny, len(p["mu"])
    V = dx * dy
    st = p["sigma_a"] + p["sigma_s"]
    interior, boundary = _faces(nx, ny, dx, dy)
    phi = I @ p["w"]
    r = np.zeros((N, K))
    for k in range(K):
        fi, fb = face_values(p, I[:, k], k, order, lim, alsm, p.get("bnd_in"))
        div = np.zeros(N)
        for (c, nb, nxx, nyy, A), v in zip(interior, fi):
            on = p["mu"][k] * nxx + p["eta"][k] * nyy
            div[c] += on * A * v / V
            div[nb] -= on * A * v / V
        for (c, nxx, nyy, A, b), v in zip(boundary, fb):
            div[c] += (p["mu"][k] * nxx + p["eta"][k] * nyy) * A * v / V
        r[:, k] = (p["sigma_s"] * phi + p["q"]) / (4 * math.pi) - st * I[:, k] - div
    return r


def increment(p, r):
    """Dense solve of the first-order-upwind increment system per ordinate."""
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    N, K = nx * ny, len(p["mu"])
    V = dx * dy
    st = p["sigma_a"] + p["sigma_s"]
    interior, boundary = _faces(nx, ny, dx, dy)
    dI = np.zeros((N, K))
    for k in range(K):
        H = np.diag(st.copy())
        for c, nb, nxx, nyy, A in interior:
            on = p["mu"][k] * nxx + p["eta"][k] * nyy
            # flux across the face carries dI of the upwind cell
            up = c if on >= 0 else nb
            H[c, up] += on * A / V
            H[nb, up] -= on * A / V
        for c, nxx, nyy, A, b in boundary:
            on = p["mu"][k] * nxx + p["eta"][k] * nyy
            if on > 0:
                H[c, c] += on * A / V
        dI[:, k] = np.linalg.solve(H, r[:, k])
    return dI


def iterate(p, I, method=1, order=2, lim=True, alsm=True, hot_face=0, synth_form=0,
            synth_sub=1):
    nx, ny, dx, dy = p["nx"], p["ny"], p["dx"], p["dy"]
    N, K = nx * ny, len(p["mu"])
    V = dx * dy
    st = p["sigma_a"] + p["sigma_s"]
    mu, eta, w = p["mu"], p["eta"], p["w"]
    Ih = I + increment(p, residual(p, I, order, lim, alsm))
    ph = Ih @ w
    if method == 0:
        return Ih, ph
    Fx, Fy = Ih @ (w * mu), Ih @ (w * eta)
    interior, boundary = _faces(nx, ny, dx, dy)
    # transport face fluxes F_T . n from I^{m+1/2}
    FTi, FTb = np.zeros(len(interior)), np.zeros(len(boundary))
    for k in range(K):
        fi, fb = face_values(p, Ih[:, k], k, order, lim, alsm, p.get("bnd_in"))
        for t, (c, nb, nxx, nyy, A) in enumerate(interior):
            FTi[t] += w[k] * (mu[k] * nxx + eta[k] * nyy) * fi[t]
        for t, (c, nxx, nyy, A, b) in enumerate(boundary):
            FTb[t] += w[k] * (mu[k] * nxx + eta[k] * nyy) * fb[t]
    G = gradient(p, ph, alsm)
    hot = np.stack([Fx, Fy], 1) + G / (3 * st)[:, None]
    D = np.diag(V * p["sigma_a"].astype(float))
    b = V * p["q"].astype(float)
    for t, (c, nb, nxx, nyy, A) in enumerate(interior):
        gam = 2.0 / (3.0 * (st[c] * (dx if nxx else dy) + st[nb] * (dx if nxx else dy)))
        D[c, c] += A * gam; D[nb, nb] += A * gam
        D[c, nb] -= A * gam; D[nb, c] -= A * gam
        if hot_face == 0:
            h = 0.5 * ((hot[c, 0] + hot[nb, 0]) * nxx + (hot[c, 1] + hot[nb, 1]) * nyy)
        else:
            h = FTi[t] - gam * (ph[c] - ph[nb])
        b[c] -= A * h
        b[nb] += A * h
    for t, (c, nxx, nyy, A, bb) in enumerate(boundary):
        kap = 2.0 / (3.0 * st[c] * (dx if nxx else dy)) + 0.25
        D[c, c] += A * kap
        b[c] -= A * (FTb[t] - kap * ph[c])
    if synth_form == 0:
        phn = np.linalg.solve(D, b)
    else:
        # the balance with the face average of the cells' diffusive fluxes
        # -(grad x / (3 sigma_t)) . n (Eq. Fij_d), assembled densely from the
        # least-squares gradient of every unit vector, then synth_sub
        # defect-correction steps D dx = b - Aw x from x = phi^{m+1/2}
        Gx, Gy = np.zeros((N, N)), np.zeros((N, N))
        for k in range(N):
            e = np.zeros(N)
            e[k] = 1.0
            g = gradient(p, e, alsm)
            Gx[:, k] = g[:, 0] / (3 * st)
            Gy[:, k] = g[:, 1] / (3 * st)
        Aw = np.diag(V * p["sigma_a"].astype(float))
        for c, nb, nxx, nyy, A in interior:
            row = -0.5 * ((Gx[c] + Gx[nb]) * nxx + (Gy[c] + Gy[nb]) * nyy)
            Aw[c] += A * row
            Aw[nb] -= A * row
        for c, nxx, nyy, A, bb in boundary:
            Aw[c, c] += A * (2.0 / (3.0 * st[c] * (dx if nxx else dy)) + 0.25)
        phn = ph.copy()
        for _ in range(synth_sub):
            phn = phn + np.linalg.solve(D, b - Aw @ phn)
    return Ih + ((phn - ph) / (4 * math.pi))[:, None], phn
