"""Dense-matrix form of the paper's graph (test infrastructure only).

Prop. 1 of the paper numbers the field nodes of an Nx x Nz grid and lists
each node's neighbourhood; Prop. 2 states that one leapfrog step is two
message-passing layers h_l <- sum_{n in N(l)} w_{l,n} h_n, first over the H
nodes, then over the E nodes, with fixed weights read off Eq. 7-9.  This
module writes that literally as two dense matrices W_H and W_E acting on the
whole node vector, so that one step is h <- W_E (W_H h) + g e_src.  It is an
independent formulation of the stencil in ``fdtd_oracle.c`` (expanded edge
weights on the old state instead of sequential updates) and pins it on tiny
grids; it also gives the spectrum of the step (stability) and the exact
transpose (adjoint).

Reading of Prop. 1 used here (TMz relabelling of the paper's TE form, paper-z
-> y): node indices t = 2i+1+Nx(3j+1) for Ez, u = i+3jNx for Hx,
q = 2i+Nx(3j+1) for Hy (the paper's Hz); the E neighbourhood is the printed
one {t_ij, u_ij, u_i,j-1, q_ij, q_i-1,j}; the H neighbourhoods use forward
offsets {u_ij, t_ij, t_i,j+1} and {q_ij, t_ij, t_i+1,j}, which is what a
consistent half-cell staggering with E owned at the lower cell corner
requires.  The absorbing layer is a CPML: its auxiliary psi values are
appended as extra nodes (four per cell in 2D, twelve in 3D) with their own
self loops and edges.  Material and profile arrays are taken from an oracle
instance.
"""
from __future__ import annotations

import numpy as np


def _prof(p, n):
    return dict(bE=p[0:n], cE=p[n:2 * n], kE=p[2 * n:3 * n],
                bH=p[3 * n:4 * n], cH=p[4 * n:5 * n], kH=p[5 * n:6 * n])


class Graph2D:
    """Dense W_H, W_E for a 2D TMz oracle instance (Oracle2D)."""

    def __init__(self, o):
        nx, ny = o.shape
        self.nx, self.ny = nx, ny
        self.o = o
        N = nx * ny
        self.nmain = 3 * N
        self.nnodes = 7 * N
        self.t = lambda i, j: 2 * i + 1 + nx * (3 * j + 1)
        self.u = lambda i, j: i + 3 * j * nx
        self.q = lambda i, j: 2 * i + nx * (3 * j + 1)
        base = {"psi_hx": 3 * N, "psi_hy": 4 * N, "psi_ezx": 5 * N, "psi_ezy": 6 * N}
        self.psi = lambda name, i, j: base[name] + i * ny + j
        self._check_bijection()
        self.WH, self.WE = self._build()

    def _check_bijection(self):
        seen = np.zeros(self.nmain, np.int32)
        for i in range(self.nx):
            for j in range(self.ny):
                for f in (self.t, self.u, self.q):
                    seen[f(i, j)] += 1
        assert np.all(seen == 1), "Prop. 1 index maps are not a bijection"

    def _build(self):
        o = self.o
        nx, ny = self.nx, self.ny
        dx, dy = o.dx
        px, py = _prof(o.prof_x, nx), _prof(o.prof_y, ny)
        ca = o.ca.reshape(nx, ny)
        cb = o.cb.reshape(nx, ny)
        db = o.db.reshape(nx, ny)
        M = self.nnodes
        WH = np.eye(M)
        WE = np.eye(M)
        t, u, q, psi = self.t, self.u, self.q, self.psi
        for i in range(nx):
            for j in range(ny):
                # Hx(i,j) <- {Hx(i,j), Ez(i,j), Ez(i,j+1)} plus its psi node
                r = u(i, j)
                w = db[i, j] * (py["kH"][j] + py["cH"][j]) / dy
                WH[r, r] = 1.0
                WH[r, psi("psi_hx", i, j)] = -db[i, j] * py["bH"][j]
                WH[r, t(i, j)] += w
                if j + 1 < ny:
                    WH[r, t(i, j + 1)] += -w
                rp = psi("psi_hx", i, j)
                WH[rp, rp] = py["bH"][j]
                WH[rp, t(i, j)] += -py["cH"][j] / dy
                if j + 1 < ny:
                    WH[rp, t(i, j + 1)] += py["cH"][j] / dy
                # Hy(i,j) <- {Hy(i,j), Ez(i,j), Ez(i+1,j)} plus its psi node
                r = q(i, j)
                w = db[i, j] * (px["kH"][i] + px["cH"][i]) / dx
                WH[r, r] = 1.0
                WH[r, psi("psi_hy", i, j)] = db[i, j] * px["bH"][i]
                WH[r, t(i, j)] += -w
                if i + 1 < nx:
                    WH[r, t(i + 1, j)] += w
                rp = psi("psi_hy", i, j)
                WH[rp, rp] = px["bH"][i]
                WH[rp, t(i, j)] += -px["cH"][i] / dx
                if i + 1 < nx:
                    WH[rp, t(i + 1, j)] += px["cH"][i] / dx
        for i in range(1, nx):
            for j in range(1, ny):
                # Ez(i,j) <- {Ez(i,j), Hx(i,j), Hx(i,j-1), Hy(i,j), Hy(i-1,j)} plus psi nodes
                r = t(i, j)
                wx = cb[i, j] * (px["kE"][i] + px["cE"][i]) / dx
                wy = cb[i, j] * (py["kE"][j] + py["cE"][j]) / dy
                WE[r, r] = ca[i, j]
                WE[r, q(i, j)] += wx
                WE[r, q(i - 1, j)] += -wx
                WE[r, u(i, j)] += -wy
                WE[r, u(i, j - 1)] += wy
                WE[r, psi("psi_ezx", i, j)] = cb[i, j] * px["bE"][i]
                WE[r, psi("psi_ezy", i, j)] = -cb[i, j] * py["bE"][j]
                rp = psi("psi_ezx", i, j)
                WE[rp, rp] = px["bE"][i]
                WE[rp, q(i, j)] += px["cE"][i] / dx
                WE[rp, q(i - 1, j)] += -px["cE"][i] / dx
                rp = psi("psi_ezy", i, j)
                WE[rp, rp] = py["bE"][j]
                WE[rp, u(i, j)] += py["cE"][j] / dy
                WE[rp, u(i, j - 1)] += -py["cE"][j] / dy
        return WH, WE

    def pack(self, st):
        nx, ny = self.nx, self.ny
        h = np.zeros(self.nnodes)
        for i in range(nx):
            for j in range(ny):
                h[self.t(i, j)] = st["ez"][i, j]
                h[self.u(i, j)] = st["hx"][i, j]
                h[self.q(i, j)] = st["hy"][i, j]
                for n in ("psi_hx", "psi_hy", "psi_ezx", "psi_ezy"):
                    h[self.psi(n, i, j)] = st[n][i, j]
        return h

    def unpack(self, h):
        nx, ny = self.nx, self.ny
        st = {n: np.zeros((nx, ny)) for n in ("ez", "hx", "hy", "psi_hx", "psi_hy",
                                              "psi_ezx", "psi_ezy")}
        for i in range(nx):
            for j in range(ny):
                st["ez"][i, j] = h[self.t(i, j)]
                st["hx"][i, j] = h[self.u(i, j)]
                st["hy"][i, j] = h[self.q(i, j)]
                for n in ("psi_hx", "psi_hy", "psi_ezx", "psi_ezy"):
                    st[n][i, j] = h[self.psi(n, i, j)]
        return st

    def step_matrix(self):
        return self.WE @ self.WH


F3 = ("ex", "ey", "ez", "hx", "hy", "hz")
PSI3 = ("psi_hxy", "psi_hxz", "psi_hyz", "psi_hyx", "psi_hzx", "psi_hzy",
        "psi_exy", "psi_exz", "psi_eyz", "psi_eyx", "psi_ezx", "psi_ezy")


class Graph3D:
    """Dense W_H, W_E for a 3D oracle instance (Oracle3D).  The paper gives
    no 3D numbering; nodes are numbered component-major (the six field
    components, then the twelve psi arrays), cell-major inside a block."""

    def __init__(self, o):
        nx, ny, nz = o.shape
        self.shape = (nx, ny, nz)
        self.o = o
        N = nx * ny * nz
        self.N = N
        self.names = F3 + PSI3
        self.nnodes = len(self.names) * N
        self.WH, self.WE = self._build()

    def idx(self, name, i, j, k):
        nx, ny, nz = self.shape
        return self.names.index(name) * self.N + (i * ny + j) * nz + k

    def _build(self):
        o = self.o
        nx, ny, nz = self.shape
        dx, dy, dz = o.dx
        P = {"x": _prof(o.prof_x, nx), "y": _prof(o.prof_y, ny), "z": _prof(o.prof_z, nz)}
        D = {"x": dx, "y": dy, "z": dz}
        ca = o.ca.reshape(self.shape)
        cb = o.cb.reshape(self.shape)
        db = o.db.reshape(self.shape)
        M = self.nnodes
        WH = np.eye(M)
        WE = np.eye(M)
        off = {"x": (1, 0, 0), "y": (0, 1, 0), "z": (0, 0, 1)}
        pos = {"x": 0, "y": 1, "z": 2}
        # H_f -= Db * (+ (D+_a E_p / kappa + psi_fa) - (D+_b E_r / kappa + psi_fb))
        hdef = {"hx": (("y", "ez", "psi_hxy"), ("z", "ey", "psi_hxz")),
                "hy": (("z", "ex", "psi_hyz"), ("x", "ez", "psi_hyx")),
                "hz": (("x", "ey", "psi_hzx"), ("y", "ex", "psi_hzy"))}
        # E_f = Ca E_f + Cb * (+ (D-_a H_p / kappa + psi_fa) - (D-_b H_r / kappa + psi_fb))
        edef = {"ex": (("y", "hz", "psi_exy"), ("z", "hy", "psi_exz")),
                "ey": (("z", "hx", "psi_eyz"), ("x", "hz", "psi_eyx")),
                "ez": (("x", "hy", "psi_ezx"), ("y", "hx", "psi_ezy"))}
        for i in range(nx):
            for j in range(ny):
                for k in range(nz):
                    c = (i, j, k)
                    for f, terms in hdef.items():
                        r = self.idx(f, *c)
                        for sgn, (ax, src, pn) in zip((1.0, -1.0), terms):
                            p = P[ax]
                            a = c[pos[ax]]
                            nb = tuple(c[m] + off[ax][m] for m in range(3))
                            inside = nb[pos[ax]] < self.shape[pos[ax]]
                            w = -sgn * db[c] * (p["kH"][a] + p["cH"][a]) / D[ax]
                            WH[r, self.idx(src, *c)] += -w
                            if inside:
                                WH[r, self.idx(src, *nb)] += w
                            rp = self.idx(pn, *c)
                            WH[r, rp] += -sgn * db[c] * p["bH"][a]
                            WH[rp, rp] = p["bH"][a]
                            WH[rp, self.idx(src, *c)] += -p["cH"][a] / D[ax]
                            if inside:
                                WH[rp, self.idx(src, *nb)] += p["cH"][a] / D[ax]
                    for f, terms in edef.items():
                        axes = [t[0] for t in terms]
                        if any(c[pos[ax]] < 1 for ax in axes):
                            continue  # tangential to a low PEC wall: not updated
                        r = self.idx(f, *c)
                        WE[r, r] = ca[c]
                        for sgn, (ax, src, pn) in zip((1.0, -1.0), terms):
                            p = P[ax]
                            a = c[pos[ax]]
                            nb = tuple(c[m] - off[ax][m] for m in range(3))
                            w = sgn * cb[c] * (p["kE"][a] + p["cE"][a]) / D[ax]
                            WE[r, self.idx(src, *c)] += w
                            WE[r, self.idx(src, *nb)] += -w
                            rp = self.idx(pn, *c)
                            WE[r, rp] += sgn * cb[c] * p["bE"][a]
                            WE[rp, rp] = p["bE"][a]
                            WE[rp, self.idx(src, *c)] += p["cE"][a] / D[ax]
                            WE[rp, self.idx(src, *nb)] += -p["cE"][a] / D[ax]
        return WH, WE

    def pack(self, st):
        return np.concatenate([st[n].ravel() for n in self.names])

    def unpack(self, h):
        return {n: h[m * self.N:(m + 1) * self.N].reshape(self.shape).copy()
                for m, n in enumerate(self.names)}

    def step_matrix(self):
        return self.WE @ self.WH


class Graph2DSplit:
    """Dense W_H, W_E of the paper's split-field PML graph (Sec. IV, the
    4 Nx Nz-node form of its Sec. III-C layer), for a 2D TMz problem.

    Nodes, in the TMz relabelling (Ey -> Ez split into Ezx and Ezy, Hz -> Hy,
    paper-z -> y): Hx u = i + 4 j Nx, Hy q = 3 i + Nx (4 j + 1), Ezx
    tx = q + 1, Ezy tz = q + 2.  Every cell carries all four.  H layer:
    Hx(i, j) gathers itself and both Ez parts at (i, j) and (i, j+1), Hy(i, j)
    itself and both parts at (i, j) and (i+1, j); E layer (cells off the PEC
    planes i = 0 and j = 0): Ezx(i, j) gathers itself and Hy at (i, j),
    (i-1, j); Ezy(i, j) itself and Hx at (i, j), (i, j-1) (the printed k
    offset of the Eyz neighbourhood read as the j offset its update needs).

    Weights, one per edge, written from the node positions: a node at
    position x along the axis of its loss term gets the layer conductivity
    s(x) = s_max rho(x)^m, rho the normalised depth into the layer (Ezx, Ezy
    at integer positions, Hx at y = j + 1/2, Hy at x = i + 1/2); the
    magnetic loss is s mu0 / eps0; with a = (cell loss + s) dt / (2 m),
    m = eps or mu of the cell, the self weight is (1 - a)/(1 + a) and the
    curl weight (dt/m)/(1 + a) divided by the step of the axis.  Nothing is
    taken from oracle/split.py but the problem's inputs."""

    def __init__(self, shape, dx, dt, eps_r=None, sigma=None, mu_r=None, npml=(0, 0, 0, 0), m=3.0,
                 sigma_max=0.0):
        nx, ny = shape
        self.nx, self.ny = nx, ny
        self.nnodes = 4 * nx * ny
        self.u = lambda i, j: i + 4 * j * nx
        self.q = lambda i, j: 3 * i + nx * (4 * j + 1)
        self.tx = lambda i, j: self.q(i, j) + 1
        self.tz = lambda i, j: self.q(i, j) + 2
        seen = np.zeros(self.nnodes, np.int32)
        for i in range(nx):
            for j in range(ny):
                for f in (self.u, self.q, self.tx, self.tz):
                    seen[f(i, j)] += 1
        assert np.all(seen == 1), "4-node index maps are not a bijection"
        eps0, mu0 = 8.8541878128e-12, 1.25663706212e-6
        eta0 = (mu0 / eps0) ** 0.5

        def s_layer(pos, n, lo, hi, delta):
            depth = 0.0
            if lo > 0 and pos < lo:
                depth = (lo - pos) / lo
            if hi > 0 and pos > n - hi:
                depth = max(depth, (pos - (n - hi)) / hi)
            smax = sigma_max if sigma_max > 0 else 0.8 * (m + 1.0) / (eta0 * delta)
            return smax * depth ** m

        def w(loss, mat):
            a = loss * dt / (2.0 * mat)
            return (1.0 - a) / (1.0 + a), (dt / mat) / (1.0 + a)

        def get(a, i, j, default):
            return default if a is None else float(np.asarray(a).reshape(shape)[i, j])

        M = self.nnodes
        WH, WE = np.eye(M), np.eye(M)
        for i in range(nx):
            for j in range(ny):
                mu = mu0 * get(mu_r, i, j, 1.0)
                eps = eps0 * get(eps_r, i, j, 1.0)
                sc = get(sigma, i, j, 0.0)
                # Hx(i, j + 1/2): -dEz/dy, magnetic loss of the y layer
                self_w, curl = w(s_layer(j + 0.5, ny, npml[2], npml[3], dx[1]) * mu0 / eps0, mu)
                r = self.u(i, j)
                WH[r, r] = self_w
                for part in (self.tx, self.tz):
                    WH[r, part(i, j)] += curl / dx[1]
                    if j + 1 < ny:
                        WH[r, part(i, j + 1)] -= curl / dx[1]
                # Hy(i + 1/2, j): +dEz/dx, magnetic loss of the x layer
                self_w, curl = w(s_layer(i + 0.5, nx, npml[0], npml[1], dx[0]) * mu0 / eps0, mu)
                r = self.q(i, j)
                WH[r, r] = self_w
                for part in (self.tx, self.tz):
                    WH[r, part(i, j)] -= curl / dx[0]
                    if i + 1 < nx:
                        WH[r, part(i + 1, j)] += curl / dx[0]
                if i == 0 or j == 0:
                    continue  # PEC planes: the E nodes keep their value
                # Ezx(i, j): +dHy/dx, the cell's loss plus the x layer's
                self_w, curl = w(sc + s_layer(float(i), nx, npml[0], npml[1], dx[0]), eps)
                r = self.tx(i, j)
                WE[r, r] = self_w
                WE[r, self.q(i, j)] += curl / dx[0]
                WE[r, self.q(i - 1, j)] -= curl / dx[0]
                # Ezy(i, j): -dHx/dy, the cell's loss plus the y layer's
                self_w, curl = w(sc + s_layer(float(j), ny, npml[2], npml[3], dx[1]), eps)
                r = self.tz(i, j)
                WE[r, r] = self_w
                WE[r, self.u(i, j)] -= curl / dx[1]
                WE[r, self.u(i, j - 1)] += curl / dx[1]
        self.WH, self.WE = WH, WE

    def ez(self, h):
        out = np.zeros((self.nx, self.ny))
        for i in range(self.nx):
            for j in range(self.ny):
                out[i, j] = h[self.tx(i, j)] + h[self.tz(i, j)]
        return out

    def field(self, h, name):
        f = {"hx": self.u, "hy": self.q, "ezx": self.tx, "ezy": self.tz}[name]
        out = np.zeros((self.nx, self.ny))
        for i in range(self.nx):
            for j in range(self.ny):
                out[i, j] = h[f(i, j)]
        return out
