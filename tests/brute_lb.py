"""Literal brute-force D3Q19 lattice Boltzmann for tiny lattices (test-only).

An independent second implementation used to pin the oracle: it stores one
Python list of 19 populations per node in a dict, collides node by node and
then *pushes* every post-collision population to x + c_i (the oracle pulls).
MRT uses the closed-form equilibrium and forcing moments
(rho u^2, rho(3u_x^2 - u^2), ..., 2 u.g, ...) and the printed basis norms
instead of projecting populations numerically as the oracle does, and the
face interpolation uses exact rational arithmetic.  Slow by design: only for
lattices of a few hundred nodes.
"""
from __future__ import annotations

import math
from fractions import Fraction

C = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
     (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
W = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
# basis norms sum_i w_i e_k(c_i)^2 of the weighted-orthogonal MRT basis
NORM = [1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9,
        2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9]


def poly(c):
    x, y, z = c
    s = x * x + y * y + z * z
    return [1, x, y, z, s - 1, 3 * x * x - s, y * y - z * z, x * y, y * z, x * z,
            (3 * s - 5) * x, (3 * s - 5) * y, (3 * s - 5) * z, (y * y - z * z) * x,
            (z * z - x * x) * y, (x * x - y * y) * z, 3 * s * s - 6 * s + 1,
            (2 * s - 3) * (3 * x * x - s), (2 * s - 3) * (y * y - z * z)]


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def feq(rho, u):
    uu = dot(u, u)
    return [W[i] * rho * (1 + 3 * dot(C[i], u) + 4.5 * dot(C[i], u) ** 2 - 1.5 * uu)
            for i in range(19)]


def collide_bgk(f, g, tau):
    rho = sum(f)
    j = [sum(C[i][a] * f[i] for i in range(19)) for a in range(3)]
    u = [(j[a] + g[a] / 2) / rho for a in range(3)]
    eq = feq(rho, u)
    out = []
    for i in range(19):
        src = W[i] * (3 * dot([C[i][a] - u[a] for a in range(3)], g) + 9 * dot(C[i], u) * dot(C[i], g))
        out.append(f[i] - (f[i] - eq[i]) / tau + (1 - 1 / (2 * tau)) * src)
    return out


def collide_mrt(f, g, tau, tau_bulk, ghost):
    P = [poly(c) for c in C]
    m = [sum(P[i][k] * f[i] for i in range(19)) for k in range(19)]
    rho = m[0]
    u = [(m[1 + a] + g[a] / 2) / rho for a in range(3)]
    ux, uy, uz = u
    gx, gy, gz = g
    ug = dot(u, g)
    meq = [rho, rho * ux, rho * uy, rho * uz, rho * dot(u, u), rho * (3 * ux * ux - dot(u, u)),
           rho * (uy * uy - uz * uz), rho * ux * uy, rho * uy * uz, rho * ux * uz] + [0.0] * 9
    mf = [0.0, gx, gy, gz, 2 * ug, 2 * (3 * ux * gx - ug), 2 * (uy * gy - uz * gz),
          ux * gy + uy * gx, uy * gz + uz * gy, ux * gz + uz * gx] + [0.0] * 9
    post = list(m)
    post[1:4] = [m[1 + a] + g[a] for a in range(3)]
    for k in range(4, 19):
        s = 1 / tau_bulk if k == 4 else (1 / tau if k < 10 else ghost)
        gam = 1 - s
        post[k] = meq[k] + gam * (m[k] - meq[k]) + (1 + gam) / 2 * mf[k]
    return [W[i] * sum(P[i][k] * post[k] / NORM[k] for k in range(19)) for i in range(19)]


class BruteBox:
    def __init__(self, dims, periodic=(False, False, False), collision="bgk", tau=0.8,
                 tau_bulk=None, ghost=1.0, rho0=1.0):
        self.n = tuple(dims)
        self.per = tuple(periodic)
        self.coll = collision
        self.tau = tau
        self.tau_bulk = tau if tau_bulk is None else tau_bulk
        self.ghost = ghost
        self.rho0 = rho0
        self.nodes = [(x, y, z) for z in range(dims[2]) for y in range(dims[1]) for x in range(dims[0])]
        self.f = {}
        self.chains = []
        self.bc = None
        self.step_no = 0
        for q in self.nodes:
            if self.interior(q):
                self.f[q] = feq(rho0, (0.0, 0.0, 0.0))

    def interior(self, q):
        return all(self.per[a] or 1 <= q[a] <= self.n[a] - 2 for a in range(3))

    def set_velocity(self, ufun):
        for q in self.nodes:
            if self.interior(q):
                self.f[q] = feq(self.rho0, ufun(q))

    # boundary ----------------------------------------------------------
    def face_of(self, q):
        for f in range(6):
            a = f // 2
            if self.per[a]:
                continue
            if q[a] == (0 if f % 2 == 0 else self.n[a] - 1):
                return f
        return None

    def ub(self, q, n):
        mode, t0, dt, data, res = self.bc
        k, rem = divmod(n - t0, dt)
        th = Fraction(rem, dt)
        if mode == "affine":
            A = [(1 - th) * data[k][e] + (th * data[k + 1][e] if rem else 0) for e in range(9)]
            r = [q[a] - (self.n[a] - 1) / 2 for a in range(3)]
            return [float(A[3 * a] * r[0] + A[3 * a + 1] * r[1] + A[3 * a + 2] * r[2]) for a in range(3)]
        f = self.face_of(q)
        a = f // 2
        au, av = [b for b in range(3) if b != a]

        def bil(kk):
            su = Fraction(q[au] * (res - 1), self.n[au] - 1)
            sv = Fraction(q[av] * (res - 1), self.n[av] - 1)
            p, qq = math.floor(su), math.floor(sv)
            al, be = su - p, sv - qq
            out = []
            for c in range(3):
                val = 0.0
                for dp_, wu in ((0, 1 - al), (1, al)):
                    for dq, wv in ((0, 1 - be), (1, be)):
                        w = wu * wv
                        if w == 0:
                            continue
                        val += float(w) * data[kk][f][qq + dq][p + dp_][c]
                out.append(val)
            return out
        v0 = bil(k)
        if rem == 0:
            return v0
        v1 = bil(k + 1)
        return [(1 - float(th)) * v0[c] + float(th) * v1[c] for c in range(3)]

    # chain ---------------------------------------------------------------
    def add_chain(self, pos, vel, substeps, fix_com, zeta, mass, k, r0, anchor):
        self.chains.append(dict(pos=[list(p) for p in pos], vel=[list(v) for v in vel], S=substeps,
                                fix=fix_com, zeta=zeta, m=mass, k=k, r0=r0, anchor=list(anchor)))

    def corners(self, r):
        base = [math.floor(r[a]) for a in range(3)]
        d = [r[a] - base[a] for a in range(3)]
        for a in range(3):
            if not self.per[a] and not (1 <= base[a] and base[a] + 1 <= self.n[a] - 2):
                raise RuntimeError("bead out")
        out = []
        for ox in (0, 1):
            for oy in (0, 1):
                for oz in (0, 1):
                    o = (ox, oy, oz)
                    w = 1.0
                    for a in range(3):
                        w *= d[a] if o[a] else 1 - d[a]
                    q = tuple((base[a] + o[a]) % self.n[a] for a in range(3))
                    out.append((q, w))
        return out

    def chain_step(self):
        g = {}
        for ch in self.chains:
            nb = len(ch["pos"])
            stencils = [self.corners(r) for r in ch["pos"]]
            ub = []
            for st in stencils:
                acc = [0.0, 0.0, 0.0]
                for q, w in st:
                    f = self.f[q]
                    rho = sum(f)
                    for a in range(3):
                        acc[a] += w * sum(C[i][a] * f[i] for i in range(19)) / rho
                ub.append(acc)
            h = 1.0 / ch["S"]
            dec = math.exp(-ch["zeta"] * h / ch["m"])
            dp = [[0.0] * 3 for _ in range(nb)]
            R, V = ch["pos"], ch["vel"]
            for _ in range(ch["S"]):
                F = [[0.0] * 3 for _ in range(nb)]
                for j in range(nb - 1):
                    r = [R[j + 1][a] - R[j][a] for a in range(3)]
                    r2 = dot(r, r)
                    if r2 >= ch["r0"] ** 2:
                        raise RuntimeError("fene")
                    fac = ch["k"] / (1 - r2 / ch["r0"] ** 2)
                    for a in range(3):
                        F[j][a] += fac * r[a]
                        F[j + 1][a] -= fac * r[a]
                for j in range(nb):
                    for a in range(3):
                        term = ub[j][a] + F[j][a] / ch["zeta"]
                        vn = term + (V[j][a] - term) * dec
                        dp[j][a] += ch["m"] * (vn - V[j][a]) - F[j][a] * h
                        V[j][a] = vn
                        R[j][a] += h * vn
                if ch["fix"]:
                    for a in range(3):
                        vb = sum(V[j][a] for j in range(nb)) / nb
                        rb = sum(R[j][a] for j in range(nb)) / nb
                        for j in range(nb):
                            V[j][a] -= vb
                            R[j][a] = R[j][a] - rb + ch["anchor"][a]
            for j, st in enumerate(stencils):
                for q, w in st:
                    acc = g.setdefault(q, [0.0, 0.0, 0.0])
                    for a in range(3):
                        acc[a] -= w * dp[j][a]
        return g

    # step ----------------------------------------------------------------
    def step(self):
        n = self.step_no
        g = self.chain_step()
        post = {}
        for q in self.nodes:
            if self.interior(q):
                gq = g.get(q, [0.0, 0.0, 0.0])
                if self.coll == "bgk":
                    post[q] = collide_bgk(self.f[q], gq, self.tau)
                else:
                    post[q] = collide_mrt(self.f[q], gq, self.tau, self.tau_bulk, self.ghost)
            else:
                post[q] = feq(self.rho0, self.ub(q, n))
        new = {q: [None] * 19 for q in self.f}
        for q, fp in post.items():
            for i in range(19):
                t = [q[a] + C[i][a] for a in range(3)]
                if not all(self.per[a] or 1 <= t[a] <= self.n[a] - 2 for a in range(3)):
                    continue
                t = tuple(t[a] % self.n[a] for a in range(3))
                new[t][i] = fp[i]
        self.f = new
        self.step_no += 1
