"""Brute-force dense evaluation of one discrete velocity's upwind system.

For a fixed velocity xi and a frozen source nu * f~S, the first-order upwind
finite-volume discretisation of eq. "iter_outer" (written out for one octant
in eq. "sweeping_example") is a linear system over all cells:

    (nu_c + sum_d a_d) f_c - sum_{d: upwind neighbour fluid} a_d f_up(c,d)
        = nu_c f~S_c + sum_{d: upwind side is a boundary} a_d f_boundary

with a_d = |xi_d| / dx_d(c), dx_d(c) the size of cell c along d (uniform or
a stretched mesh).  Here it is assembled as a dense matrix and solved
with LU (numpy), i.e. without any notion of sweep order, so it checks the
oracle's sweep (traversal order, upwind selection, boundary bookkeeping).

order=2: the flux through each face is the upwind cell's value extrapolated
linearly from that cell and its own upwind neighbour, i.e. the straight
line through the two cell centres evaluated at the face,
f_u + theta_u (f_u - f_uu) with theta_u = h_u / (h_u + h_uu) along d (1/2 on
a uniform mesh; just f_u when the upwind cell's upwind side is a boundary),
and a boundary's inflow value where the face is a boundary; the cell's
balance per axis is a_d (F_out(c) - F_in(c)).  A symmetry plane is an
interior face whose far side is the mirror image (of the same size):
spec_mirror then holds two planes (the mirror's f and its extrapolated face
value).
"""
from __future__ import annotations

import numpy as np

from paper_1810_00348_amd.cases import FREE, SPECULAR, WALL


def dense_velocity_solve(case, alpha, feq, nu, rho_w, ghat_of_kind, spec_mirror=None, order=1):
    nx, ny, nz = case.n
    N = nx * ny * nz
    mx, my, mz = case.m
    a3 = alpha % mx
    b3 = (alpha // mx) % my
    c3 = alpha // (mx * my)
    axes = []
    for d in range(3):
        M, V = case.m[d], case.vmax[d]
        axes.append(np.linspace(-V, V, M))
    xi = np.array([axes[0][a3], axes[1][b3], axes[2][c3]])
    sp = getattr(case, "spacing", None)
    h = [np.full(n, case.L[d] / n) for d, n in enumerate((nx, ny, nz))]
    if sp is not None:
        h = [h[d] if sp[d] is None else np.asarray(sp[d], dtype=np.float64) for d in range(3)]
    solid = case.solid_flat() if case.solid is not None else np.zeros(N, np.uint8)
    ext = [nx, ny, nz]

    def upwind(pos, d, c):
        """What lies on the upwind side of cell pos along d:
        ("cell", index, pos), ("spec", i + nx j) or ("bnd", inflow value)."""
        step = -1 if xi[d] >= 0 else +1
        side = 2 * d + (0 if xi[d] >= 0 else 1)
        p = list(pos)
        p[d] += step
        if 0 <= p[d] < ext[d]:
            nb = p[0] + nx * (p[1] + ny * p[2])
            if not solid[nb]:
                return ("cell", nb, p)
            return ("bnd", rho_w[side, c] * ghat_of_kind(6)[alpha])
        kind = case.faces[side].code
        if kind == WALL:
            return ("bnd", rho_w[side, c] * ghat_of_kind(side)[alpha])
        if kind == FREE:
            return ("bnd", case.faces[side].rho * ghat_of_kind(side)[alpha])
        if kind == SPECULAR:
            return ("spec", pos[0] + nx * pos[1])
        raise ValueError(kind)

    A = np.zeros((N, N))
    b = np.zeros(N)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                if solid[c]:
                    A[c, c] = 1.0
                    continue
                A[c, c] = nu[c]
                b[c] = nu[c] * feq[c]
                pos = [i, j, k]
                for d in range(3):
                    ad = abs(xi[d]) / h[d][pos[d]]
                    if ad == 0:
                        continue
                    up = upwind(pos, d, c)
                    if order == 1:
                        A[c, c] += ad
                        if up[0] == "cell":
                            A[c, up[1]] -= ad
                        elif up[0] == "spec":
                            b[c] += ad * spec_mirror[up[1]]
                        else:
                            b[c] += ad * up[1]
                        continue
                    if up[0] == "bnd":
                        # first-order face: a (f_c - f_b)
                        A[c, c] += ad
                        b[c] += ad * up[1]
                        continue
                    # interior face: a ((1 + t_c) f_c - t_c f_u - F_out(u)),
                    # t = own size / (own size + upwind neighbour's size)
                    hc = h[d][pos[d]]
                    if up[0] == "spec":
                        tc = hc / (hc + hc)
                        A[c, c] += (1.0 + tc) * ad
                        nxy = nx * ny
                        b[c] += ad * (tc * spec_mirror[up[1]] + spec_mirror[nxy + up[1]])
                        continue
                    u = up[1]
                    hu = h[d][up[2][d]]
                    tc = hc / (hc + hu)
                    A[c, c] += (1.0 + tc) * ad
                    A[c, u] -= tc * ad
                    uu = upwind(up[2], d, u)
                    if uu[0] == "bnd":            # F_out(u) = f_u
                        A[c, u] -= ad
                    elif uu[0] == "cell":         # F_out(u) = (1 + t_u) f_u - t_u f_uu
                        tu = hu / (hu + h[d][uu[2][d]])
                        A[c, u] -= (1.0 + tu) * ad
                        A[c, uu[1]] += tu * ad
                    else:                         # beyond u: the mirror image, t_u = 1/2
                        tu = hu / (hu + hu)
                        A[c, u] -= (1.0 + tu) * ad
                        b[c] -= tu * ad * spec_mirror[uu[1]]
    return np.linalg.solve(A, b)
