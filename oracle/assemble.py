"""Per-mode Mueller-Nystrom matrices (Sections 2.1, 3 and 5).

Unknowns per node j (columns 4j..4j+3): J^1, J^2, M^1, M^2 -- the t and
e_theta components of J = n x H and M = n x E (eq. emcurrent) in mode m.
Equations per target node i (rows 4i..4i+3):

  rows 0,1  i w mu0 (n x H_inc)_{t,theta} = (i w/2)(mu0+mu1) J - (K^{k0}-K^{k1}) M
                                            - i w (mu0 N^{k0} - mu1 N^{k1}) J
  rows 2,3  i w eps0 (n x E_inc)_{t,theta} = (i w/2)(eps0+eps1) M + (K^{k0}-K^{k1}) J
                                             - i w (eps0 N^{k0} - eps1 N^{k1}) M

(eq. mullerrep; the magnetic equation is placed first so that the identity
terms sit on the diagonal).  The indirect system (eq. dualmullrep, Section
2.2) uses the same operators with other weights:

  rows 0,1  i w eps0 (n x H_inc) = -(i w/2)(eps0+eps1) J - i w (eps0 N^{k0} - eps1 N^{k1}) J
                                    - (eps0/mu0) (K^{k0}-K^{k1}) M
  rows 2,3  i w mu0 (n x E_inc)  = -(i w/2)(mu0+mu1) M - i w (mu0 N^{k0} - mu1 N^{k1}) M
                                    + (mu0/eps0) (K^{k0}-K^{k1}) J

(its N terms written with the printed i w (eps1 N^{k1} - eps0 N^{k0}) =
-i w (eps0 N^{k0} - eps1 N^{k1}), its K terms with K^{k1}-K^{k0} = -(K^{k0}-K^{k1})).  The tabulated kernels are g^{k0} and g^{k0} - g^{k1}
(with their derivatives), so mu0 N^{k0} - mu1 N^{k1} is formed as
(mu0 - mu1) N^{k0} + mu1 (N^{k0} - N^{k1}).  N and K act on a tangential
density a = (a^1, a^2)
through the coefficients of Lemma 1 (eqs. equc1-equc3),

  c^1 = int a^1 r r' g^2 - i int a^2 r g^3,   c^2 = i int a^1 r r' g^3 + int a^2 r g^2,
  c^3 = int a^1 r z' g^1,

with g^2_m = (g_{m+1} + g_{m-1})/2 and g^3_m = (g_{m-1} - g_{m+1})/2 (the
relation equrelation for g^2; for g^3 the sign and factor follow from green31
directly), and the mode-m expansions of Section 3:

  [N a]_t     = d_z c^1 - d_r c^3
  [N a]_theta = -[(z'/r)(c^2 + r d_r c^2 - i m c^1) + r' ((i m/r) c^3 - d_z c^2)]
  [K a]_t     = k^2 c^2 + (i m/r^2) c^1 + (i m/r) d_r c^1 - (m^2/r^2) c^2 + (i m/r) d_z c^3
  [K a]_theta = -[k^2 (z' c^3 + r' c^1) + z' d_z D + r' d_r D]
  d_z D = (1/r) d_z c^1 + d_rz c^1 + (i m/r) d_z c^2 + d_zz c^3
  d_r D = -c^1/r^2 + (1/r) d_r c^1 + d_rr c^1 - (i m/r^2) c^2 + (i m/r) d_r c^2 + d_rz c^3

(target quantities r = r_t, r' = r'_t, z' = z'_t).  The e_theta rows are the
negatives of the printed ones: n x V = V_theta t - (r' V_r + z' V_z) e_theta for
n = z' e_r - r' e_z, which the printed expansions do not follow.  In K^{k0}-K^{k1}
the k^2 c terms use each wavenumber's own kernels, written
(k0^2 - k1^2) c(g^{k0}) + k1^2 c(g^{k0} - g^{k1}); every other term uses the
difference g^{k0} - g^{k1} and the tabulated differences of derivatives.

Quadrature (eq. disequ, eq_nyslike2): far panels use w_j K(x_i, x_j); the
target's own panel and its neighbours use the support nodes.  Finally the L^2
weighting (Section 6, first remark): A_ij -> sqrt(w_i / w_j) A_ij, a similarity
transform applied to the stored matrix; the solver undoes it.
"""
from __future__ import annotations

import numpy as np

from .discretize import neighbours


def blocks(tab_m, m, rt, trt, tzt, rs, trs, tzs, k0, k1, omega, eps0, mu0, eps1, mu1, formulation="direct"):
    """4x4 kernel blocks for one mode: [4, 4, ...] over the broadcast pair shape.

    tab_m: dict with arrays for modes m-1, m, m+1 (indices 0..2) of the nine
    types, each [3, 9, ...]; rt.. target geometry, rs.. source geometry.
    """
    T = tab_m  # [3, 9, ...]
    G1 = T[1]
    G2 = 0.5 * (T[2] + T[0])
    G3 = 0.5 * (T[0] - T[2])
    im = 1j * m

    def cvals(typ_g):
        """c^1, c^2, c^3 for densities beta = t, theta from kernel type index."""
        g1, g2, g3 = G1[typ_g], G2[typ_g], G3[typ_g]
        c1 = (rs * trs * g2, -1j * rs * g3)
        c2 = (1j * rs * trs * g3, rs * g2)
        c3 = (rs * tzs * g1, 0.0 * g1)
        return c1, c2, c3

    # per-wavenumber families: (g, dr, dz) at type indices (0,1,2) and (3,4,5)
    def N_op(base):
        c1, c2, c3 = cvals(base + 0)
        dr1, dr2, dr3 = cvals(base + 1)
        dz1, dz2, dz3 = cvals(base + 2)
        out = np.zeros((2, 2) + np.broadcast(G1[0], rs).shape, dtype=complex)
        for b in range(2):
            out[0, b] = dz1[b] - dr3[b]
            out[1, b] = -((tzt / rt) * (c2[b] + rt * dr2[b] - im * c1[b])
                          + trt * ((im / rt) * c3[b] - dz2[b]))
        return out

    N0 = N_op(0)
    dN = N_op(3)  # N^{k0} - N^{k1}: N is linear in the kernel family
    # difference family (tabulated directly)
    D = G1[3:6], G2[3:6], G3[3:6]

    def cd(i):
        g1, g2, g3 = D[0][i], D[1][i], D[2][i]
        c1 = (rs * trs * g2, -1j * rs * g3)
        c2 = (1j * rs * trs * g3, rs * g2)
        c3 = (rs * tzs * g1, 0.0 * g1)
        return c1, c2, c3

    def c2nd(i):
        g1, g2, g3 = G1[i], G2[i], G3[i]
        c1 = (rs * trs * g2, -1j * rs * g3)
        c3 = (rs * tzs * g1, 0.0 * g1)
        return c1, c3

    c1, c2, c3 = cd(0)
    r1, r2, r3 = cd(1)
    z1, z2, z3 = cd(2)
    rr1, rr3 = c2nd(6)
    rz1, rz3 = c2nd(7)
    zz1, zz3 = c2nd(8)
    k0c = cvals(0)
    dkc = cvals(3)  # c-values of g^{k0} - g^{k1}
    K = np.zeros_like(N0)
    kd2 = k0 ** 2 - k1 ** 2
    for b in range(2):
        # k0^2 c(g^{k0}) - k1^2 c(g^{k1}) = (k0^2 - k1^2) c(g^{k0}) + k1^2 c(g^{k0} - g^{k1})
        Kt = (kd2 * k0c[1][b] + k1 ** 2 * dkc[1][b]) + (im / rt ** 2) * c1[b] \
            + (im / rt) * r1[b] - (m * m / rt ** 2) * c2[b] + (im / rt) * z3[b]
        dzD = (1 / rt) * z1[b] + rz1[b] + (im / rt) * z2[b] + zz3[b]
        drD = -c1[b] / rt ** 2 + (1 / rt) * r1[b] + rr1[b] - (im / rt ** 2) * c2[b] \
            + (im / rt) * r2[b] + rz3[b]
        kk = kd2 * (tzt * k0c[2][b] + trt * k0c[0][b]) + k1 ** 2 * (tzt * dkc[2][b] + trt * dkc[0][b])
        Kth = -(kk + tzt * dzD + trt * drD)
        K[0, b] = Kt
        K[1, b] = Kth
    iw = 1j * omega
    B = np.zeros((4, 4) + K.shape[2:], dtype=complex)
    if formulation == "direct":
        # mu0 N^{k0} - mu1 N^{k1} = (mu0 - mu1) N^{k0} + mu1 (N^{k0} - N^{k1})
        B[0:2, 0:2] = -iw * ((mu0 - mu1) * N0 + mu1 * dN)
        B[0:2, 2:4] = -K
        B[2:4, 0:2] = K
        B[2:4, 2:4] = -iw * ((eps0 - eps1) * N0 + eps1 * dN)
    elif formulation == "indirect":
        B[0:2, 0:2] = -iw * ((eps0 - eps1) * N0 + eps1 * dN)
        B[0:2, 2:4] = -(eps0 / mu0) * K
        B[2:4, 0:2] = (mu0 / eps0) * K
        B[2:4, 2:4] = -iw * ((mu0 - mu1) * N0 + mu1 * dN)
    else:
        raise ValueError(formulation)
    return B


def assemble_mode(curve, sup, table, m, k0, k1, omega, eps0, mu0, eps1, mu1, w, rows=None,
                  formulation="direct"):
    """Weighted matrix rows for mode m >= 0: [len(rows)*4, 4N] complex.

    table: [M+2, 9, len(rows), N+S] (rows as in oracle.modal.tabulate);
    formulation "direct" (eq. mullerrep) or "indirect" (eq. dualmullrep).
    """
    N = curve.n
    order = curve.order
    S = sup.r.shape[1]
    rows = np.arange(N) if rows is None else np.asarray(rows)
    tr_nodes = -curve.nz
    tz_nodes = curve.nr
    npan = curve.n_panels
    left, right = neighbours(npan, curve.closed)
    A = np.zeros((4 * rows.size, 4 * N), dtype=complex)
    sw = np.sqrt(w)
    for i, t in enumerate(rows):
        tab = table[[abs(m - 1), m, m + 1], :, i, :]  # [3, 9, N+S]
        rs = np.concatenate([curve.r, sup.r[t]])
        trs = np.concatenate([tr_nodes, sup.tr[t]])
        tzs = np.concatenate([tz_nodes, sup.tz[t]])
        B = blocks(tab, m, curve.r[t], tr_nodes[t], tz_nodes[t], rs, trs, tzs,
                   k0, k1, omega, eps0, mu0, eps1, mu1, formulation)  # [4, 4, N+S]
        p = t // order
        nearp = [p] + [q for q in (left[p], right[p]) if q >= 0]
        wts = w.copy()
        for q in nearp:
            wts[q * order:(q + 1) * order] = 0.0
        row = B[:, :, :N] * wts[None, None, :]  # far panels
        # near panels through the support nodes
        wq = sup.wq[t]
        contrib = B[:, :, N:] * wq[None, None, :]  # [4, 4, S]
        for s in range(S):
            pq = sup.panel[t, s]
            if pq < 0 or wq[s] == 0.0:
                continue
            row[:, :, pq * order:(pq + 1) * order] += contrib[:, :, s, None] * sup.lag[t, s][None, None, :]
        # jump terms
        if formulation == "direct":
            jJ, jM = 0.5j * omega * (mu0 + mu1), 0.5j * omega * (eps0 + eps1)
        else:
            jJ, jM = -0.5j * omega * (eps0 + eps1), -0.5j * omega * (mu0 + mu1)
        row[0, 0, t] += jJ
        row[1, 1, t] += jJ
        row[2, 2, t] += jM
        row[3, 3, t] += jM
        # [4, 4, N] -> rows 4i..4i+3, columns 4j + beta; L2 weighting
        blk = row.transpose(0, 2, 1).reshape(4, 4 * N)
        A[4 * i:4 * i + 4] = blk * (sw[t] / np.repeat(sw, 4))[None, :]
    return A
