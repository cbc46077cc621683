"""TRT-RLB lattice Boltzmann update in NumPy, FP64.  Test infrastructure.

An independent second definition of the collision, written from Sec. 2.2
of arXiv 2602.06686 (Eq. TRT-RLB with the Hermite projection Eq. projection
and reconstruction Eq. R2R3_hermite), sharing no code or table with the C
oracle.  The paper's equivalence theorems (Theorems 2 and 3, Remark on
exactness) state that it gives the same post-collision state as P-TRT on
D2Q9 and D3Q19, which is what the tests use it for.

Readings (the same as the C oracle's where they overlap):

* tau_{s,1} also relaxes the first-order non-equilibrium moment (the sentence
  after Eq. TRT-RLB; order-epsilon Chapman-Enskog equation).  That term is
  computed here from f^neq itself: w_i e_ia (sum_j e_ja f^neq_j) / c_s^2.
* Source term: Scheme II (Eq. source_simple), with or without the cubic
  correction G_i (Eq. Gi; Phi_aaa = rho u_a^3, central differences with
  periodic wrap, Phi = 0 at solid nodes), or Scheme I (Eq. source_guo) with
  the -u.F/c_s^2 part under the tau+ factor (as printed it sits under the
  tau- factor, which does not conserve mass).  With Scheme I the first-order
  non-equilibrium moment relaxes with tau- (standard TRT, the antisymmetric
  rate), which gives a momentum gain of exactly F.
* Third-order reconstruction on D3Q19.  The literal tensor contraction of
  Eq. R2R3_hermite is an orthogonal projection only if the independent
  third-order Hermite polynomials are mutually orthogonal under the weighted
  inner product.  That holds on D2Q9 but not on D3Q19 (H_xxy and H_yzz
  overlap), so the reconstruction here is the orthogonal projection onto
  their span, R3_i = w_i sum_kl H_ki (G^-1)_kl A_l with the Gram matrix
  G_kl = sum_i w_i H_ki H_li.  On D2Q9 that equals the printed formula
  (checked by a test).
* D3Q27 (App. A.3) has seven third-order modes (the six H_aab and H_xyz);
  they are mutually orthogonal there, so the printed contraction is the
  projection, as on D2Q9 (checked by a test).
"""
import itertools

import numpy as np

CS2 = 1.0 / 3.0


def d2q9():
    """Eq. D2Q9, printed order."""
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                  [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.float64)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return e, w


def d3q19():
    """D3Q19 (App. A.2): rest, 6 axial, 12 face diagonals; textbook weights."""
    vel = [(0, 0, 0)]
    for a in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[a] = s
            vel.append(tuple(v))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
            v = [0, 0, 0]
            v[a], v[b] = sa, sb
            vel.append(tuple(v))
    e = np.array(vel, dtype=np.float64)
    n2 = (e ** 2).sum(1)
    w = np.where(n2 == 0, 1 / 3, np.where(n2 == 1, 1 / 18, 1 / 36))
    return e, w


def d3q27():
    """D3Q27 (App. A.3): every velocity with components in {-1, 0, 1}; the
    D3Q19 order, then the body diagonals, each followed by its opposite;
    weights are products of the 1D weights 2/3 (0) and 1/6 (+-1)."""
    e19, _ = d3q19()
    diag = [(1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
            (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]
    e = np.vstack([e19, np.array(diag, dtype=np.float64)])
    w = np.prod(np.where(e == 0, 2 / 3, 1 / 6), axis=1)
    return e, w


def lattice(name):
    return {"D2Q9": d2q9, "D3Q19": d3q19, "D3Q27": d3q27}[name]()


def opposite(e):
    return np.array([int(np.where((e == -ei).all(1))[0][0]) for ei in e])


def hermite2(e):
    """H^(2)_{i,ab} = e_ia e_ib - c_s^2 delta_ab, shape [Q,D,D]."""
    D = e.shape[1]
    return np.einsum("ia,ib->iab", e, e) - CS2 * np.eye(D)[None]


def hermite3(e):
    """H^(3)_{i,abc} = e_ia e_ib e_ic - c_s^2 (e_ia d_bc + e_ib d_ca + e_ic d_ab)."""
    D = e.shape[1]
    d = np.eye(D)
    return (np.einsum("ia,ib,ic->iabc", e, e, e)
            - CS2 * (np.einsum("ia,bc->iabc", e, d) + np.einsum("ib,ca->iabc", e, d)
                     + np.einsum("ic,ab->iabc", e, d)))


def equilibrium(e, w, rho, u):
    """Eq. feq with every Hermite tensor term; rho [n], u [n,D] -> [n,Q]."""
    H2 = hermite2(e)
    H3 = hermite3(e)
    t1 = u @ e.T
    t2 = np.einsum("iab,na,nb->ni", H2, u, u)
    t3 = np.einsum("iabc,na,nb,nc->ni", H3, u, u, u)
    return w[None] * rho[:, None] * (1 + t1 / CS2 + t2 / (2 * CS2 ** 2) + t3 / (6 * CS2 ** 3))


def third_order_modes(e):
    """The independent third-order polynomials H_aab (a != b) and, where the
    lattice supports it (not identically zero), H_xyz, as rows [M,Q]."""
    H3 = hermite3(e)
    D = e.shape[1]
    rows = []
    for a, b in itertools.permutations(range(D), 2):
        rows.append(H3[:, a, a, b])
    if D == 3 and np.any(H3[:, 0, 1, 2] != 0):
        rows.append(H3[:, 0, 1, 2])
    return np.array(rows)


def reconstruct_third_literal(e, w, fneq):
    """R^(3) of Eq. R2R3_hermite as printed: w_i H^(3)_i : A^(3) / (6 c_s^6)."""
    H3 = hermite3(e)
    A3 = np.einsum("iabc,ni->nabc", H3, fneq)
    return w[None] * np.einsum("iabc,nabc->ni", H3, A3) / (6 * CS2 ** 3)


def reconstruct_third_projection(e, w, fneq):
    """Orthogonal projection of f^neq onto the span of the third-order modes."""
    M = third_order_modes(e)
    G = (M * w[None]) @ M.T
    A = fneq @ M.T
    return w[None] * (A @ np.linalg.inv(G) @ M)


def collide(lattice_name, f, g, tau_plus, tau_minus, third="auto", scheme="II", dphi=None):
    """TRT-RLB post-collision state, f [n,Q] -> [n,Q] (Eq. TRT-RLB).

    g is the body acceleration (F = rho g).  ``third`` selects the third-order
    reconstruction: "literal", "projection" or "auto" (literal on D2Q9 and
    D3Q27, projection on D3Q19).  ``scheme``: "II" (Eq. source_simple without
    G_i), "II+G" (with G_i; ``dphi`` [n,D] holds d_a Phi_aaa per node) or
    "I" (Eq. source_guo, mass-conserving split)."""
    e, w = lattice(lattice_name)
    D = e.shape[1]
    g = np.zeros(D) if g is None else np.asarray(g, dtype=np.float64)[:D]
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(1)
    F = rho[:, None] * g[None]
    u = (f @ e + 0.5 * F) / rho[:, None]                     # Eq. macro
    feq = equilibrium(e, w, rho, u)
    fneq = f - feq
    H2 = hermite2(e)
    A2 = np.einsum("iab,ni->nab", H2, fneq)                  # Eq. projection
    R2 = w[None] * np.einsum("iab,nab->ni", H2, A2) / (2 * CS2 ** 2)
    if third == "auto":
        third = "projection" if lattice_name == "D3Q19" else "literal"
    R3 = (reconstruct_third_literal if third == "literal" else reconstruct_third_projection)(e, w, fneq)
    P1 = w[None] * ((fneq @ e) @ e.T) / CS2                  # first-order part
    ap, am = 1 - 1 / tau_plus, 1 - 1 / tau_minus
    bp, bm = 1 - 1 / (2 * tau_plus), 1 - 1 / (2 * tau_minus)
    if scheme == "I":
        eu, eF = u @ e.T, F @ e.T
        uF = (u * F).sum(1)[:, None]
        S = w[None] * (bp * (eu * eF / CS2 ** 2 - uF / CS2) + bm * eF / CS2)
        return feq + ap * R2 + am * (P1 + R3) + S
    S = bp * w[None] * (F @ e.T) / CS2                       # Scheme II
    if scheme == "II+G":
        T = np.einsum("na,ab->nab", np.asarray(dphi, dtype=np.float64)[:, :D], np.eye(D))
        S = S - bp * w[None] * np.einsum("iab,nab->ni", H2, T) / (6 * CS2 ** 3)
    elif scheme != "II":
        raise ValueError(scheme)
    return feq + ap * (R2 + P1) + am * R3 + S


def phi_gradient(lattice_name, f, shape, g, solid=None):
    """d_a (rho u_a^3) by central differences with periodic wrap, Phi = 0 at
    solid nodes; f [Q, *shape] -> [N, D]."""
    e, _ = lattice(lattice_name)
    Q, D = e.shape
    fl = f.reshape(Q, -1)
    rho = fl.sum(0)
    g = np.zeros(D) if g is None else np.asarray(g, dtype=np.float64)[:D]
    safe = np.where(rho == 0.0, 1.0, rho)                      # solid nodes hold zeros
    u = (e.T @ fl + 0.5 * rho[None] * g[:, None]) / safe[None]
    phi = rho[None] * u ** 3
    if solid is not None:
        phi[:, np.asarray(solid, dtype=bool).ravel()] = 0.0
    nd = len(shape)
    out = np.zeros((fl.shape[1], D))
    for a in range(D):
        axis = nd - 1 - a                                     # x is the last array axis
        p = phi[a].reshape(shape)
        out[:, a] = (0.5 * (np.roll(p, -1, axis=axis) - np.roll(p, 1, axis=axis))).ravel()
    return out


def stream(lattice_name, fstar, shape, solid=None):
    """Collide-then-stream transport with periodic wrap and halfway
    bounce-back; fstar [Q, *shape] -> f [Q, *shape] (shape = (nz, ny, nx)
    or (ny, nx)).  Solid-node entries are left at zero."""
    e, _ = lattice(lattice_name)
    opp = opposite(e)
    Q = e.shape[0]
    out = np.zeros_like(fstar)
    nd = len(shape)
    axes = tuple(range(nd))[::-1]  # x is the last array axis
    for i in range(Q):
        shift = [0] * nd
        for a in range(e.shape[1]):
            shift[axes[a]] = int(e[i, a])
        moved = np.roll(fstar[i], shift=shift, axis=tuple(range(nd)))
        if solid is None:
            out[i] = moved
        else:
            # target x+e_i solid: the population returns as opp(i) at its source
            dest_solid = np.roll(solid, shift=[-s for s in shift], axis=tuple(range(nd)))
            out[opp[i]] += np.where(dest_solid & ~solid, fstar[i], 0.0)
            out[i] += np.where(~solid, np.where(np.roll(solid, shift=shift, axis=tuple(range(nd))),
                                                 0.0, moved), 0.0)
    return out


def run(lattice_name, f, shape, g, tau_plus, tau_minus, nsteps, solid=None, scheme="II"):
    """Advance populations f [Q, *shape] by nsteps TRT-RLB steps."""
    e, _ = lattice(lattice_name)
    Q = e.shape[0]
    f = np.array(f, dtype=np.float64).reshape((Q,) + tuple(shape))
    sol = None if solid is None else np.asarray(solid, dtype=bool).reshape(shape)
    for _ in range(nsteps):
        flat = f.reshape(Q, -1).T
        dphi = phi_gradient(lattice_name, f, shape, g, sol) if scheme == "II+G" else None
        if sol is None:
            fs = collide(lattice_name, flat, g, tau_plus, tau_minus, scheme=scheme, dphi=dphi)
        else:
            fs = np.zeros_like(flat)
            fl = ~sol.ravel()
            fs[fl] = collide(lattice_name, flat[fl], g, tau_plus, tau_minus, scheme=scheme,
                             dphi=None if dphi is None else dphi[fl])
        f = stream(lattice_name, fs.T.reshape(f.shape), shape, sol)
    return f
