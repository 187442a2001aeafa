"""Q1 finite element matrices on a uniform tensor grid (oracle; test infrastructure only).

Unknowns are the nodal values at interior nodes of the uniform partition of
each axis (Section 2.1, the space V_h of eq. (2.4)); Dirichlet nodes are
dropped.  Arrays of nodal values have shape (n_{d-1}, ..., n_0) with axis 0
(x) fastest, n_a = N_a - 1, so a flat index is sum_a i_a * prod_{b<a} n_b.

With periodic boundary conditions (the variant discussed at the end of
Section 4) the space is spanned by the periodic extensions of the hat
functions: node N_a coincides with node 0, the unknowns are the N_a nodes
j = 0 .. N_a - 1 of every axis and n_a = N_a.
"""
import itertools

import numpy as np
import scipy.sparse as sp


def p1_element_matrices(h):
    """Mass and stiffness matrices of one linear element of length h.

    Entry (a, b) of the mass matrix is the integral of phi_a * phi_b over the
    element and of the stiffness matrix the integral of phi_a' * phi_b', for
    the two hat-function pieces phi_0, phi_1 of the element (Section 2.1).
    """
    me = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    ke = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return me, ke


def assemble_1d(N, h, bc="dirichlet"):
    """1D mass matrix A and stiffness matrix B (dense).

    Built by summing element matrices over the N elements of the uniform
    partition.  Dirichlet: the two boundary nodes are removed (homogeneous
    data, eq. (2.1)), (N-1)x(N-1); Section 4 states the result as A = (h/6) R
    and B = (1/h) G^D.  Periodic: element N-1 joins node N-1 to node 0, NxN;
    Section 4 states B = (1/h) G^P.  The tests check both independently.
    """
    me, ke = p1_element_matrices(h)
    if bc == "periodic":
        m = np.zeros((N, N))
        k = np.zeros((N, N))
        for e in range(N):
            idx = [e, (e + 1) % N]
            for a in range(2):
                for b in range(2):
                    m[idx[a], idx[b]] += me[a, b]
                    k[idx[a], idx[b]] += ke[a, b]
        return m, k
    if bc != "dirichlet":
        raise ValueError(bc)
    full_m = np.zeros((N + 1, N + 1))
    full_k = np.zeros((N + 1, N + 1))
    for e in range(N):
        idx = [e, e + 1]
        for a in range(2):
            for b in range(2):
                full_m[idx[a], idx[b]] += me[a, b]
                full_k[idx[a], idx[b]] += ke[a, b]
    return full_m[1:N, 1:N].copy(), full_k[1:N, 1:N].copy()


def assemble_1d_all_nodes(N, h):
    """1D mass and stiffness matrices over all N + 1 nodes of the uniform
    partition (no node removed), summed from the element matrices."""
    me, ke = p1_element_matrices(h)
    m = np.zeros((N + 1, N + 1))
    k = np.zeros((N + 1, N + 1))
    for e in range(N):
        idx = [e, e + 1]
        for a in range(2):
            for b in range(2):
                m[idx[a], idx[b]] += me[a, b]
                k[idx[a], idx[b]] += ke[a, b]
    return m, k


def boundary_nodes(N):
    """Boolean mask over all nodes (shape (N_{d-1}+1, ..., N_0+1), x fastest) that
    marks the Dirichlet boundary nodes (some index equal to 0 or N_a)."""
    d = len(N)
    mask = np.zeros(tuple(N[a] + 1 for a in reversed(range(d))), dtype=bool)
    for a in range(d):
        sl = [slice(None)] * d
        sl[d - 1 - a] = 0
        mask[tuple(sl)] = True
        sl[d - 1 - a] = N[a]
        mask[tuple(sl)] = True
    return mask


def boundary_coupling(N, h, D, origin=None):
    """Interior-row, boundary-column blocks Mb, Kb of the all-node Q1 mass and
    stiffness matrices, and the coordinates of the boundary nodes.

    Nonhomogeneous Dirichlet data g(t) (the extension noted at the start of
    Section 4): writing u_h = sum_interior u_i phi_i + sum_boundary g_j(t) phi_j
    and testing eq. (2.3) with the interior hat functions gives
        M u' + K u = F - Mb g'(t) - Kb g(t),
    so the boundary values enter as one more forcing term.  The all-node
    matrices are Kronecker products of assemble_1d_all_nodes (x fastest);
    rows are the interior nodes in the package layout, columns the boundary
    nodes in the flat order of boundary_nodes(N).  Returns (Mb, Kb, Xb) with
    Xb a list of 1-D coordinate arrays, one per axis, of the boundary nodes.
    """
    d = len(N)
    origin = [0.0] * d if origin is None else list(origin)
    ones = [assemble_1d_all_nodes(N[a], h[a]) for a in range(d)]
    A = [ones[a][0] for a in range(d)]
    B = [ones[a][1] for a in range(d)]
    Mf = _kron_list([A[a] for a in reversed(range(d))])
    Kf = None
    for ax in range(d):
        term = _kron_list([B[a] if a == ax else A[a] for a in reversed(range(d))])
        Kf = term if Kf is None else Kf + term
    Kf = D * Kf
    bmask = boundary_nodes(N).reshape(-1)
    rows = np.flatnonzero(~bmask)
    cols = np.flatnonzero(bmask)
    Mb = Mf.tocsr()[rows][:, cols].tocsr()
    Kb = Kf.tocsr()[rows][:, cols].tocsr()
    full = np.meshgrid(*[origin[a] + h[a] * np.arange(N[a] + 1) for a in reversed(range(d))], indexing="ij")
    Xb = [full[d - 1 - a].reshape(-1)[cols] for a in range(d)]
    return Mb, Kb, Xb


def n_unknowns(N, bc="dirichlet"):
    """Unknowns per axis: N - 1 (Dirichlet) or N (periodic)."""
    return N if bc == "periodic" else N - 1


def _kron_list(mats):
    out = sp.csr_matrix(mats[0])
    for m in mats[1:]:
        out = sp.kron(out, sp.csr_matrix(m), format="csr")
    return out


def mass_stiffness(N, h, D, bc="dirichlet"):
    """Global mass M and stiffness K (sparse CSR) of the tensor Q1 space.

    Section 4, eq. (4.1): M = A_z (x) A_y (x) A_x and
    K = D * sum over axes of the same product with that axis' A replaced by
    its B.  Kronecker factors are ordered slowest axis first so that x is the
    fastest index, matching the array layout of this package.
    """
    d = len(N)
    ones = [assemble_1d(N[a], h[a], bc) for a in range(d)]
    A = [ones[a][0] for a in range(d)]
    B = [ones[a][1] for a in range(d)]
    M = _kron_list([A[a] for a in reversed(range(d))])
    K = None
    for ax in range(d):
        fac = [B[a] if a == ax else A[a] for a in reversed(range(d))]
        term = _kron_list(fac)
        K = term if K is None else K + term
    return M, (D * K).tocsr()


def q1_quadrature_assembly(N, h, D, origin=None, bc="dirichlet", all_nodes=False):
    """Mass and stiffness by Gauss quadrature over each Q1 element (dense).

    Independent of the Kronecker formula: for every box element, the 2^d
    multilinear shape functions and their gradients are evaluated at the
    2-point-per-axis Gauss points (exact for these polynomial integrands),
    giving (phi_i, phi_j) and a(phi_i, phi_j) = int D grad phi_i . grad phi_j
    (eq. (2.3)), which are summed into the interior-node numbering.
    With all_nodes=True no node is dropped: the numbering runs over all
    prod(N_a + 1) nodes (x fastest).  Only meant for tiny grids.
    """
    d = len(N)
    periodic = bc == "periodic"
    n = [N[a] + 1 if all_nodes else n_unknowns(N[a], bc) for a in range(d)]
    ndof = int(np.prod(n))
    strides = [int(np.prod(n[:a])) for a in range(d)]
    gp = np.array([-1.0, 1.0]) / np.sqrt(3.0)  # on [-1, 1]
    gw = np.array([1.0, 1.0])
    M = np.zeros((ndof, ndof))
    K = np.zeros((ndof, ndof))
    corners = list(itertools.product([0, 1], repeat=d))
    # reference element [0,1]^d scaled by h: shape fn of corner c is
    # prod_a (xi_a if c_a else 1 - xi_a), xi in [0,1]
    qpts = list(itertools.product(range(2), repeat=d))
    for elem in itertools.product(*[range(N[a]) for a in range(d)]):
        gidx = []
        for c in corners:
            node = [elem[a] + c[a] for a in range(d)]
            if all_nodes:
                gidx.append(sum(node[a] * strides[a] for a in range(d)))
            elif periodic:
                gidx.append(sum((node[a] % N[a]) * strides[a] for a in range(d)))
            elif any(node[a] == 0 or node[a] == N[a] for a in range(d)):
                gidx.append(-1)
            else:
                gidx.append(sum((node[a] - 1) * strides[a] for a in range(d)))
        me = np.zeros((len(corners), len(corners)))
        ke = np.zeros((len(corners), len(corners)))
        for q in qpts:
            xi = [(gp[q[a]] + 1.0) / 2.0 for a in range(d)]
            w = np.prod([gw[q[a]] * h[a] / 2.0 for a in range(d)])
            val = []
            grad = []
            for c in corners:
                f1 = [xi[a] if c[a] else 1.0 - xi[a] for a in range(d)]
                df = [(1.0 if c[a] else -1.0) / h[a] for a in range(d)]
                val.append(np.prod(f1))
                g = []
                for a in range(d):
                    g.append(df[a] * np.prod([f1[b] for b in range(d) if b != a]))
                grad.append(np.array(g))
            for i in range(len(corners)):
                for j in range(len(corners)):
                    me[i, j] += w * val[i] * val[j]
                    ke[i, j] += w * D * float(np.dot(grad[i], grad[j]))
        for i, gi in enumerate(gidx):
            if gi < 0:
                continue
            for j, gj in enumerate(gidx):
                if gj < 0:
                    continue
                M[gi, gj] += me[i, j]
                K[gi, gj] += ke[i, j]
    return M, K


def node_coords(N, h, origin=None, bc="dirichlet"):
    """Coordinates of the unknown nodes, one 1-D array per axis.

    Node j of axis a sits at a_a + j * h_a (Section 2.1); the unknowns are
    j = 1 .. N_a - 1 (Dirichlet) or j = 0 .. N_a - 1 (periodic).
    """
    d = len(N)
    origin = [0.0] * d if origin is None else list(origin)
    first = 0 if bc == "periodic" else 1
    return [origin[a] + h[a] * np.arange(first, N[a]) for a in range(d)]


def mesh(N, h, origin=None, bc="dirichlet"):
    """Broadcastable coordinate arrays shaped like a nodal array (x fastest)."""
    d = len(N)
    xs = node_coords(N, h, origin, bc)
    out = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = len(xs[a])
        out.append(xs[a].reshape(shape))
    return out
