"""Host checks of the tree-cotree split (etpic_tree_cotree, no GPU): the
spanning trees are valid (acyclic, spanning; the split is not unique, so its
validity is what is checked), the restricted incidences are nonsingular, and
a divergence-free field (the oracle's projections) is fixed by its cotree
values."""
import numpy as np
import pytest

from paper_2208_12795_amd import etpic, synth

EPS0 = 8.8541878128e-12


class UnionFind:
    def __init__(self, n):
        self.p = np.arange(n)

    def find(self, a):
        while self.p[a] != a:
            self.p[a] = self.p[self.p[a]]
            a = self.p[a]
        return a

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.p[ra] = rb
        return True


@pytest.fixture(scope="module", params=[(1, 1, 1), (4, 3, 5)])
def case(request, ora):
    xyz, tv = synth.kuhn_mesh(request.param, (1.0, 0.8, 1.2), 0.15, np.random.default_rng(6))
    et, ft = etpic.tree_cotree(xyz, tv)
    return ora.OracleMesh(xyz, tv), et, ft


def test_edge_tree_spans_the_vertices(case):
    m, et, _ = case
    assert et.sum() == m.nv - 1 and (~et).sum() == m.ne - m.nv + 1
    uf = UnionFind(m.nv)
    for a, b in m.edges()[et]:
        assert uf.union(a, b)                     # no cycle
    assert len({uf.find(v) for v in range(m.nv)}) == 1


def test_face_tree_spans_the_dual_graph(case):
    """Dual graph: tets plus the exterior (node N_t); a face joins its tets,
    a boundary face its tet and the exterior."""
    m, _, ft = case
    assert ft.sum() == m.nt and (~ft).sum() == m.nf - m.nt
    owners = [[] for _ in range(m.nf)]
    for t, fs in enumerate(m.tet_faces()):
        for f in fs:
            owners[f].append(t)
    uf = UnionFind(m.nt + 1)
    for f in np.flatnonzero(ft):
        a, b = (owners[f] + [m.nt])[:2]
        assert uf.union(a, b)
    assert len({uf.find(v) for v in range(m.nt + 1)}) == 1


def test_restricted_incidences_are_nonsingular(case):
    """D on the tree edges without the root vertex, and div on the tree faces,
    are square and nonsingular (determinant +-1: unimodular)."""
    from oracle import gauss, qh
    m, et, ft = case
    D = gauss.incidence(m).toarray()[et][:, 1:]
    assert D.shape == (m.nv - 1, m.nv - 1)
    assert np.isclose(abs(np.linalg.det(D)), 1.0)
    Dv = qh.div_matrix(m).toarray()[:, ft]
    assert Dv.shape == (m.nt, m.nt)
    assert np.isclose(abs(np.linalg.det(Dv)), 1.0)


def test_divergence_free_fields_follow_from_their_cotree_values(case):
    """P^Lambda_b b is fixed by its cotree faces (div_T b_T = -div_C b_C); a
    field with Sigma^T v = 0 (P^Lambda_e d) by its cotree edges."""
    from oracle import qh
    m, et, ft = case
    Q = qh.QhOracle(m, EPS0)
    rng = np.random.default_rng(8)
    b = Q.project_b(rng.standard_normal(m.nf))
    div = Q.div.toarray()
    bt = np.linalg.solve(div[:, ft], -div[:, ~ft] @ b[~ft])
    assert np.abs(bt - b[ft]).max() < 1e-10 * np.abs(b).max()
    _, v, _ = Q.project_e(rng.standard_normal(m.ne) * 1e-11)
    St = Q.Sigma.T.toarray()
    vt = np.linalg.lstsq(St[:, et], -St[:, ~et] @ v[~et], rcond=None)[0]
    assert np.abs(vt - v[et]).max() < 1e-8 * np.abs(v).max()


def test_projectors_reject_a_disconnected_mesh():
    """Two separate tets: Sigma^T Sigma would have two constant null vectors;
    the projector object refuses the mesh before it touches a device."""
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0],
                    [5, 0, 0], [6, 0, 0], [5, 1, 0], [5, 0, 1.0]])
    tv = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    with pytest.raises(etpic.EtpicError) as e:
        etpic.QhProjectors(xyz, tv, EPS0)
    assert e.value.code == etpic.EMESH
    et, ft = etpic.tree_cotree(xyz, tv)           # a forest: one tree per component
    assert et.sum() == 8 - 2 and ft.sum() == 2
