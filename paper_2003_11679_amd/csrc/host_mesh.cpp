// RWG topology of concatenated closed triangle meshes (Sec. III-A: n x E and
// n x H expanded in RWG functions).  Standard RWG definition (Rao, Wilton and
// Glisson 1982): on T+ of edge n, f_n = l/(2A+) (r - p+); on T-,
// f_n = -l/(2A-) (r - p-).  Numbering: interior edges {a, b}, a < b, sorted by
// (a, b); T+ is the triangle whose counter-clockwise order runs a -> b.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace sie {

void build_topology(Mesh &m) {
    const int64_t T = m.nt();
    m.area.assign(T, 0.0);
    m.normal.assign(3 * T, 0.0);
    m.centroid.assign(3 * T, 0.0);
    for (int64_t t = 0; t < T; ++t) {
        const double *v[3];
        for (int k = 0; k < 3; ++k) {
            int32_t vi = m.tri[3 * t + k];
            SIE_CHECK(vi >= 0 && vi < m.nv(), SIE_EMESH, "triangle vertex index out of range");
            v[k] = &m.xyz[3 * vi];
        }
        double e1[3], e2[3], c[3];
        for (int k = 0; k < 3; ++k) { e1[k] = v[1][k] - v[0][k]; e2[k] = v[2][k] - v[0][k]; }
        c[0] = e1[1] * e2[2] - e1[2] * e2[1];
        c[1] = e1[2] * e2[0] - e1[0] * e2[2];
        c[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double nn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        SIE_CHECK(nn > 0.0, SIE_EMESH, "degenerate triangle " + std::to_string(t));
        m.area[t] = 0.5 * nn;
        for (int k = 0; k < 3; ++k) {
            m.normal[3 * t + k] = c[k] / nn;
            // ((v0 + v1) + v2) / 3, evaluated in this order (stencil anchoring
            // depends on these bits)
            volatile double s = v[0][k] + v[1][k];
            s = s + v[2][k];
            m.centroid[3 * t + k] = s / 3.0;
        }
    }
    // half-edges: key (min, max), triangle, local edge (opposite vertex), forward?
    struct HE { int32_t a, b, t, e; bool fwd; };
    std::vector<HE> he;
    he.reserve(3 * T);
    for (int64_t t = 0; t < T; ++t)
        for (int e = 0; e < 3; ++e) {
            int32_t p = m.tri[3 * t + (e + 1) % 3], q = m.tri[3 * t + (e + 2) % 3];
            SIE_CHECK(p != q, SIE_EMESH, "repeated vertex in triangle " + std::to_string(t));
            he.push_back({std::min(p, q), std::max(p, q), (int32_t)t, e, p < q});
        }
    std::sort(he.begin(), he.end(), [](const HE &x, const HE &y) {
        return x.a != y.a ? x.a < y.a : (x.b != y.b ? x.b < y.b : x.fwd > y.fwd);
    });
    SIE_CHECK(he.size() % 2 == 0, SIE_EMESH, "odd number of half-edges: mesh not closed");
    const int64_t E = (int64_t)he.size() / 2;
    m.nrwg = E;
    m.edge_v.assign(2 * E, 0);
    m.tpm.assign(2 * E, 0);
    m.epm.assign(2 * E, 0);
    m.len.assign(E, 0.0);
    m.tri_rwg.assign(3 * T, -1);
    m.tri_sign.assign(3 * T, 0.0);
    for (int64_t n = 0; n < E; ++n) {
        const HE &h0 = he[2 * n], &h1 = he[2 * n + 1];
        SIE_CHECK(h0.a == h1.a && h0.b == h1.b, SIE_EMESH,
                  "edge (" + std::to_string(h0.a) + "," + std::to_string(h0.b) + ") not shared by two triangles");
        if (2 * n + 2 < (int64_t)he.size())
            SIE_CHECK(!(he[2 * n + 2].a == h0.a && he[2 * n + 2].b == h0.b), SIE_EMESH,
                      "edge shared by more than two triangles");
        SIE_CHECK(h0.fwd && !h1.fwd, SIE_EMESH, "inconsistent triangle orientation");
        SIE_CHECK(m.tri_obj[h0.t] == m.tri_obj[h1.t], SIE_EMESH, "edge shared between objects");
        m.edge_v[2 * n] = h0.a; m.edge_v[2 * n + 1] = h0.b;
        m.tpm[2 * n] = h0.t; m.tpm[2 * n + 1] = h1.t;
        m.epm[2 * n] = h0.e; m.epm[2 * n + 1] = h1.e;
        const double *pa = &m.xyz[3 * h0.a], *pb = &m.xyz[3 * h0.b];
        double d0 = pb[0] - pa[0], d1 = pb[1] - pa[1], d2 = pb[2] - pa[2];
        m.len[n] = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        m.tri_rwg[3 * h0.t + h0.e] = (int32_t)n; m.tri_sign[3 * h0.t + h0.e] = 1.0;
        m.tri_rwg[3 * h1.t + h1.e] = (int32_t)n; m.tri_sign[3 * h1.t + h1.e] = -1.0;
    }
    // RWG ranges per object (vertex numbering is object-contiguous, so the
    // (a, b) order keeps objects contiguous)
    m.obj_rwg0.assign(m.nobj + 1, E);
    for (int64_t n = E - 1; n >= 0; --n) m.obj_rwg0[m.tri_obj[m.tpm[2 * n]]] = n;
    for (int i = m.nobj - 1; i >= 0; --i)
        if (m.obj_rwg0[i] > m.obj_rwg0[i + 1]) m.obj_rwg0[i] = m.obj_rwg0[i + 1];
}

}  // namespace sie
