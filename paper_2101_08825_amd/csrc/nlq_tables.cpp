// Host-side tables: quadrature rules, kernel constants and the barycentric
// coordinates of the quadrature points of every sub-element produced by the
// midpoint refinement of Algorithm 1 (Section 5).
#include <cmath>

#include <map>
#include <vector>

#include "nlq_box.hpp"
#include "nlq_internal.hpp"
#include "nlq_p2.hpp"
#include "nlq_refine.hpp"

namespace nlq {

namespace {

// Degree-5 rules on the reference simplex; barycentric points, weights sum 1.
// Triangle: the 7-point Radon / Dunavant rule named in Section 6: centroid,
// then the orbits (1-2a, a, a) and (1-2b, b, b), a,b = (6 -+ sqrt 15)/21, each
// listed with the distinguished coordinate in position 0, 1, 2.
// Tetrahedron: Keast's 15-point rule: centroid; (0,1/3,1/3,1/3) orbit;
// (8/11,1/11,1/11,1/11) orbit (distinguished coordinate in position 0..3);
// (c,c,d,d) orbit with c = (13 - sqrt 91)/52, d = 1/2 - c, the two c's at the
// index pairs (0,1),(0,2),(0,3),(1,2),(1,3),(2,3).
void simplex_rule(int dim, std::vector<double> &bary, std::vector<double> &w)
{
    if (dim == 2) {
        const double r15 = std::sqrt(15.0);
        const double orbit_a[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
        const double orbit_w[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
        bary = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
        w = {9.0 / 40.0};
        for (int o = 0; o < 2; ++o)
            for (int pos = 0; pos < 3; ++pos) {
                for (int j = 0; j < 3; ++j)
                    bary.push_back(j == pos ? 1.0 - 2.0 * orbit_a[o] : orbit_a[o]);
                w.push_back(orbit_w[o]);
            }
        return;
    }
    const double wc = 0.1817020685825350548382618;
    const double w_face = 0.03616071428571428571428571;
    const double w_11 = 0.06987149451617381646536165;
    const double w_edge = 0.06569484936831875607385811;
    bary = {0.25, 0.25, 0.25, 0.25};
    w = {wc};
    for (int pos = 0; pos < 4; ++pos) {
        for (int j = 0; j < 4; ++j) bary.push_back(j == pos ? 0.0 : 1.0 / 3.0);
        w.push_back(w_face);
    }
    for (int pos = 0; pos < 4; ++pos) {
        for (int j = 0; j < 4; ++j) bary.push_back(j == pos ? 8.0 / 11.0 : 1.0 / 11.0);
        w.push_back(w_11);
    }
    const double c = (13.0 - std::sqrt(91.0)) / 52.0;
    const double d = 0.5 - c;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j) {
            for (int k = 0; k < 4; ++k) bary.push_back((k == i || k == j) ? c : d);
            w.push_back(w_edge);
        }
}

// Gauss-Legendre rule on [-1, 1]: roots of P_n by Newton from the Tricomi
// initial guess; weights 2 / ((1 - x^2) P_n'(x)^2).
void legendre_rule(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int k = 1; k <= n; ++k) {
        double t = std::cos(pi * (4.0 * k - 1.0) / (4.0 * n + 2.0));
        double deriv = 1.0;
        for (int iter = 0; iter < 60; ++iter) {
            double pm1 = 1.0, p = t;
            for (int j = 1; j < n; ++j) {
                double pn = ((2.0 * j + 1.0) * t * p - j * pm1) / (j + 1.0);
                pm1 = p;
                p = pn;
            }
            deriv = n * (pm1 - t * p) / (1.0 - t * t);
            double step = p / deriv;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double pm1 = 1.0, p = t;
        for (int j = 1; j < n; ++j) {
            double pn = ((2.0 * j + 1.0) * t * p - j * pm1) / (j + 1.0);
            pm1 = p;
            p = pn;
        }
        deriv = n * (pm1 - t * p) / (1.0 - t * t);
        x[k - 1] = t;
        w[k - 1] = 2.0 / ((1.0 - t * t) * deriv * deriv);
    }
}

double xi_host(double r)
{
    double s = r * r;
    return 0.5 + r * (315.0 / 256.0 + s * (-420.0 / 256.0 + s * (378.0 / 256.0 +
                                            s * (-180.0 / 256.0 + s * (35.0 / 256.0)))));
}

// Polynomials in the barycentric coordinates: exponent vector -> coefficient.
using Poly = std::map<std::vector<int>, double>;

Poly poly_mul(const Poly &a, const Poly &b)
{
    Poly out;
    for (const auto &x : a)
        for (const auto &y : b) {
            std::vector<int> e(x.first.size());
            for (size_t k = 0; k < e.size(); ++k) e[k] = x.first[k] + y.first[k];
            out[e] += x.second * y.second;
        }
    return out;
}

// P2 basis function I as a homogeneous quadratic (sum lambda = 1 inserted where
// the degree is lower): vertex i: 2 lambda_i^2 - lambda_i sum_k lambda_k; edge
// (i, j): 4 lambda_i lambda_j (edges in lexicographic order).
Poly p2_basis_hom(int nv, int I)
{
    Poly p;
    auto unit = [&](int i, int j) {
        std::vector<int> e(nv, 0);
        e[i] += 1;
        e[j] += 1;
        return e;
    };
    if (I < nv) {
        p[unit(I, I)] += 2.0;
        for (int k = 0; k < nv; ++k) p[unit(I, k)] -= 1.0;
        return p;
    }
    int r = nv;
    for (int i = 0; i < nv; ++i)
        for (int j = i + 1; j < nv; ++j, ++r)
            if (r == I) p[unit(i, j)] = 4.0;
    return p;
}

}  // namespace

// Map from the monomial rows accumulated for P2 elements to the rows the
// epilogue needs (see nlq_p2.hpp): [NU + NB + 1][NR] with rows
//   u < NU          phi_I phi_J for the upper-triangle slot u = (I, J) (u < NB the
//                   diagonal, then I < J in lexicographic order),
//   NU + I          phi_I (sum lambda)^2,
//   NU + NB         (sum lambda)^4,
// every one a homogeneous quartic written in the monomials of Mono4.
std::vector<double> make_p2_map(int dim)
{
    const int nv = dim + 1, nb = p2_nodes(dim), nu = nb * (nb + 1) / 2, nr = p2_monomials(dim);
    std::vector<std::vector<int>> mono;
    if (nv == 3) {
        constexpr Mono4<3> m{};
        for (int k = 0; k < m.N; ++k) mono.emplace_back(m.e[k], m.e[k] + 3);
    } else {
        constexpr Mono4<4> m{};
        for (int k = 0; k < m.N; ++k) mono.emplace_back(m.e[k], m.e[k] + 4);
    }
    std::map<std::vector<int>, int> index;
    for (int k = 0; k < nr; ++k) index[mono[k]] = k;
    Poly sum1;
    for (int k = 0; k < nv; ++k) {
        std::vector<int> e(nv, 0);
        e[k] = 1;
        sum1[e] = 1.0;
    }
    const Poly sum2 = poly_mul(sum1, sum1), sum4 = poly_mul(sum2, sum2);
    std::vector<Poly> rows(nu + nb + 1);
    std::vector<Poly> phi(nb);
    for (int I = 0; I < nb; ++I) phi[I] = p2_basis_hom(nv, I);
    for (int u = 0; u < nu; ++u) {
        int I = u, J = u;
        if (u >= nb) {
            int r = nb;
            for (int a = 0; a < nb; ++a)
                for (int c = a + 1; c < nb; ++c, ++r)
                    if (r == u) {
                        I = a;
                        J = c;
                    }
        }
        rows[u] = poly_mul(phi[I], phi[J]);
    }
    for (int I = 0; I < nb; ++I) rows[nu + I] = poly_mul(phi[I], sum2);
    rows[nu + nb] = sum4;
    std::vector<double> map(static_cast<size_t>(nu + nb + 1) * nr, 0.0);
    for (size_t r = 0; r < rows.size(); ++r)
        for (const auto &t : rows[r]) {
            auto it = index.find(t.first);
            if (it == index.end()) fail(NLQ_EDEVICE, "P2 map: a product is not a quartic");
            map[r * nr + it->second] += t.second;
        }
    // the kernels keep the map in FP32: every coefficient is a small integer
    for (double v : map)
        if (static_cast<double>(static_cast<float>(v)) != v || v != std::floor(v))
            fail(NLQ_EDEVICE, "P2 map: a coefficient is not a small integer");
    return map;
}

// Tables of quadrilateral / hexahedral elements (see nlq_box.hpp).  The nodal
// basis is built from its definition: phi_I is the function of the element's
// space (Q1 or serendipity monomials on [0,1]^N) with phi_I(node_J) = delta_IJ,
// from the inverse of the space's Vandermonde matrix at the nodes.  Returns
//   rule  [nq][dim] points, then [nq] weights (product order of nlq_box.hpp);
//   psi   [nb][qs]  phi_J at rule point b (qs = 16 in 2D, 32 in 3D, padding 0);
//   phi   [nb][nr]  phi_I over the product monomials of BoxMono;
//   prod  [nu][nr]  phi_I phi_J, slot u: u < nb the diagonal, then I < J in
//                   lexicographic order.
BoxTablesHost make_box_tables(int dim, int order)
{
    const int nq = box_nq(dim), qs = dim == 2 ? 16 : 32, nb = box_node_count(dim, order);
    const int nu = nb * (nb + 1) / 2;
    BoxTablesHost T;
    T.rule.assign(static_cast<size_t>(nq) * (dim + 1), 0.0);
    for (int q = 0; q < nq; ++q) {
        const int i[3] = {q % 3, (q / 3) % 3, q / 9};
        double w = 1.0;
        for (int k = 0; k < dim; ++k) {
            T.rule[q * dim + k] = box_gauss_node(i[k]);
            w *= box_gauss_weight(i[k]);
        }
        T.rule[nq * dim + q] = w;
    }
    using E3 = std::vector<int>;
    std::vector<E3> rows, space;
    for (int q = 0; q < (dim == 2 ? 25 : 125); ++q) {
        int e[3] = {q % 5, (q / 5) % 5, q / 25};
        if (box_is_product(order, dim, e)) rows.push_back(E3(e, e + dim));
    }
    for (int q = 0; q < (dim == 2 ? 9 : 27); ++q) {
        int e[3] = {q % 3, (q / 3) % 3, q / 9};
        if (box_in_space(order, dim, e)) space.push_back(E3(e, e + dim));
    }
    if (static_cast<int>(space.size()) != nb) fail(NLQ_EDEVICE, "box element space size mismatch");
    std::vector<E3> nodes;
    for (int c = 0; c < (1 << dim); ++c) {
        E3 t(dim);
        for (int k = 0; k < dim; ++k) t[k] = 2 * ((c >> k) & 1);
        nodes.push_back(t);
    }
    if (order == 2)
        for (int q = 0; q < (dim == 2 ? 9 : 27); ++q) {
            E3 t(dim);
            int odd = 0;
            for (int k = 0; k < dim; ++k) {
                t[k] = (q / (k == 0 ? 1 : (k == 1 ? 3 : 9))) % 3;
                odd += t[k] == 1;
            }
            if (odd == 1) nodes.push_back(t);
        }
    auto mono = [&](const E3 &e, const double *x) {
        double v = 1.0;
        for (int k = 0; k < dim; ++k) v *= std::pow(x[k], e[k]);
        return v;
    };
    // Vandermonde V[i][j] = space_j(node_i), inverted by Gauss-Jordan elimination
    std::vector<double> V(static_cast<size_t>(nb) * nb), Cinv(static_cast<size_t>(nb) * nb, 0.0);
    for (int i = 0; i < nb; ++i) {
        double x[3];
        for (int k = 0; k < dim; ++k) x[k] = 0.5 * nodes[i][k];
        for (int j = 0; j < nb; ++j) V[i * nb + j] = mono(space[j], x);
        Cinv[i * nb + i] = 1.0;
    }
    for (int col = 0; col < nb; ++col) {
        int piv = col;
        for (int r = col + 1; r < nb; ++r)
            if (std::fabs(V[r * nb + col]) > std::fabs(V[piv * nb + col])) piv = r;
        if (std::fabs(V[piv * nb + col]) < 1e-12) fail(NLQ_EDEVICE, "box basis: singular Vandermonde matrix");
        for (int c = 0; c < nb; ++c) {
            std::swap(V[col * nb + c], V[piv * nb + c]);
            std::swap(Cinv[col * nb + c], Cinv[piv * nb + c]);
        }
        const double d = V[col * nb + col];
        for (int c = 0; c < nb; ++c) {
            V[col * nb + c] /= d;
            Cinv[col * nb + c] /= d;
        }
        for (int r = 0; r < nb; ++r) {
            if (r == col) continue;
            const double f = V[r * nb + col];
            if (f == 0.0) continue;
            for (int c = 0; c < nb; ++c) {
                V[r * nb + c] -= f * V[col * nb + c];
                Cinv[r * nb + c] -= f * Cinv[col * nb + c];
            }
        }
    }
    // phi_I = sum_j Cinv[j][I] space_j
    const int nr = static_cast<int>(rows.size());
    auto row_of = [&](const E3 &e) {
        for (int r = 0; r < nr; ++r)
            if (rows[r] == e) return r;
        fail(NLQ_EDEVICE, "box basis: a product is not among the rows");
        return -1;
    };
    T.phi.assign(static_cast<size_t>(nb) * nr, 0.0);
    for (int I = 0; I < nb; ++I)
        for (int j = 0; j < nb; ++j) T.phi[I * nr + row_of(space[j])] += Cinv[j * nb + I];
    T.prod.assign(static_cast<size_t>(nu) * nr, 0.0);
    for (int u = 0; u < nu; ++u) {
        int I = u, J = u;
        if (u >= nb) {
            int r = nb;
            for (int a = 0; a < nb; ++a)
                for (int c = a + 1; c < nb; ++c, ++r)
                    if (r == u) {
                        I = a;
                        J = c;
                    }
        }
        for (int j = 0; j < nb; ++j)
            for (int jj = 0; jj < nb; ++jj) {
                E3 e(dim);
                for (int k = 0; k < dim; ++k) e[k] = space[j][k] + space[jj][k];
                T.prod[u * nr + row_of(e)] += Cinv[j * nb + I] * Cinv[jj * nb + J];
            }
    }
    T.psi.assign(static_cast<size_t>(nb) * qs, 0.0);
    for (int J = 0; J < nb; ++J)
        for (int b = 0; b < nq; ++b) {
            double v = 0.0;
            for (int j = 0; j < nb; ++j) v += Cinv[j * nb + J] * mono(space[j], &T.rule[b * dim]);
            T.psi[J * qs + b] = v;
        }
    return T;
}

// Kernel constant C.  eta = 1: C_{delta,eps} of Section 6 (kappa = 1).  Gaussian
// eta: c such that c * omega_N * int_0^{delta+eps} rho^{N+1} eta mu drho = N
// (L_eps u = Laplacian u for quadratic u), 40 Gauss-Legendre points on each
// smooth piece [0, delta-eps] and [delta-eps, delta+eps].
double kernel_constant(int dim, int kernel, double delta, double eps)
{
    const double pi = 3.14159265358979323846;
    if (kernel == NLQ_ETA_CONST) {
        const double q2 = (eps / delta) * (eps / delta);
        if (dim == 2)
            return (4.0 / (pi * std::pow(delta, 4))) / (1.0 + q2 * (6.0 / 11.0 + q2 * (3.0 / 143.0)));
        return (15.0 / (4.0 * pi * std::pow(delta, 5))) /
               (1.0 + q2 * (10.0 / 11.0 + q2 * (15.0 / 143.0)));
    }
    std::vector<double> gx, gw;
    legendre_rule(40, gx, gw);
    const double omega = (dim == 2) ? 2.0 * pi : 4.0 * pi;
    double moment = 0.0;
    const double a[2] = {0.0, delta - eps}, b[2] = {delta - eps, delta + eps};
    for (int piece = 0; piece < 2; ++piece) {
        const double half = 0.5 * (b[piece] - a[piece]), mid = 0.5 * (b[piece] + a[piece]);
        for (size_t i = 0; i < gx.size(); ++i) {
            double rho = mid + half * gx[i];
            double m = (rho < delta - eps) ? 1.0 : (rho > delta + eps ? 0.0 : xi_host((delta - rho) / eps));
            moment += half * gw[i] * std::pow(rho, dim + 1) * std::exp(-(rho * rho) / (delta * delta)) * m;
        }
    }
    return dim / (omega * moment);
}

std::unique_ptr<Tables> make_tables(Ctx *ctx, int dim, int lmax)
{
    auto t = std::make_unique<Tables>();
    t->dim = dim;
    t->lmax = lmax;
    t->nv = dim + 1;
    simplex_rule(dim, t->bary, t->w);
    t->nq = static_cast<int>(t->w.size());
    const int nv = t->nv, nq = t->nq, nch = 1 << dim;
    t->lvl_off.assign(lmax + 2, 0);
    int64_t per_level = 1;
    for (int lev = 1; lev <= lmax; ++lev) {
        t->lvl_off[lev + 1] = t->lvl_off[lev] + per_level;
        per_level *= nch;
    }
    t->n_sub = t->lvl_off[lmax + 1];
    std::vector<double> lam(static_cast<size_t>(t->n_sub) * nq * nv);
    std::vector<float> lam32(lam.size());
    // barycentric vertices of every sub-element, level by level
    std::vector<double> cur(nv * nv, 0.0), next;
    for (int i = 0; i < nv; ++i) cur[i * nv + i] = 1.0;
    for (int lev = 1; lev <= lmax; ++lev) {
        const int64_t count = t->lvl_off[lev + 1] - t->lvl_off[lev];
        for (int64_t c = 0; c < count; ++c) {
            const double *V = &cur[static_cast<size_t>(c) * nv * nv];
            double *out = &lam[static_cast<size_t>(t->lvl_off[lev] + c) * nq * nv];
            for (int a = 0; a < nq; ++a)
                for (int i = 0; i < nv; ++i) {
                    double s = 0.0;
                    for (int v = 0; v < nv; ++v) s += t->bary[a * nv + v] * V[v * nv + i];
                    out[a * nv + i] = s;
                }
        }
        if (lev == lmax) break;
        next.assign(static_cast<size_t>(count) * nch * nv * nv, 0.0);
        for (int64_t c = 0; c < count; ++c)
            for (int ch = 0; ch < nch; ++ch)
                refine_child(dim, nv, &cur[static_cast<size_t>(c) * nv * nv], ch,
                             &next[(static_cast<size_t>(c) * nch + ch) * nv * nv]);
        cur.swap(next);
    }
    for (size_t k = 0; k < lam.size(); ++k) lam32[k] = static_cast<float>(lam[k]);
    {
        // the same FP32 operations as forming the rows point by point: w scaled
        // by 2^-dim(level-1) exactly, then products rounded one at a time
        const int stride = dim == 2 ? 8 : 16, nr = nv * (nv + 1) / 2;
        std::vector<float> pt(static_cast<size_t>(t->n_sub * nq + 1) * stride, 0.0f);
        for (int lev = 1; lev <= lmax; ++lev)
            for (int64_t sub = t->lvl_off[lev]; sub < t->lvl_off[lev + 1]; ++sub)
                for (int a = 0; a < nq; ++a) {
                    const float *l = &lam32[(static_cast<size_t>(sub) * nq + a) * nv];
                    float *o = &pt[(static_cast<size_t>(sub) * nq + a) * stride];
                    const float w = std::ldexp(static_cast<float>(t->w[a]), -dim * (lev - 1));
                    for (int i = 0; i < nv; ++i) o[i] = w * l[i];
                    int r = nv;
                    for (int i = 0; i < nv; ++i)
                        for (int j = i + 1; j < nv; ++j) o[r++] = o[i] * l[j];
                    for (int i = 1; i < nv; ++i) o[nr + i - 1] = l[i];
                }
        t->pt32.alloc(ctx, pt.size() * sizeof(float));
        NLQ_HIP(hipMemcpy(t->pt32.as<void>(), pt.data(), pt.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    std::vector<double> rule(t->bary);
    rule.insert(rule.end(), t->w.begin(), t->w.end());
    t->rule.alloc(ctx, rule.size() * sizeof(double));
    NLQ_HIP(hipMemcpy(t->rule.as<void>(), rule.data(), rule.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    t->lam64.alloc(ctx, lam.size() * sizeof(double));
    NLQ_HIP(hipMemcpy(t->lam64.as<void>(), lam.data(), lam.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    const std::vector<double> p2 = make_p2_map(dim);
    t->p2map.alloc(ctx, p2.size() * sizeof(double));
    NLQ_HIP(hipMemcpy(t->p2map.as<void>(), p2.data(), p2.size() * sizeof(double), hipMemcpyHostToDevice));
    auto upload = [&](DevBuf &b, const std::vector<double> &v) {
        b.alloc(ctx, v.size() * sizeof(double));
        NLQ_HIP(hipMemcpy(b.as<void>(), v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    };
    for (int order = 1; order <= 2; ++order) {
        const BoxTablesHost bt = make_box_tables(dim, order);
        if (order == 1) upload(t->boxrule, bt.rule);
        upload(t->boxpsi[order - 1], bt.psi);
        upload(t->boxphi[order - 1], bt.phi);
        upload(t->boxprod[order - 1], bt.prod);
    }
    return t;
}

const Tables &Ctx::get_tables(int dim, int lmax)
{
    std::lock_guard<std::mutex> g(tables_mu);
    auto key = std::make_pair(dim, lmax);
    auto it = tables.find(key);
    if (it != tables.end()) return *it->second;
    NLQ_HIP(hipSetDevice(device));
    auto t = make_tables(this, dim, lmax);
    const Tables &ref = *t;
    tables.emplace(key, std::move(t));
    return ref;
}

}  // namespace nlq
