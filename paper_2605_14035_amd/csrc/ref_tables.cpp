// Reference-element tables: quadrature rules in closed form and the nodal
// Lagrange basis evaluated at their points (the precompute step of the
// paper's assembly functions, section 5.2, and Listing 1 (a)).
//
// Rules (weights sum to the reference measure: 1, 1/2, 1/6):
//   segment      Gauss-Legendre with 2 points (degree 3) and 3 points (degree 5)
//                in closed form; 5 and 6 points (degree 9, 11): the roots of
//                the Legendre polynomial by Newton's method on its three-term
//                recurrence, weights 2 / ((1 - t^2) P_n'(t)^2), mapped to [0, 1]
//   triangle     3 points, degree 2: barycentric orbit of (2/3, 1/6, 1/6)
//                6 points, degree 4: two orbits (a, a, 1-2a) with
//                a = (8 - sqrt10 +- sqrt(38 - 44 sqrt(2/5))) / 18,
//                weights (620 +- sqrt(213125 - 53320 sqrt10)) / 3720, times 1/2
//                16 points, degree 8 (the high-order rule of sections 3.2.2, 5.2): the
//                centroid, three orbits (a, a, 1-2a) and one orbit of six
//                permutations (a, b, 1-a-b); Dunavant's published values to
//                15 digits (area-one weights, times 1/2)
//   tetrahedron  4 points, degree 2: orbit (a,a,a,1-3a), a = (5 - sqrt5)/20
//                11 points, degree 4: centroid (-148/1875), orbit (1/14 x3, 11/14)
//                (343/7500), orbit (a, a, 1/2-a, 1/2-a), a = (1 + sqrt(5/14))/4
//                (56/375); volume-one weights, times 1/6
//                35 points, degree 7 (the degree of the paper's tetrahedral rule,
//                section 5.2): the centroid, one orbit (a,a,a,1-3a), one orbit
//                (a,a,1/2-a,1/2-a) and two orbits of twelve (a,a,b,1-2a-b), all
//                weights positive and all points inside; the eleven weights and
//                parameters are the root of the moment equations described at
//                solve_tet35, found by Newton's method from a six-digit start
// Basis, in barycentric coordinates l_0 = 1 - sum xi, l_i = xi_i: P1 l_i;
// P2 corners l_i (2 l_i - 1), edge nodes 4 l_i l_j with the edge order
// segment (0,1); triangle (0,1), (1,2), (2,0); tetrahedron (0,1), (1,2),
// (0,2), (0,3), (1,3), (2,3).  Orders 3 and 4 on segments and triangles (the
// paper notes that its assembly extends to degree 3 and up, section 1, and its
// mesh utility builds orders 2 to 4, section 5.4): the lattice basis described
// at eval_lattice below; they default to the high-order rules.
#include <algorithm>
#include <array>
#include <cmath>

#include "lfem_internal.hpp"

namespace lfem {

namespace {

struct Rule {
    std::vector<std::vector<double>> pts;  // reference coordinates
    std::vector<double> w;
};

void add_bary(Rule &r, std::initializer_list<double> lam, double w)
{
    std::vector<double> l(lam);
    r.pts.emplace_back(l.begin() + 1, l.end());
    r.w.push_back(w);
}

// n-point Gauss-Legendre rule on [0, 1]
void gauss_legendre(int n, Rule &r)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double t = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            // P_n(t) and P_n'(t) from (j+1) P_{j+1} = (2j+1) t P_j - j P_{j-1}
            double p0 = 1.0, p1 = t;
            for (int j = 1; j < n; ++j) {
                const double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        r.pts.push_back({0.5 * (1.0 + t)});
        r.w.push_back(1.0 / ((1.0 - t * t) * dp * dp));
    }
}

void add_orbit21(Rule &r, double a, double w)
{
    const double b = 1.0 - 2.0 * a;
    add_bary(r, {b, a, a}, w);
    add_bary(r, {a, b, a}, w);
    add_bary(r, {a, a, b}, w);
}

void add_orbit111(Rule &r, double a, double b, double w)
{
    const double c = 1.0 - a - b;
    add_bary(r, {a, b, c}, w);
    add_bary(r, {a, c, b}, w);
    add_bary(r, {b, a, c}, w);
    add_bary(r, {b, c, a}, w);
    add_bary(r, {c, a, b}, w);
    add_bary(r, {c, b, a}, w);
}

// Symmetric tetrahedral rule of degree 7 with 35 points.  Unknowns x: weights
// and orbit parameters, in the order centroid (w), (a,a,a,1-3a) (w, a),
// (a,a,1/2-a,1/2-a) (w, a), (a,a,b,1-2a-b) twice (w, a, b).  Equations: for
// each exponent vector e = (e0 >= e1 >= e2 >= e3), |e| = 7 (eleven of them),
// the full symmetrisation P_e(l) = sum over the 24 permutations s of
// prod_i l_s(i)^e_i is integrated exactly; its exact integral over the
// reference tetrahedron (volume 1/6) is 24 prod_i e_i! / 10!.  With
// l0 + l1 + l2 + l3 = 1 the P_e span every symmetric polynomial of degree at
// most 7, and a rule invariant under the permutations of the vertices that
// integrates those exactly integrates every polynomial of degree 7 exactly.
constexpr int kT35Orbits = 5;
constexpr int kT35Size[kT35Orbits] = {1, 4, 6, 12, 12};
constexpr int kT35Par[kT35Orbits] = {0, 1, 1, 2, 2};

void t35_rep(int o, const double *par, double l[4])
{
    switch (o) {
    case 0: l[0] = l[1] = l[2] = l[3] = 0.25; break;
    case 1: l[0] = 1.0 - 3.0 * par[0]; l[1] = l[2] = l[3] = par[0]; break;
    case 2: l[0] = l[1] = par[0]; l[2] = l[3] = 0.5 - par[0]; break;
    default: l[0] = l[1] = par[0]; l[2] = par[1]; l[3] = 1.0 - 2.0 * par[0] - par[1]; break;
    }
}

void t35_residual(const double *x, const int (*ex)[4], int ne, double *res)
{
    static const int perm[24][4] = {
        {0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1},
        {1, 0, 2, 3}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0},
        {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {2, 3, 1, 0},
        {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};
    for (int i = 0; i < ne; ++i) {
        double exact = 24.0;
        for (int j = 0; j < 4; ++j)
            for (int f = 2; f <= ex[i][j]; ++f) exact *= f;
        for (int f = 2; f <= 10; ++f) exact /= f;
        double sum = 0.0;
        int at = 0;
        for (int o = 0; o < kT35Orbits; ++o) {
            const double w = x[at];
            double l[4];
            t35_rep(o, x + at + 1, l);
            at += 1 + kT35Par[o];
            double pe = 0.0;
            for (const auto &s : perm) {
                double t = 1.0;
                for (int j = 0; j < 4; ++j)
                    for (int c = 0; c < ex[i][j]; ++c) t *= l[s[j]];
                pe += t;
            }
            sum += kT35Size[o] * w * pe;
        }
        res[i] = sum / exact - 1.0;
    }
}

bool solve_tet35(Rule &r)
{
    constexpr int n = 11;
    int ex[n][4], ne = 0;
    for (int a = 7; a >= 0; --a)
        for (int b = std::min(a, 7 - a); b >= 0; --b)
            for (int c = std::min(b, 7 - a - b); c >= 0; --c) {
                const int d = 7 - a - b - c;
                if (d < 0 || d > c) continue;
                if (ne == n) return false;
                ex[ne][0] = a, ex[ne][1] = b, ex[ne][2] = c, ex[ne][3] = d;
                ++ne;
            }
    if (ne != n) return false;
    double x[n] = {0.0159142, 0.00705493, 0.315701, 0.00531615, 0.449510, 0.00135180,
                   0.0212655, 0.146639,   0.00620119, 0.188834, 0.0471607};
    double f[n], J[n][n + 1];
    for (int it = 0; it < 8; ++it) {
        t35_residual(x, ex, n, f);
        for (int j = 0; j < n; ++j) {  // central differences
            const double h = 1e-6 * std::max(std::fabs(x[j]), 1e-3);
            double xp[n], xm[n], fp[n], fm[n];
            std::copy(x, x + n, xp);
            std::copy(x, x + n, xm);
            xp[j] += h;
            xm[j] -= h;
            t35_residual(xp, ex, n, fp);
            t35_residual(xm, ex, n, fm);
            for (int i = 0; i < n; ++i) J[i][j] = (fp[i] - fm[i]) / (2.0 * h);
        }
        for (int i = 0; i < n; ++i) J[i][n] = -f[i];
        for (int c = 0; c < n; ++c) {  // Gaussian elimination, partial pivoting
            int piv = c;
            for (int i = c + 1; i < n; ++i)
                if (std::fabs(J[i][c]) > std::fabs(J[piv][c])) piv = i;
            if (J[piv][c] == 0.0) return false;
            for (int j = 0; j <= n; ++j) std::swap(J[c][j], J[piv][j]);
            for (int i = c + 1; i < n; ++i) {
                const double m = J[i][c] / J[c][c];
                for (int j = c; j <= n; ++j) J[i][j] -= m * J[c][j];
            }
        }
        for (int c = n - 1; c >= 0; --c) {
            double v = J[c][n];
            for (int j = c + 1; j < n; ++j) v -= J[c][j] * J[j][n];
            J[c][n] = v / J[c][c];
        }
        for (int j = 0; j < n; ++j) x[j] += J[j][n];
    }
    t35_residual(x, ex, n, f);
    for (int i = 0; i < n; ++i)
        if (!(std::fabs(f[i]) < 1e-13)) return false;
    int at = 0;
    for (int o = 0; o < kT35Orbits; ++o) {
        const double w = x[at];
        double l[4];
        t35_rep(o, x + at + 1, l);
        at += 1 + kT35Par[o];
        if (!(w > 0.0) || !(std::min(std::min(l[0], l[1]), std::min(l[2], l[3])) > 0.0)) return false;
        // the distinct permutations of the representative
        std::vector<std::array<double, 4>> seen;
        int idx[4] = {0, 1, 2, 3};
        do {
            const std::array<double, 4> q = {l[idx[0]], l[idx[1]], l[idx[2]], l[idx[3]]};
            if (std::find(seen.begin(), seen.end(), q) == seen.end()) seen.push_back(q);
        } while (std::next_permutation(idx, idx + 4));
        if (static_cast<int>(seen.size()) != kT35Size[o]) return false;
        for (const auto &q : seen) add_bary(r, {q[0], q[1], q[2], q[3]}, w);
    }
    return true;
}

bool make_rule(int d, int npts, Rule &r)
{
    r = Rule{};
    if (d == 1) {
        if (npts == 5 || npts == 6) {
            gauss_legendre(npts, r);
            return true;
        }
        if (npts == 2) {
            double s = 0.5 / std::sqrt(3.0);
            r.pts = {{0.5 - s}, {0.5 + s}};
            r.w = {0.5, 0.5};
            return true;
        }
        if (npts == 3) {
            double s = 0.5 * std::sqrt(0.6);
            r.pts = {{0.5 - s}, {0.5}, {0.5 + s}};
            r.w = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
            return true;
        }
        return false;
    }
    if (d == 2) {
        if (npts == 3) {
            const double a = 1.0 / 6.0, b = 2.0 / 3.0, w = 1.0 / 6.0;
            add_bary(r, {b, a, a}, w);
            add_bary(r, {a, b, a}, w);
            add_bary(r, {a, a, b}, w);
            return true;
        }
        if (npts == 6) {
            const double s10 = std::sqrt(10.0);
            const double root = std::sqrt(38.0 - 44.0 * std::sqrt(0.4));
            const double wroot = std::sqrt(213125.0 - 53320.0 * s10);
            const double a[2] = {(8.0 - s10 + root) / 18.0, (8.0 - s10 - root) / 18.0};
            const double w[2] = {(620.0 + wroot) / 3720.0 * 0.5, (620.0 - wroot) / 3720.0 * 0.5};
            for (int o = 0; o < 2; ++o) add_orbit21(r, a[o], w[o]);
            return true;
        }
        if (npts == 16) {
            add_bary(r, {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0}, 0.5 * 0.144315607677787);
            add_orbit21(r, 0.459292588292723, 0.5 * 0.095091634267285);
            add_orbit21(r, 0.170569307751760, 0.5 * 0.103217370534718);
            add_orbit21(r, 0.050547228317031, 0.5 * 0.032458497623198);
            add_orbit111(r, 0.008394777409958, 0.263112829634638, 0.5 * 0.027230314174435);
            return true;
        }
        return false;
    }
    if (d == 3) {
        if (npts == 4) {
            const double a = (5.0 - std::sqrt(5.0)) / 20.0, b = 1.0 - 3.0 * a, w = 1.0 / 24.0;
            add_bary(r, {b, a, a, a}, w);
            add_bary(r, {a, b, a, a}, w);
            add_bary(r, {a, a, b, a}, w);
            add_bary(r, {a, a, a, b}, w);
            return true;
        }
        if (npts == 11) {
            add_bary(r, {0.25, 0.25, 0.25, 0.25}, -148.0 / 1875.0 / 6.0);
            const double a1 = 1.0 / 14.0, b1 = 11.0 / 14.0, w1 = 343.0 / 7500.0 / 6.0;
            add_bary(r, {b1, a1, a1, a1}, w1);
            add_bary(r, {a1, b1, a1, a1}, w1);
            add_bary(r, {a1, a1, b1, a1}, w1);
            add_bary(r, {a1, a1, a1, b1}, w1);
            const double a2 = 0.25 * (1.0 + std::sqrt(5.0 / 14.0));
            const double b2 = 0.5 - a2, w2 = 56.0 / 375.0 / 6.0;
            for (int i = 0; i < 4; ++i)
                for (int j = i + 1; j < 4; ++j) {
                    double l[4] = {b2, b2, b2, b2};
                    l[i] = a2;
                    l[j] = a2;
                    add_bary(r, {l[0], l[1], l[2], l[3]}, w2);
                }
            return true;
        }
        if (npts == 35) return solve_tet35(r);
        return false;
    }
    return false;
}

const int EDGE_SEG[1][2] = {{0, 1}};
const int EDGE_TRI[3][2] = {{0, 1}, {1, 2}, {2, 0}};
const int EDGE_TET[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

// Orders 3 and 4: node a is the lattice point alpha / p (|alpha| = p),
// ordered vertices, then p - 1 nodes per edge (u, v) of the edge list from u
// to v, then on a tetrahedron the nodes inside its faces (0,1,2), (0,1,3),
// (0,2,3), (1,2,3) (p = 3: the face centroid; p = 4: (2,1,1), (1,2,1),
// (1,1,2) over the face's vertices), then the interior nodes (triangle:
// p = 3 (1,1,1), p = 4 (2,1,1), (1,2,1), (1,1,2); tetrahedron, p = 4:
// (1,1,1,1)); its Lagrange function is
//   phi_alpha(l) = prod_j prod_{r < alpha_j} (p l_j - r) / (r + 1).
const int FACE_TET[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

int lattice_nodes(int d, int p, int (*alpha)[4])
{
    int n = 0;
    for (int i = 0; i <= d; ++i, ++n)
        for (int j = 0; j <= d; ++j) alpha[n][j] = i == j ? p : 0;
    const int ne = d == 1 ? 1 : (d == 2 ? 3 : 6);
    const int(*E)[2] = d == 1 ? EDGE_SEG : (d == 2 ? EDGE_TRI : EDGE_TET);
    for (int s = 0; s < ne; ++s)
        for (int i = 1; i < p; ++i, ++n) {
            for (int j = 0; j <= d; ++j) alpha[n][j] = 0;
            alpha[n][E[s][0]] = p - i;
            alpha[n][E[s][1]] = i;
        }
    if (d == 2) {
        const int interior = p == 3 ? 1 : 3;
        for (int c = 0; c < interior; ++c, ++n) {
            alpha[n][0] = alpha[n][1] = alpha[n][2] = 1;
            if (p == 4) alpha[n][c] = 2;
        }
    }
    if (d == 3) {
        const int per_face = p == 3 ? 1 : 3;
        for (int f = 0; f < 4; ++f)
            for (int c = 0; c < per_face; ++c, ++n) {
                for (int j = 0; j <= d; ++j) alpha[n][j] = 0;
                for (int v = 0; v < 3; ++v) alpha[n][FACE_TET[f][v]] = 1;
                if (p == 4) alpha[n][FACE_TET[f][c]] = 2;
            }
        if (p == 4) {
            alpha[n][0] = alpha[n][1] = alpha[n][2] = alpha[n][3] = 1;
            ++n;
        }
    }
    return n;
}

void eval_lattice(int d, int p, const double *l, const double (*dl)[3], double *phi, double *g)
{
    int alpha[35][4];
    const int k = lattice_nodes(d, p, alpha);
    for (int a = 0; a < k; ++a) {
        double f[4], df[4];
        for (int j = 0; j <= d; ++j) {
            // f_j = prod_{r < alpha_j} (p l_j - r) / (r + 1) and its l_j-derivative
            double v = 1.0, dv = 0.0;
            for (int r = 0; r < alpha[a][j]; ++r) {
                const double t = (p * l[j] - r) / (r + 1);
                dv = dv * t + v * p / (r + 1);
                v *= t;
            }
            f[j] = v;
            df[j] = dv;
        }
        double val = 1.0;
        for (int j = 0; j <= d; ++j) val *= f[j];
        phi[a] = val;
        for (int m = 0; m < d; ++m) {
            double s = 0.0;
            for (int j = 0; j <= d; ++j) {
                double rest = df[j] * dl[j][m];
                for (int i = 0; i <= d; ++i)
                    if (i != j) rest *= f[i];
                s += rest;
            }
            g[a * d + m] = s;
        }
    }
}

// values phi[k] and reference gradients g[k][d] at xi
void eval_basis(int d, int p, const double *xi, double *phi, double *g)
{
    double l[4];
    double dl[4][3] = {};
    l[0] = 1.0;
    for (int m = 0; m < d; ++m) {
        l[0] -= xi[m];
        dl[0][m] = -1.0;
        l[m + 1] = xi[m];
        dl[m + 1][m] = 1.0;
    }
    if (p >= 3) {
        eval_lattice(d, p, l, dl, phi, g);
        return;
    }
    const int nc = d + 1;
    for (int i = 0; i < nc; ++i) {
        if (p == 1) {
            phi[i] = l[i];
            for (int m = 0; m < d; ++m) g[i * d + m] = dl[i][m];
        } else {
            phi[i] = l[i] * (2.0 * l[i] - 1.0);
            for (int m = 0; m < d; ++m) g[i * d + m] = (4.0 * l[i] - 1.0) * dl[i][m];
        }
    }
    if (p == 2) {
        const int ne = d == 1 ? 1 : (d == 2 ? 3 : 6);
        const int(*E)[2] = d == 1 ? EDGE_SEG : (d == 2 ? EDGE_TRI : EDGE_TET);
        for (int s = 0; s < ne; ++s) {
            const int i = E[s][0], j = E[s][1], r = nc + s;
            phi[r] = 4.0 * l[i] * l[j];
            for (int m = 0; m < d; ++m) g[r * d + m] = 4.0 * (dl[i][m] * l[j] + l[i] * dl[j][m]);
        }
    }
}

}  // namespace

int default_rule(int d, int p)
{
    if (d == 1) return p == 1 ? 2 : (p == 2 ? 3 : (p == 3 ? 5 : 6));
    if (d == 2) return p == 1 ? 3 : (p == 2 ? 6 : 16);
    return p == 1 ? 4 : (p == 2 ? 11 : 35);
}

bool build_ref_table(int d, int p, int npts, RefTable &out)
{
    if (npts == 0) npts = default_rule(d, p);
    Rule r;
    if (!make_rule(d, npts, r)) return false;
    const int k = nodes_per_elem(d, p), np = k * (k + 1) / 2;
    out.Q = npts;
    out.k = k;
    out.d = d;
    const int nsym = d * (d + 1) / 2;
    out.stride = 1 + d + k + k * d + np + np * nsym;
    out.data.assign(static_cast<size_t>(out.stride) * npts, 0.0);
    for (int q = 0; q < npts; ++q) {
        double *t = out.data.data() + static_cast<size_t>(q) * out.stride;
        double phi[35], g[105];
        eval_basis(d, p, r.pts[q].data(), phi, g);
        t[0] = r.w[q];
        for (int m = 0; m < d; ++m) t[1 + m] = r.pts[q][m];
        for (int a = 0; a < k; ++a) t[1 + d + a] = phi[a];
        for (int i = 0; i < k * d; ++i) t[1 + d + k + i] = g[i];
        int pi = 0;
        for (int a = 0; a < k; ++a)
            for (int b = a; b < k; ++b) t[1 + d + k + k * d + pi++] = phi[a] * phi[b];
        // reference stiffness tensor R[p][s], s over (m <= n)
        double *R = t + 1 + d + k + k * d + np;
        pi = 0;
        for (int a = 0; a < k; ++a)
            for (int b = a; b < k; ++b, ++pi) {
                int si = 0;
                for (int m = 0; m < d; ++m)
                    for (int n = m; n < d; ++n, ++si)
                        R[pi * nsym + si] = m == n ? g[a * d + m] * g[b * d + m]
                                                   : g[a * d + m] * g[b * d + n] + g[a * d + n] * g[b * d + m];
            }
    }
    out.pstride = npts * (1 + nsym);
    out.pairs.assign(static_cast<size_t>(out.pstride) * np, 0.0);
    for (int pi = 0; pi < np; ++pi)
        for (int q = 0; q < npts; ++q) {
            const double *t = out.data.data() + static_cast<size_t>(q) * out.stride;
            double *dst = out.pairs.data() + static_cast<size_t>(pi) * out.pstride;
            dst[q] = t[1 + d + k + k * d + pi];
            for (int si = 0; si < nsym; ++si)
                dst[npts + q * nsym + si] = t[1 + d + k + k * d + np + pi * nsym + si];
        }
    return true;
}

}  // namespace lfem
