// Problem builder for the structured workloads: Kuhn-tetrahedral fine mesh of the unit
// cube, lowest-order Nedelec / Raviart-Thomas matrices (eq. (2.2)), and the AMGe
// hierarchy of section 3 for 2x2x2 agglomerates.
//
// Every agglomerate of a level is a translate of the same 2x2x2 block (uniform Kuhn
// mesh), so the local problems of section 3.3 are solved once per level on a reference
// block and the resulting local prolongators are placed at every agglomerate.  With
// coefficient-aware extensions (the remark closing section 3.3: the system space's
// element masses weighted by beta, the next space's by alpha) an agglomerate whose cells
// carry different weights solves its own block; one whose cells share a weight keeps
// the reference solution (scaling a local problem's mass does not move its minimiser).
// Shared rows receive identical values from both sides ("overwriting" assembly,
// section 2.2 footnote): face values come from face problems, which no cell weight
// enters.  With essential boundary conditions every level keeps only the entities off
// the boundary of the cube.
//
// Local extension problems (eqs. (3.6), (3.8)): minimise the L2 norm of the extension
// subject to the derivative constraint on the entity's interior, with the trace on its
// boundary fixed.  Solved by the null-space method with a pivoted Householder QR of the
// constraint (particular solution on its range, mass minimised over its null space).
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <chrono>
#include <cstdlib>
#include <string>

#include "common.hpp"
#include "setup_device.hpp"
#include "spgemm_device.hpp"

namespace amge {
namespace {

// ------------------------------------------------------------------ small dense algebra
struct Mat {
    int r = 0, c = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
    double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

Mat matmul(const Mat& A, const Mat& B) {
    Mat C(A.r, B.c);
    for (int i = 0; i < A.r; ++i)
        for (int k = 0; k < A.c; ++k) {
            double v = A(i, k);
            if (v == 0) continue;
            for (int j = 0; j < B.c; ++j) C(i, j) += v * B(k, j);
        }
    return C;
}

Mat tmatmul(const Mat& A, const Mat& B) {  // A^T B
    Mat C(A.c, B.c);
    for (int k = 0; k < A.r; ++k)
        for (int i = 0; i < A.c; ++i) {
            double v = A(k, i);
            if (v == 0) continue;
            for (int j = 0; j < B.c; ++j) C(i, j) += v * B(k, j);
        }
    return C;
}

// In-place Cholesky (lower), returns false if not positive definite.
bool cholesky(Mat& L) {
    int n = L.r;
    for (int j = 0; j < n; ++j) {
        double d = L(j, j);
        for (int k = 0; k < j; ++k) d -= L(j, k) * L(j, k);
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        L(j, j) = d;
        for (int i = j + 1; i < n; ++i) {
            double s = L(i, j);
            for (int k = 0; k < j; ++k) s -= L(i, k) * L(j, k);
            L(i, j) = s / d;
        }
        for (int k = j + 1; k < n; ++k) L(j, k) = 0.0;
    }
    return true;
}

// Solve L L^T X = B in place (B: n x m).
void chol_solve(const Mat& L, Mat& B) {
    int n = L.r;
    for (int col = 0; col < B.c; ++col) {
        for (int i = 0; i < n; ++i) {
            double s = B(i, col);
            for (int k = 0; k < i; ++k) s -= L(i, k) * B(k, col);
            B(i, col) = s / L(i, i);
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = B(i, col);
            for (int k = i + 1; k < n; ++k) s -= L(k, i) * B(k, col);
            B(i, col) = s / L(i, i);
        }
    }
}

// Householder QR with column pivoting of an r x c matrix A (in place): A P = Q R.
// On return A holds R in its upper triangle, Qf the r x r orthogonal factor, piv the
// column order, and the rank is the number of diagonal entries of R above
// tol * |R(0, 0)|.
int qr_pivoted(Mat& A, Mat& Qf, std::vector<int>& piv, double tol) {
    const int r = A.r, c = A.c, kmax = std::min(r, c);
    piv.resize(c);
    for (int j = 0; j < c; ++j) piv[j] = j;
    Qf = Mat(r, r);
    for (int i = 0; i < r; ++i) Qf(i, i) = 1.0;
    std::vector<double> v(r);
    double r00 = 0;
    int rank = 0;
    for (int k = 0; k < kmax; ++k) {
        // the remaining column of largest norm
        int best = -1;
        double bn = -1;
        for (int j = k; j < c; ++j) {
            double s = 0;
            for (int i = k; i < r; ++i) s += A(i, j) * A(i, j);
            if (s > bn) { bn = s; best = j; }
        }
        bn = std::sqrt(bn);
        if (k == 0) r00 = bn;
        if (!(bn > tol * r00) || bn == 0) break;
        if (best != k) {
            for (int i = 0; i < r; ++i) std::swap(A(i, k), A(i, best));
            std::swap(piv[k], piv[best]);
        }
        // reflector H = I - 2 v v^T / (v^T v) mapping A(k:, k) to -sign(a_kk) |.| e_k
        const double alpha = A(k, k) >= 0 ? -bn : bn;
        double vv = 0;
        for (int i = k; i < r; ++i) {
            v[i] = A(i, k) - (i == k ? alpha : 0.0);
            vv += v[i] * v[i];
        }
        if (vv > 0) {
            for (int j = k; j < c; ++j) {
                double d = 0;
                for (int i = k; i < r; ++i) d += v[i] * A(i, j);
                d = 2 * d / vv;
                for (int i = k; i < r; ++i) A(i, j) -= d * v[i];
            }
            for (int j = 0; j < r; ++j) {   // Qf <- Qf H (Qf accumulates the reflectors)
                double d = 0;
                for (int i = k; i < r; ++i) d += Qf(j, i) * v[i];
                d = 2 * d / vv;
                for (int i = k; i < r; ++i) Qf(j, i) -= d * v[i];
            }
        }
        ++rank;
    }
    return rank;
}

// Null space of a constraint block K_I (m x nI): pivoted Householder QR K_I^T P = Q R.
// The constraint K_I u = g reads R^T (Q^T u) = P^T g: its first `rk` rows fix the part
// y1 of y = Q^T u on the range (a triangular solve), the rest of y spans the null space
// Q2 = Q(:, rk:).
struct NullSpace {
    int nI = 0, m = 0, rk = 0;
    Mat R, Qf;
    std::vector<int> piv;
    explicit NullSpace(const Mat& KI) : nI(KI.c), m(KI.r), R(KI.c, KI.r) {
        for (int i = 0; i < m; ++i)
            for (int a = 0; a < nI; ++a) R(a, i) = KI(i, a);
        rk = qr_pivoted(R, Qf, piv, 1e-12);
    }
    // Q1 y1 with R11^T y1 = (P^T G)(0:rk): the particular solution of minimal norm for
    // the right-hand sides G (m x t)
    Mat particular(const Mat& G) const {
        Mat Y1(rk, G.c);
        for (int t = 0; t < G.c; ++t)
            for (int i = 0; i < rk; ++i) {
                double s = G(piv[i], t);
                for (int l = 0; l < i; ++l) s -= R(l, i) * Y1(l, t);
                Y1(i, t) = s / R(i, i);
            }
        Mat U(nI, G.c);
        for (int a = 0; a < nI; ++a)
            for (int t = 0; t < G.c; ++t) {
                double s = 0;
                for (int i = 0; i < rk; ++i) s += Qf(a, i) * Y1(i, t);
                U(a, t) = s;
            }
        return U;
    }
    Mat Q2() const {
        Mat Z(nI, nI - rk);
        for (int a = 0; a < nI; ++a)
            for (int j = 0; j < nI - rk; ++j) Z(a, j) = Qf(a, rk + j);
        return Z;
    }
};

// Interior / boundary split of a local problem: K_I, and G = S - K_B u_B.
void split_constraint(const Mat& K, const std::vector<char>& intr, const Mat& S, const Mat& UB, std::vector<int>& I,
                      std::vector<int>& B, Mat& KI, Mat& G) {
    const int nd = K.c, m = K.r, nrhs = S.c;
    I.clear();
    B.clear();
    for (int j = 0; j < nd; ++j) (intr[j] ? I : B).push_back(j);
    KI = Mat(m, (int)I.size());
    G = Mat(m, nrhs);
    for (int i = 0; i < m; ++i) {
        for (size_t a = 0; a < I.size(); ++a) KI(i, (int)a) = K(i, I[a]);
        for (int t = 0; t < nrhs; ++t) {
            double v = S(i, t);
            for (size_t b = 0; b < B.size(); ++b) v -= K(i, B[b]) * UB((int)b, t);
            G(i, t) = v;
        }
    }
}

// Every constraint row (the dependent ones too) must hold for the extension U.
void check_consistent(const Mat& KI, const Mat& G, const Mat& U) {
    double res = 0, gn = 0;
    for (int i = 0; i < KI.r; ++i)
        for (int t = 0; t < G.c; ++t) {
            double v = -G(i, t);
            for (int a = 0; a < KI.c; ++a) v += KI(i, a) * U(a, t);
            res = std::max(res, std::fabs(v));
            gn = std::max(gn, std::fabs(G(i, t)));
        }
    if (res > 1e-10 * std::max(1.0, gn)) fail(AMGE_ERR_ARG, "inconsistent extension constraint");
}

// Minimum-mass extension on one entity (eqs. (3.6), (3.8) read as the optimality
// conditions of: minimise the mass of the extension subject to the derivative
// constraint on the entity's interior, its trace on the boundary fixed).
//   M     mass on the entity's closure dofs (nd x nd), or empty if the constraint alone
//         determines the interior values
//   K     constraint rows over the closure dofs (m x nd)
//   intr  interior mask (nd)
//   S     right-hand sides of the constraint (m x nrhs)
//   UB    boundary values (nB x nrhs), in closure order of the non-interior dofs
// Returns U_I (nI x nrhs).  Null-space method: the particular solution on the range of
// K_I^T, then the mass minimised over its null space Q2: (Q2^T M_II Q2) y2 =
// -Q2^T (M_II u_p + M_IB u_B).  The constraint then holds to rounding whatever the
// conditioning of the mass (coefficient-weighted masses).
Mat extend(const Mat& M, const Mat& K, const std::vector<char>& intr, const Mat& S, const Mat& UB) {
    std::vector<int> I, B;
    Mat KI, G;
    split_constraint(K, intr, S, UB, I, B, KI, G);
    const int nI = (int)I.size(), nrhs = S.c;
    NullSpace ns(KI);
    Mat U = ns.particular(G);
    const int nz = nI - ns.rk;
    if (nz > 0) {
        if (M.r == 0) fail(AMGE_ERR_ARG, "extension not determined by its constraint");
        Mat MII(nI, nI), F(nI, nrhs);
        for (int a = 0; a < nI; ++a) {
            for (int b = 0; b < nI; ++b) MII(a, b) = M(I[a], I[b]);
            for (int t = 0; t < nrhs; ++t) {
                double v = 0;
                for (size_t b = 0; b < B.size(); ++b) v += M(I[a], B[b]) * UB((int)b, t);
                for (int b = 0; b < nI; ++b) v += M(I[a], I[b]) * U(b, t);
                F(a, t) = v;   // M_II u_p + M_IB u_B
            }
        }
        Mat Q2 = ns.Q2();
        Mat Red = tmatmul(Q2, matmul(MII, Q2));
        Mat W2 = tmatmul(Q2, F);
        for (double& v : W2.a) v = -v;
        if (!cholesky(Red)) fail(AMGE_ERR_NOT_SPD, "local mass not positive definite on the null space");
        chol_solve(Red, W2);
        Mat Z = matmul(Q2, W2);
        for (int a = 0; a < nI; ++a)
            for (int t = 0; t < nrhs; ++t) U(a, t) += Z(a, t);
    }
    check_consistent(KI, G, U);
    return U;
}

// ------------------------------------------------------------------ geometry
struct V3 {
    double x, y, z;
};
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

const int TE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};   // local edges
const int TF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};       // face opposite vertex i

// Element data of one tetrahedron from its vertex lattice coordinates (ints) and h.
struct Tet {
    double vol;
    V3 x[4], g[4];   // coordinates, barycentric gradients
    double s[4];     // +1 if the face's orientation normal points outward
};

Tet make_tet(const std::array<std::array<int, 3>, 4>& P, double h) {
    Tet t;
    for (int i = 0; i < 4; ++i) t.x[i] = {P[i][0] * h, P[i][1] * h, P[i][2] * h};
    // barycentric gradients from the cofactors of the edge vectors e_a = x_a - x_0
    V3 e1 = t.x[1] - t.x[0], e2 = t.x[2] - t.x[0], e3 = t.x[3] - t.x[0];
    double det = dot(e1, cross(e2, e3));
    t.vol = std::fabs(det) / 6.0;
    t.g[1] = (1.0 / det) * cross(e2, e3);
    t.g[2] = (1.0 / det) * cross(e3, e1);
    t.g[3] = (1.0 / det) * cross(e1, e2);
    t.g[0] = -1.0 * (t.g[1] + t.g[2] + t.g[3]);
    for (int i = 0; i < 4; ++i) {
        const int* f = TF[i];
        V3 nrm = cross(t.x[f[1]] - t.x[f[0]], t.x[f[2]] - t.x[f[0]]);
        t.s[i] = dot(nrm, t.x[f[0]] - t.x[i]) > 0 ? 1.0 : -1.0;
    }
    return t;
}

// Whitney edge mass: w_p = sum_a lambda_a v_{p,a} with v_{p,i} = grad l_j, v_{p,j} = -grad l_i
void nd_mass(const Tet& t, double M[6][6]) {
    V3 v[6][4];
    for (int p = 0; p < 6; ++p) {
        for (int a = 0; a < 4; ++a) v[p][a] = {0, 0, 0};
        v[p][TE[p][0]] = t.g[TE[p][1]];
        v[p][TE[p][1]] = -1.0 * t.g[TE[p][0]];
    }
    for (int p = 0; p < 6; ++p)
        for (int q = 0; q < 6; ++q) {
            double s = 0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) s += dot(v[p][a], v[q][b]) * (a == b ? 2.0 : 1.0);
            M[p][q] = s * t.vol / 20.0;
        }
}

// Curl-curl element matrix, curl w_ij = 2 grad l_i x grad l_j (constant).
void curlcurl(const Tet& t, double K[6][6]) {
    V3 c[6];
    for (int p = 0; p < 6; ++p) c[p] = 2.0 * cross(t.g[TE[p][0]], t.g[TE[p][1]]);
    for (int p = 0; p < 6; ++p)
        for (int q = 0; q < 6; ++q) K[p][q] = t.vol * dot(c[p], c[q]);
}

// Face (RT) mass: w_i = s_i (x - x_i) / (3 vol); integral of (x-a).(x-b) over the tet is
// vol [ (c-a).(c-b) + sum_k |x_k - c|^2 / 20 ] with c the centroid.
void rt_mass(const Tet& t, double M[4][4]) {
    V3 c = 0.25 * (t.x[0] + t.x[1] + t.x[2] + t.x[3]);
    double mom = 0;
    for (int k = 0; k < 4; ++k) mom += dot(t.x[k] - c, t.x[k] - c);
    mom /= 20.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double in = t.vol * (dot(c - t.x[i], c - t.x[j]) + mom);
            M[i][j] = t.s[i] * t.s[j] * in / (9.0 * t.vol * t.vol);
        }
}

// Tangential-trace (2D Whitney edge) mass on a triangle, local edges (01),(02),(12).
void tri_trace_mass(V3 x0, V3 x1, V3 x2, double M[3][3]) {
    V3 e1 = x1 - x0, e2 = x2 - x0;
    V3 n = cross(e1, e2);
    double nn = dot(n, n);
    double area = 0.5 * std::sqrt(nn);
    // in-plane barycentric gradients: grad l_1 = (e2 x n)/|n|^2 ... orthogonal to e2, dot e1 = 1
    V3 g1 = (1.0 / nn) * cross(e2, n);
    V3 g2 = (1.0 / nn) * cross(n, e1);
    V3 g[3] = {-1.0 * (g1 + g2), g1, g2};
    const int E[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    V3 v[3][3];
    for (int p = 0; p < 3; ++p) {
        for (int a = 0; a < 3; ++a) v[p][a] = {0, 0, 0};
        v[p][E[p][0]] = g[E[p][1]];
        v[p][E[p][1]] = -1.0 * g[E[p][0]];
    }
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
            double s = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += dot(v[p][a], v[q][b]) * (a == b ? 2.0 : 1.0);
            M[p][q] = s * area / 12.0;
        }
}

// ------------------------------------------------------------------ Kuhn mesh
// Every edge of the Kuhn triangulation runs from a vertex v to v + d for a nonempty
// 0/1 step d (an axis, a face diagonal or the cube diagonal, always towards increasing
// coordinates), and every triangle is (u, u + s, u + s + t) with s, t nonempty and
// disjoint: the in-plane triangles (|s| = |t| = 1) of the squares and the six interior
// triangles of the cube at u.  An entity exists iff its steps stay inside the grid.
// Entities are numbered in the order of their sorted vertex tuples, so with steps as
// bit masks (x = 1, y = 2, z = 4: the vertex offset grows with the mask) the index is
// the count of entities at lower vertices plus the step's rank among those existing at
// the vertex, in closed form.
namespace kuhn_steps {
// the 12 triangle types (s, s | t) in increasing order
constexpr int NTRI = 12;
constexpr int TRI[NTRI][2] = {{1, 3}, {1, 5}, {1, 7}, {2, 3}, {2, 6}, {2, 7}, {3, 7}, {4, 5}, {4, 6}, {4, 7}, {5, 7}, {6, 7}};
struct Tables {
    int ecnt[8], erank[8][8], fcnt[8], frank[8][8][8];
    Tables() {
        for (int f = 0; f < 8; ++f) {
            int c = 0;
            for (int d = 0; d < 8; ++d) {
                erank[f][d] = -1;
                if (d && (d & ~f) == 0) erank[f][d] = c++;
            }
            ecnt[f] = c;
            c = 0;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) frank[f][a][b] = -1;
            for (auto& tr : TRI)
                if ((tr[1] & ~f) == 0) frank[f][tr[0]][tr[1]] = c++;
            fcnt[f] = c;
        }
    }
};
const Tables& tables() {
    static const Tables t;
    return t;
}
}  // namespace kuhn_steps

struct Kuhn {
    int n = 0;
    int64_t nv = 0;
    std::vector<std::array<int32_t, 2>> E;
    std::vector<std::array<int32_t, 3>> F;
    std::vector<std::array<int32_t, 4>> T;
    std::vector<int64_t> eoff, foff;   // first edge / face with tail vertex v (nv + 1 entries)
    std::vector<std::array<int32_t, 6>> te;
    std::vector<std::array<int32_t, 4>> tf;
    std::vector<std::array<int32_t, 3>> fe;
    std::array<int, 3> coord(int64_t v) const {
        int m = n + 1;
        return {(int)(v % m), (int)((v / m) % m), (int)(v / ((int64_t)m * m))};
    }
    int64_t vid(int i, int j, int k) const { int64_t m = n + 1; return i + m * (j + m * k); }
    // axes along which a step from v stays inside the grid
    int room(int64_t v) const {
        auto c = coord(v);
        return (c[0] < n ? 1 : 0) | (c[1] < n ? 2 : 0) | (c[2] < n ? 4 : 0);
    }
    int64_t step(int d) const {
        int64_t m = n + 1;
        return (d & 1) + ((d >> 1) & 1) * m + ((d >> 2) & 1) * m * m;
    }
    // 0/1 step mask from a to b, -1 if b - a is not such a step
    int mask(int64_t a, int64_t b) const {
        if (a < 0 || b < 0 || a >= nv || b >= nv) return -1;
        auto ca = coord(a), cb = coord(b);
        int d = 0;
        for (int x = 0; x < 3; ++x) {
            const int q = cb[x] - ca[x];
            if (q != 0 && q != 1) return -1;
            d |= q << x;
        }
        return d;
    }
    int32_t edge(int64_t a, int64_t b) const {
        const int d = mask(a, b);
        const int r = d > 0 ? kuhn_steps::tables().erank[room(a)][d] : -1;
        if (r < 0) fail(AMGE_ERR_ARG, "edge not in mesh");
        return (int32_t)(eoff[a] + r);
    }
    int32_t face(int64_t a, int64_t b, int64_t c) const {
        const int s = mask(a, b), st = mask(a, c);
        const int r = s > 0 && st > 0 ? kuhn_steps::tables().frank[room(a)][s][st] : -1;
        if (r < 0) fail(AMGE_ERR_ARG, "face not in mesh");
        return (int32_t)(foff[a] + r);
    }
};

Kuhn build_kuhn(int n) {
    using namespace kuhn_steps;
    const Tables& tb = tables();
    Kuhn K;
    K.n = n;
    const int64_t m = n + 1;
    K.nv = m * m * m;
    if ((double)n * n * n * 6 > 2.0e9) fail(AMGE_ERR_ARG, "mesh too large");
    K.eoff.assign(K.nv + 1, 0);
    K.foff.assign(K.nv + 1, 0);
    for (int64_t v = 0; v < K.nv; ++v) {
        const int f = K.room(v);
        K.eoff[v + 1] = K.eoff[v] + tb.ecnt[f];
        K.foff[v + 1] = K.foff[v] + tb.fcnt[f];
    }
    if (K.eoff[K.nv] > INT32_MAX || K.foff[K.nv] > INT32_MAX) fail(AMGE_ERR_ARG, "mesh too large");
    K.E.resize(K.eoff[K.nv]);
    K.F.resize(K.foff[K.nv]);
    parallel_for(K.nv, [&](int64_t s, int64_t e) {
        for (int64_t v = s; v < e; ++v) {
            const int f = K.room(v);
            for (int d = 1; d < 8; ++d)
                if (tb.erank[f][d] >= 0) K.E[K.eoff[v] + tb.erank[f][d]] = {(int32_t)v, (int32_t)(v + K.step(d))};
            for (auto& tr : TRI)
                if (tb.frank[f][tr[0]][tr[1]] >= 0)
                    K.F[K.foff[v] + tb.frank[f][tr[0]][tr[1]]] = {(int32_t)v, (int32_t)(v + K.step(tr[0])),
                                                                  (int32_t)(v + K.step(tr[1]))};
        }
    });
    // six tetrahedra per cube along the paths base -> base + (1,1,1) adding one axis at a
    // time, in the axis orders below; cubes in increasing base vertex, so the tetrahedra
    // come out in increasing order of their vertex tuples
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int64_t ncube = (int64_t)n * n * n;
    K.T.resize(ncube * 6);
    K.te.resize(K.T.size());
    K.tf.resize(K.T.size());
    parallel_for(ncube, [&](int64_t s, int64_t e) {
        for (int64_t q = s; q < e; ++q) {
            const int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((int64_t)n * n));
            const int64_t base = K.vid(i, j, k);
            for (int p = 0; p < 6; ++p) {
                const int cm[4] = {0, 1 << perms[p][0], (1 << perms[p][0]) | (1 << perms[p][1]), 7};
                int64_t v[4];
                int rm[4];
                for (int a = 0; a < 4; ++a) {
                    v[a] = base + K.step(cm[a]);
                    rm[a] = K.room(v[a]);
                }
                const int64_t t = q * 6 + p;
                K.T[t] = {(int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3]};
                for (int a = 0; a < 6; ++a) {
                    const int x = TE[a][0], y = TE[a][1];
                    K.te[t][a] = (int32_t)(K.eoff[v[x]] + tb.erank[rm[x]][cm[y] ^ cm[x]]);
                }
                for (int a = 0; a < 4; ++a) {
                    const int x = TF[a][0], y = TF[a][1], z = TF[a][2];
                    K.tf[t][a] = (int32_t)(K.foff[v[x]] + tb.frank[rm[x]][cm[y] ^ cm[x]][cm[z] ^ cm[x]]);
                }
            }
        }
    });
    K.fe.resize(K.F.size());
    parallel_for((int64_t)K.F.size(), [&](int64_t s, int64_t e) {
        for (int64_t f = s; f < e; ++f) {
            auto& v = K.F[f];
            K.fe[f] = {K.edge(v[0], v[1]), K.edge(v[0], v[2]), K.edge(v[1], v[2])};
        }
    });
    return K;
}

Tet kuhn_tet(const Kuhn& K, int64_t t, double h) {
    std::array<std::array<int, 3>, 4> P;
    for (int i = 0; i < 4; ++i) P[i] = K.coord(K.T[t][i]);
    return make_tet(P, h);
}

// ------------------------------------------------------------------ cube complex
// Canonical orders: vertices by i + M(j + M k); edges by (tail, head) vertex indices;
// faces by their sorted vertex tuples (for one base vertex: normal z, then y, then x);
// cubes by base vertex.  Edge (p,a) runs along +e_a; face (p,a) has normal +e_a.
struct Cubes {
    int N = 0;
    int64_t M = 0;
    std::vector<int32_t> e0, f0;   // first edge / face index per base vertex
    int32_t nE = 0, nF = 0, nT = 0, nV = 0;
    static bool edge_ok(int N, int p[3], int a) { return p[a] < N; }
    static bool face_ok(int N, int p[3], int a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        return p[b] < N && p[c] < N;
    }
    explicit Cubes(int N_) : N(N_), M(N_ + 1) {
        nV = (int32_t)(M * M * M);
        e0.resize(nV + 1);
        f0.resize(nV + 1);
        int32_t ce = 0, cf = 0;
        for (int64_t v = 0; v < nV; ++v) {
            int p[3] = {(int)(v % M), (int)((v / M) % M), (int)(v / (M * M))};
            e0[v] = ce;
            f0[v] = cf;
            for (int a = 0; a < 3; ++a) ce += edge_ok(N, p, a);
            for (int a = 0; a < 3; ++a) cf += face_ok(N, p, a);
        }
        e0[nV] = ce;
        f0[nV] = cf;
        nE = ce;
        nF = cf;
        nT = N * N * N;
    }
    int64_t vid(const int p[3]) const { return p[0] + M * (p[1] + M * (int64_t)p[2]); }
    int32_t edge(const int p[3], int a) const {
        int32_t id = e0[vid(p)];
        for (int b = 0; b < a; ++b) id += (p[b] < N);
        return id;
    }
    int32_t face(const int p[3], int a) const {   // order within a base vertex: a = 2, 1, 0
        int32_t id = f0[vid(p)];
        for (int b = 2; b > a; --b) id += face_ok(N, (int*)p, b);
        return id;
    }
    int32_t cube(const int p[3]) const { return p[0] + N * (p[1] + N * p[2]); }
    // incidences
    Csr grad() const {
        Csr G;
        G.nrows = nE; G.ncols = nV;
        for (int64_t v = 0; v < nV; ++v) {
            int p[3] = {(int)(v % M), (int)((v / M) % M), (int)(v / (M * M))};
            for (int a = 0; a < 3; ++a) {
                if (p[a] >= N) continue;
                int q[3] = {p[0], p[1], p[2]};
                q[a]++;
                G.col.push_back((int32_t)v); G.val.push_back(-1.0);
                G.col.push_back((int32_t)vid(q)); G.val.push_back(1.0);
                G.rowptr.push_back((int32_t)G.col.size());
            }
        }
        return G;
    }
    Csr curl() const {
        std::vector<int64_t> keys;
        std::vector<double> vals;
        for (int64_t v = 0; v < nV; ++v) {
            int p[3] = {(int)(v % M), (int)((v / M) % M), (int)(v / (M * M))};
            for (int a = 0; a < 3; ++a) {
                if (!face_ok(N, p, a)) continue;
                int b = (a + 1) % 3, c = (a + 2) % 3;
                int32_t f = face(p, a);
                int pb[3] = {p[0], p[1], p[2]}, pc[3] = {p[0], p[1], p[2]};
                pb[b]++; pc[c]++;
                int32_t es[4] = {edge(p, b), edge(pb, c), edge(pc, b), edge(p, c)};
                double sg[4] = {1, 1, -1, -1};
                for (int t = 0; t < 4; ++t) { keys.push_back((int64_t)f * nE + es[t]); vals.push_back(sg[t]); }
            }
        }
        return from_triplets(nF, nE, keys, vals, true);
    }
    Csr div() const {
        std::vector<int64_t> keys;
        std::vector<double> vals;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    int p[3] = {i, j, k};
                    int32_t t = cube(p);
                    for (int a = 0; a < 3; ++a) {
                        int q[3] = {i, j, k};
                        q[a]++;
                        keys.push_back((int64_t)t * nF + face(q, a)); vals.push_back(1.0);
                        keys.push_back((int64_t)t * nF + face(p, a)); vals.push_back(-1.0);
                    }
                }
        return from_triplets(nT, nF, keys, vals, true);
    }
};

// ------------------------------------------------------------------ reference block
// A 2x2x2 block of cells (Kuhn hexes on the fine level, cubes on coarser levels) and
// the single coarse cube it forms.  Block entities are classified by the coarse entity
// holding them in its relative interior: an axis is "pinned" when all vertices of the
// entity have the same coordinate 0 or 2 on it; owner dimension = number of free axes.
struct Owner {
    int dim;        // 0..3
    int id;         // index in the coarse cube's canonical local order (N = 1 complex)
    double phi;     // orientation of the block entity relative to the coarse one
    double ratio;   // measure(entity) / measure(owner) when dims agree
};

struct Block {
    // block entity counts and incidences (block-local canonical orders)
    int nV = 27, nE = 0, nF = 0, nC = 0;
    Csr C, Dv;                         // block curl (F x E), div (C x F)
    std::vector<Owner> eo, fo, co;     // owners of edges / faces / cells
    Mat Mnd, Mrt;                      // block masses over all block edges / faces
    std::vector<std::vector<int>> fedges;   // edges of each block face
    std::vector<Mat> ftrace;           // tangential-trace mass of each block face
};

// Canonical local orders of the single coarse cube (N = 1 complex).
struct Unit {
    Cubes cc{1};
    int edge(int o[3], int a) const { return cc.edge(o, a); }
    int face(int o[3], int a) const { return cc.face(o, a); }
};

// Owner of a block entity given the lattice coordinates of its vertices (0..2).
Owner classify(const std::vector<std::array<int, 3>>& X, const Unit& U) {
    int pinned[3], val[3];
    int nfree = 0, freeax = -1, pinax = -1;
    for (int a = 0; a < 3; ++a) {
        int v = X[0][a];
        bool same = true;
        for (auto& x : X) same &= (x[a] == v);
        pinned[a] = same && (v == 0 || v == 2);
        val[a] = pinned[a] ? v / 2 : 0;
        if (!pinned[a]) { ++nfree; freeax = a; } else pinax = a;
    }
    Owner o{nfree, 0, 1.0, 0.0};
    if (nfree == 0) o.id = (int)U.cc.vid(val);
    if (nfree == 1) o.id = U.edge(val, freeax);
    if (nfree == 2) o.id = U.face(val, pinax);
    if (nfree == 3) o.id = 0;
    return o;
}

// Level-1 block: the Kuhn mesh of a 2x2x2 hex block.  w (optional): per block hex
// (i + 2 j + 4 k) the factors of its ND and RT element masses.
Block kuhn_block(double h, const Kuhn& B, const Unit& U, const std::array<double, 2>* w = nullptr) {
    Block blk;
    blk.nE = (int)B.E.size(); blk.nF = (int)B.F.size(); blk.nC = (int)B.T.size();
    // incidences
    {
        std::vector<int64_t> keys; std::vector<double> vals;
        for (int f = 0; f < blk.nF; ++f) {
            double sg[3] = {1, -1, 1};   // boundary of (a,b,c): (a,b) - (a,c) + (b,c)
            for (int t = 0; t < 3; ++t) { keys.push_back((int64_t)f * blk.nE + B.fe[f][t]); vals.push_back(sg[t]); }
        }
        blk.C = from_triplets(blk.nF, blk.nE, keys, vals, true);
        keys.clear(); vals.clear();
        for (int t = 0; t < blk.nC; ++t) {
            Tet g = kuhn_tet(B, t, h);
            for (int i = 0; i < 4; ++i) { keys.push_back((int64_t)t * blk.nF + B.tf[t][i]); vals.push_back(g.s[i]); }
        }
        blk.Dv = from_triplets(blk.nC, blk.nF, keys, vals, true);
    }
    // owners
    for (int e = 0; e < blk.nE; ++e) {
        std::vector<std::array<int, 3>> X = {B.coord(B.E[e][0]), B.coord(B.E[e][1])};
        Owner o = classify(X, U);
        if (o.dim == 1) {
            int a = -1;
            for (int ax = 0; ax < 3; ++ax) if (X[0][ax] != X[1][ax]) a = ax;
            double d = X[1][a] - X[0][a];
            o.phi = d > 0 ? 1.0 : -1.0;
            o.ratio = std::fabs(d) / 2.0;
        }
        blk.eo.push_back(o);
    }
    for (int f = 0; f < blk.nF; ++f) {
        std::vector<std::array<int, 3>> X = {B.coord(B.F[f][0]), B.coord(B.F[f][1]), B.coord(B.F[f][2])};
        Owner o = classify(X, U);
        if (o.dim == 2) {
            V3 x0{(double)X[0][0], (double)X[0][1], (double)X[0][2]}, x1{(double)X[1][0], (double)X[1][1], (double)X[1][2]},
               x2{(double)X[2][0], (double)X[2][1], (double)X[2][2]};
            V3 nrm = cross(x1 - x0, x2 - x0);
            int a = -1;
            for (int ax = 0; ax < 3; ++ax) if (X[0][ax] == X[1][ax] && X[1][ax] == X[2][ax]) a = ax;
            o.phi = comp(nrm, a) > 0 ? 1.0 : -1.0;
            o.ratio = 0.5 * std::sqrt(dot(nrm, nrm)) / 4.0;
        }
        blk.fo.push_back(o);
    }
    for (int t = 0; t < blk.nC; ++t) {
        Owner o{3, 0, 1.0, (1.0 / 6.0) / 8.0};
        blk.co.push_back(o);
    }
    // masses
    blk.Mnd = Mat(blk.nE, blk.nE);
    blk.Mrt = Mat(blk.nF, blk.nF);
    for (int t = 0; t < blk.nC; ++t) {
        Tet g = kuhn_tet(B, t, h);
        double Mn[6][6], Mr[4][4];
        nd_mass(g, Mn);
        rt_mass(g, Mr);
        double wn = 1.0, wr = 1.0;
        if (w) {
            auto c = B.coord(B.T[t][0]);   // the tet's hex: its lowest vertex
            wn = w[c[0] + 2 * c[1] + 4 * c[2]][0];
            wr = w[c[0] + 2 * c[1] + 4 * c[2]][1];
        }
        for (int p = 0; p < 6; ++p)
            for (int q = 0; q < 6; ++q) blk.Mnd(B.te[t][p], B.te[t][q]) += wn * Mn[p][q];
        for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q) blk.Mrt(B.tf[t][p], B.tf[t][q]) += wr * Mr[p][q];
    }
    for (int f = 0; f < blk.nF; ++f) {
        auto c0 = B.coord(B.F[f][0]), c1 = B.coord(B.F[f][1]), c2 = B.coord(B.F[f][2]);
        V3 x0{c0[0] * h, c0[1] * h, c0[2] * h}, x1{c1[0] * h, c1[1] * h, c1[2] * h}, x2{c2[0] * h, c2[1] * h, c2[2] * h};
        double Mt[3][3];
        tri_trace_mass(x0, x1, x2, Mt);
        Mat m(3, 3);
        for (int p = 0; p < 3; ++p) for (int q = 0; q < 3; ++q) m(p, q) = Mt[p][q];
        blk.fedges.push_back({B.fe[f][0], B.fe[f][1], B.fe[f][2]});
        blk.ftrace.push_back(m);
    }
    return blk;
}

// Element data of a cube-complex level, identical for every cell/face of the level:
// ND mass of a cube over its 12 edges and RT mass over its 6 faces (unit-cube canonical
// local order), ND trace mass of a face over its 4 edges in cyclic order
// (p,b), (p+e_b,c), (p+e_c,b), (p,c) for each normal axis a.
struct CubeElem {
    Mat nd, rt;
    Mat trace[3];
};

// Coarser-level block: the 2x2x2 cube complex.  Cell c (= i + 2 j + 4 k) carries the ND
// and RT masses cel[c]->nd * w[c][0] and cel[c]->rt * w[c][1]; the face trace masses
// are the level's `tr` (they do not depend on the cell weights).
Block cube_block(const CubeElem* const cel[8], const std::array<double, 2> w[8], const CubeElem& tr,
                 const Unit& U) {
    const CubeElem& el = tr;
    Block blk;
    Cubes c2(2);
    blk.nE = c2.nE; blk.nF = c2.nF; blk.nC = c2.nT;
    blk.C = c2.curl();
    blk.Dv = c2.div();
    // owners: entity vertex lists in block lattice coordinates
    for (int64_t v = 0; v < c2.nV; ++v) {
        int p[3] = {(int)(v % 3), (int)((v / 3) % 3), (int)(v / 9)};
        for (int a = 0; a < 3; ++a) {
            if (p[a] >= 2) continue;
            std::array<int, 3> x0 = {p[0], p[1], p[2]}, x1 = x0;
            x1[a]++;
            Owner o = classify({x0, x1}, U);
            if (o.dim == 1) { o.phi = 1.0; o.ratio = 0.5; }
            blk.eo.push_back(o);
        }
    }
    // faces in canonical order: per base vertex a = 2, 1, 0
    std::vector<std::array<int, 4>> fdesc;   // p0, p1, p2, a
    for (int64_t v = 0; v < c2.nV; ++v) {
        int p[3] = {(int)(v % 3), (int)((v / 3) % 3), (int)(v / 9)};
        for (int a = 2; a >= 0; --a) {
            if (!Cubes::face_ok(2, p, a)) continue;
            int b = (a + 1) % 3, c = (a + 2) % 3;
            std::array<int, 3> x0 = {p[0], p[1], p[2]}, xb = x0, xc = x0, xbc = x0;
            xb[b]++; xc[c]++; xbc[b]++; xbc[c]++;
            Owner o = classify({x0, xb, xc, xbc}, U);
            if (o.dim == 2) { o.phi = 1.0; o.ratio = 0.25; }
            blk.fo.push_back(o);
            fdesc.push_back({p[0], p[1], p[2], a});
        }
    }
    for (int t = 0; t < blk.nC; ++t) blk.co.push_back(Owner{3, 0, 1.0, 0.125});
    if ((int)blk.eo.size() != blk.nE || (int)blk.fo.size() != blk.nF) fail(AMGE_ERR_ARG, "block enumeration");
    // masses: every cell carries the element masses, mapped through the unit-cube order
    blk.Mnd = Mat(blk.nE, blk.nE);
    blk.Mrt = Mat(blk.nF, blk.nF);
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) {
                int q[3] = {i, j, k};
                std::vector<int> le(12), lf(6);
                for (int a = 0; a < 3; ++a)
                    for (int s = 0; s < 2; ++s)
                        for (int r = 0; r < 2; ++r) {
                            int o[3] = {0, 0, 0};
                            o[(a + 1) % 3] = s; o[(a + 2) % 3] = r;
                            int g[3] = {q[0] + o[0], q[1] + o[1], q[2] + o[2]};
                            le[U.edge(o, a)] = c2.edge(g, a);
                        }
                for (int a = 0; a < 3; ++a)
                    for (int s = 0; s < 2; ++s) {
                        int o[3] = {0, 0, 0};
                        o[a] = s;
                        int g[3] = {q[0] + o[0], q[1] + o[1], q[2] + o[2]};
                        lf[U.face(o, a)] = c2.face(g, a);
                    }
                const int cidx = i + 2 * j + 4 * k;
                const CubeElem& ce = *cel[cidx];
                if (ce.nd.r)
                    for (int p = 0; p < 12; ++p)
                        for (int r = 0; r < 12; ++r) blk.Mnd(le[p], le[r]) += w[cidx][0] * ce.nd(p, r);
                for (int p = 0; p < 6; ++p)
                    for (int r = 0; r < 6; ++r) blk.Mrt(lf[p], lf[r]) += w[cidx][1] * ce.rt(p, r);
            }
    for (auto& d : fdesc) {
        int p[3] = {d[0], d[1], d[2]}, a = d[3], b = (a + 1) % 3, c = (a + 2) % 3;
        int pb[3] = {p[0], p[1], p[2]}, pc[3] = {p[0], p[1], p[2]};
        pb[b]++; pc[c]++;
        blk.fedges.push_back({c2.edge(p, b), c2.edge(pb, c), c2.edge(pc, b), c2.edge(p, c)});
        blk.ftrace.push_back(el.trace[a].r ? el.trace[a] : Mat(4, 4));
    }
    return blk;
}

// Local prolongators of a block: rows = block entities, cols = unit-cube entities.
struct LocalP {
    Mat rt;   // nF x 6
    Mat nd;   // nE x 12
};

LocalP solve_block(const Block& blk, const Unit& U, bool need_nd) {
    const Cubes& cc = U.cc;
    Csr CH = cc.curl(), DH = cc.div();   // unit-cube incidences: 6 x 12, 1 x 6
    LocalP L;
    // ---- RT: PV traces on the coarse faces, eq. (3.5)
    L.rt = Mat(blk.nF, 6);
    for (int f = 0; f < blk.nF; ++f)
        if (blk.fo[f].dim == 2) L.rt(f, blk.fo[f].id) = blk.fo[f].phi * blk.fo[f].ratio;
    // ---- RT: face -> cube extension, eq. (3.6): div u = D^H[T,F] PV_T on every cell
    {
        std::vector<char> intr(blk.nF);
        for (int f = 0; f < blk.nF; ++f) intr[f] = blk.fo[f].dim == 3;
        Mat K(blk.nC, blk.nF);
        for (int t = 0; t < blk.nC; ++t)
            for (int k = blk.Dv.rowptr[t]; k < blk.Dv.rowptr[t + 1]; ++k) K(t, blk.Dv.col[k]) = blk.Dv.val[k];
        Mat S(blk.nC, 6), UB;
        for (int F = 0; F < 6; ++F) {
            double dh = 0;
            for (int k = DH.rowptr[0]; k < DH.rowptr[1]; ++k) if (DH.col[k] == F) dh = DH.val[k];
            for (int t = 0; t < blk.nC; ++t) S(t, F) = dh * blk.co[t].ratio;
        }
        int nB = 0;
        for (int f = 0; f < blk.nF; ++f) nB += !intr[f];
        UB = Mat(nB, 6);
        for (int f = 0, b = 0; f < blk.nF; ++f)
            if (!intr[f]) { for (int F = 0; F < 6; ++F) UB(b, F) = L.rt(f, F); ++b; }
        Mat UI = extend(blk.Mrt, K, intr, S, UB);
        for (int f = 0, a = 0; f < blk.nF; ++f)
            if (intr[f]) { for (int F = 0; F < 6; ++F) L.rt(f, F) = UI(a, F); ++a; }
    }
    if (!need_nd) return L;
    // ---- ND: PV traces on the coarse edges
    L.nd = Mat(blk.nE, 12);
    for (int e = 0; e < blk.nE; ++e)
        if (blk.eo[e].dim == 1) L.nd(e, blk.eo[e].id) = blk.eo[e].phi * blk.eo[e].ratio;
    // ---- ND: edge -> face extensions, eq. (3.6) in 2D: curl u = C^H[F,E] PV_F on F
    for (int F = 0; F < 6; ++F) {
        std::vector<int> dofs;           // block edges in the closure of F
        for (int e = 0; e < blk.nE; ++e) {
            const Owner& o = blk.eo[e];
            bool in = (o.dim == 2 && o.id == F);
            if (o.dim == 1)
                for (int k = CH.rowptr[F]; k < CH.rowptr[F + 1]; ++k) in |= (CH.col[k] == o.id);
            if (in) dofs.push_back(e);
        }
        std::vector<int> rows;           // block faces interior to F
        for (int f = 0; f < blk.nF; ++f) if (blk.fo[f].dim == 2 && blk.fo[f].id == F) rows.push_back(f);
        int nd = (int)dofs.size();
        std::map<int, int> loc;
        for (int i = 0; i < nd; ++i) loc[dofs[i]] = i;
        std::vector<char> intr(nd);
        for (int i = 0; i < nd; ++i) intr[i] = blk.eo[dofs[i]].dim == 2;
        Mat M(nd, nd), K((int)rows.size(), nd);
        for (int r = 0; r < (int)rows.size(); ++r) {
            int f = rows[r];
            const auto& fe = blk.fedges[f];
            const Mat& T = blk.ftrace[f];
            for (size_t p = 0; p < fe.size(); ++p)
                for (size_t q = 0; q < fe.size(); ++q) M(loc[fe[p]], loc[fe[q]]) += T((int)p, (int)q);
            for (int k = blk.C.rowptr[f]; k < blk.C.rowptr[f + 1]; ++k) K(r, loc[blk.C.col[k]]) = blk.C.val[k];
        }
        std::vector<int> Es;             // coarse edges of F
        std::vector<double> cs;
        for (int k = CH.rowptr[F]; k < CH.rowptr[F + 1]; ++k) { Es.push_back(CH.col[k]); cs.push_back(CH.val[k]); }
        int ne = (int)Es.size();
        Mat S((int)rows.size(), ne), UB(nd - [&] { int c = 0; for (char x : intr) c += x; return c; }(), ne);
        for (int r = 0; r < (int)rows.size(); ++r)
            for (int j = 0; j < ne; ++j) S(r, j) = cs[j] * L.rt(rows[r], F);
        for (int i = 0, b = 0; i < nd; ++i)
            if (!intr[i]) { for (int j = 0; j < ne; ++j) UB(b, j) = L.nd(dofs[i], Es[j]); ++b; }
        Mat UI = extend(M, K, intr, S, UB);
        for (int i = 0, a = 0; i < nd; ++i)
            if (intr[i]) { for (int j = 0; j < ne; ++j) L.nd(dofs[i], Es[j]) = UI(a, j); ++a; }
    }
    // ---- ND: face -> cube extension, eq. (3.8): curl u = sum_F C^H[F,E] (RT basis of F)
    {
        std::vector<char> intr(blk.nE);
        for (int e = 0; e < blk.nE; ++e) intr[e] = blk.eo[e].dim == 3;
        std::vector<int> rows;
        for (int f = 0; f < blk.nF; ++f) if (blk.fo[f].dim == 3) rows.push_back(f);
        Mat K((int)rows.size(), blk.nE);
        for (int r = 0; r < (int)rows.size(); ++r)
            for (int k = blk.C.rowptr[rows[r]]; k < blk.C.rowptr[rows[r] + 1]; ++k) K(r, blk.C.col[k]) = blk.C.val[k];
        Mat S((int)rows.size(), 12);
        for (int F = 0; F < 6; ++F)
            for (int k = CH.rowptr[F]; k < CH.rowptr[F + 1]; ++k)
                for (int r = 0; r < (int)rows.size(); ++r) S(r, CH.col[k]) += CH.val[k] * L.rt(rows[r], F);
        int nB = 0;
        for (char x : intr) nB += !x;
        Mat UB(nB, 12);
        for (int e = 0, b = 0; e < blk.nE; ++e)
            if (!intr[e]) { for (int E = 0; E < 12; ++E) UB(b, E) = L.nd(e, E); ++b; }
        Mat UI = extend(blk.Mnd, K, intr, S, UB);
        for (int e = 0, a = 0; e < blk.nE; ++e)
            if (intr[e]) { for (int E = 0; E < 12; ++E) L.nd(e, E) = UI(a, E); ++a; }
    }
    return L;
}

// Element data of the next level: RAP of the block masses with the local prolongators.
CubeElem next_elem(const Block& blk, const LocalP& L, const Unit& U, bool need_nd) {
    CubeElem el;
    el.rt = tmatmul(L.rt, matmul(blk.Mrt, L.rt));
    if (!need_nd) return el;
    el.nd = tmatmul(L.nd, matmul(blk.Mnd, L.nd));
    const Cubes& cc = U.cc;
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        int o[3] = {0, 0, 0};
        int F = cc.face(o, a);
        int ob[3] = {0, 0, 0}, oc[3] = {0, 0, 0};
        ob[b] = 1; oc[c] = 1;
        int Es[4] = {cc.edge(o, b), cc.edge(ob, c), cc.edge(oc, b), cc.edge(o, c)};
        // trace mass on F: block faces interior to F, over their edges
        std::map<int, int> loc;
        std::vector<int> dofs;
        for (int f = 0; f < blk.nF; ++f)
            if (blk.fo[f].dim == 2 && blk.fo[f].id == F)
                for (int e : blk.fedges[f])
                    if (!loc.count(e)) { loc[e] = (int)dofs.size(); dofs.push_back(e); }
        Mat M((int)dofs.size(), (int)dofs.size());
        for (int f = 0; f < blk.nF; ++f)
            if (blk.fo[f].dim == 2 && blk.fo[f].id == F) {
                const auto& fe = blk.fedges[f];
                for (size_t p = 0; p < fe.size(); ++p)
                    for (size_t q = 0; q < fe.size(); ++q) M(loc[fe[p]], loc[fe[q]]) += blk.ftrace[f]((int)p, (int)q);
            }
        Mat PF((int)dofs.size(), 4);
        for (size_t i = 0; i < dofs.size(); ++i)
            for (int j = 0; j < 4; ++j) PF((int)i, j) = L.nd(dofs[i], Es[j]);
        el.trace[a] = tmatmul(PF, matmul(M, PF));
    }
    return el;
}

// ------------------------------------------------------------------ batched weighted local problems
// The weighted local problems of the first agglomeration step.  Every agglomerate of the
// step has the reference block's topology, constraints, PV traces and face extensions
// (no cell weight enters those); its RT and ND masses are sums over its eight hexes
// ("slots") of the slot's unit mass times the hex weight, M(w) = sum_s w_s M_s.  So the
// null space of each constraint, the particular solution (RT) and every slot's reduced
// matrices are formed once, and an agglomerate's problem reduces to weighted sums of
// small matrices and one Cholesky solve:
//   RT:  u = u_p + Q2 y,  (sum_s w_s H_s) y = -(sum_s w_s h_s),
//        H_s = Q2^T M_s,II Q2,  h_s = Q2^T (M_s,II u_p + M_s,IB u_B);
//        next-level RT element  L^T M(w) L = sum_s w_s C_s + h(w)^T y  (the Schur form:
//        C_s = L_p^T M_s L_p with L_p the particular local prolongator).
//   ND (H(curl)): the constraint's right-hand side is the coarse curl of the RT
//        solution, G = u_I C^H - G0, so u_p = Wn G varies; the ND mass M(w) is formed
//        explicitly (26 x 26) and minimised over its null space Q2n.
// This is what the device path (setup_device.hip) computes per agglomerate.
struct KuhnPlan {
    bool nd = false;
    std::vector<int> fI, eI;     // interior block faces / edges (constraint order)
    int nI = 0, nz = 0;          // RT interior faces, null-space dimension
    Mat up, Q2;                  // nI x 6, nI x nz
    Mat H[8], h[8], C[8];        // per slot: nz x nz, nz x 6, 6 x 6
    int nIn = 0, nzn = 0;        // ND interior edges, null-space dimension
    Mat CH, G0, Wn, Q2n;         // 6 x 12, nI x 12, nIn x nI, nIn x nzn
    Mat Mn[8], Fn[8], Cn[8];     // per slot: nIn x nIn, nIn x 12, 12 x 12
    LocalP ref;                  // unit-weight solution: the rows every agglomerate shares
    CubeElem ref_el;             // unit-weight next element (its trace masses are shared)
};

KuhnPlan kuhn_plan(double h, const Kuhn& B, const Unit& U, bool need_nd) {
    KuhnPlan P;
    P.nd = need_nd;
    Block blk = kuhn_block(h, B, U);
    P.ref = solve_block(blk, U, need_nd);
    P.ref_el = next_elem(blk, P.ref, U, need_nd);
    const Cubes& cc = U.cc;
    Csr CHs = cc.curl(), DH = cc.div();
    // RT: constraint div u = D^H[T,F] PV_T on every cell, interior = faces inside the cube
    std::vector<char> fin(blk.nF);
    for (int f = 0; f < blk.nF; ++f) fin[f] = blk.fo[f].dim == 3;
    Mat K(blk.nC, blk.nF), S(blk.nC, 6);
    for (int t = 0; t < blk.nC; ++t)
        for (int k = blk.Dv.rowptr[t]; k < blk.Dv.rowptr[t + 1]; ++k) K(t, blk.Dv.col[k]) = blk.Dv.val[k];
    for (int F = 0; F < 6; ++F) {
        double dh = 0;
        for (int k = DH.rowptr[0]; k < DH.rowptr[1]; ++k) if (DH.col[k] == F) dh = DH.val[k];
        for (int t = 0; t < blk.nC; ++t) S(t, F) = dh * blk.co[t].ratio;
    }
    std::vector<int> fB;
    for (int f = 0; f < blk.nF; ++f) (fin[f] ? P.fI : fB).push_back(f);
    Mat UB((int)fB.size(), 6);
    for (size_t b = 0; b < fB.size(); ++b)
        for (int F = 0; F < 6; ++F) UB((int)b, F) = P.ref.rt(fB[b], F);
    Mat KI, G;
    std::vector<int> Iv, Bv;
    split_constraint(K, fin, S, UB, Iv, Bv, KI, G);
    NullSpace ns(KI);
    P.nI = ns.nI;
    P.nz = ns.nI - ns.rk;
    P.up = ns.particular(G);
    P.Q2 = ns.Q2();
    // per slot (hex s of the block): unit RT and ND masses
    Block bs[8];
    for (int sl = 0; sl < 8; ++sl) {
        std::array<double, 2> w[8];
        for (int i = 0; i < 8; ++i) w[i] = {i == sl ? 1.0 : 0.0, i == sl ? 1.0 : 0.0};
        bs[sl] = kuhn_block(h, B, U, w);
    }
    // boundary / interior parts of the particular local prolongator (RT)
    Mat Lp = P.ref.rt;
    for (int a = 0; a < P.nI; ++a)
        for (int F = 0; F < 6; ++F) Lp(P.fI[a], F) = P.up(a, F);
    for (int sl = 0; sl < 8; ++sl) {
        const Mat& M = bs[sl].Mrt;
        Mat MII(P.nI, P.nI), Fs(P.nI, 6);
        for (int a = 0; a < P.nI; ++a) {
            for (int b = 0; b < P.nI; ++b) MII(a, b) = M(P.fI[a], P.fI[b]);
            for (int F = 0; F < 6; ++F) {
                double v = 0;
                for (size_t b = 0; b < fB.size(); ++b) v += M(P.fI[a], fB[b]) * UB((int)b, F);
                for (int b = 0; b < P.nI; ++b) v += MII(a, b) * P.up(b, F);
                Fs(a, F) = v;   // M_II u_p + M_IB u_B
            }
        }
        P.H[sl] = tmatmul(P.Q2, matmul(MII, P.Q2));
        P.h[sl] = tmatmul(P.Q2, Fs);
        P.C[sl] = tmatmul(Lp, matmul(M, Lp));
    }
    if (!need_nd) return P;
    // ND: constraint curl u = sum_F C^H[F,E] (RT basis of F) on the faces inside the cube,
    // interior = edges inside the cube; the boundary edges carry the shared PV and face
    // extension values
    P.CH = Mat(6, 12);
    for (int F = 0; F < 6; ++F)
        for (int k = CHs.rowptr[F]; k < CHs.rowptr[F + 1]; ++k) P.CH(F, CHs.col[k]) = CHs.val[k];
    std::vector<char> ein(blk.nE);
    for (int e = 0; e < blk.nE; ++e) ein[e] = blk.eo[e].dim == 3;
    Mat Kn(P.nI, blk.nE);
    for (int r = 0; r < P.nI; ++r)
        for (int k = blk.C.rowptr[P.fI[r]]; k < blk.C.rowptr[P.fI[r] + 1]; ++k) Kn(r, blk.C.col[k]) = blk.C.val[k];
    std::vector<int> eB;
    for (int e = 0; e < blk.nE; ++e) (ein[e] ? P.eI : eB).push_back(e);
    Mat UBn((int)eB.size(), 12);
    for (size_t b = 0; b < eB.size(); ++b)
        for (int E = 0; E < 12; ++E) UBn((int)b, E) = P.ref.nd(eB[b], E);
    Mat KnI, G0neg;
    Mat zeroS(P.nI, 12);
    split_constraint(Kn, ein, zeroS, UBn, Iv, Bv, KnI, G0neg);   // G0neg = -K_B u_B
    P.G0 = G0neg;
    for (double& v : P.G0.a) v = -v;                             // G0 = K_B u_B
    NullSpace nsn(KnI);
    P.nIn = nsn.nI;
    P.nzn = nsn.nI - nsn.rk;
    Mat Id(P.nI, P.nI);
    for (int i = 0; i < P.nI; ++i) Id(i, i) = 1.0;
    P.Wn = nsn.particular(Id);                                   // u_p = Wn G
    P.Q2n = nsn.Q2();
    for (int sl = 0; sl < 8; ++sl) {
        const Mat& M = bs[sl].Mnd;
        P.Mn[sl] = Mat(P.nIn, P.nIn);
        P.Fn[sl] = Mat(P.nIn, 12);
        P.Cn[sl] = Mat(12, 12);
        for (int a = 0; a < P.nIn; ++a) {
            for (int b = 0; b < P.nIn; ++b) P.Mn[sl](a, b) = M(P.eI[a], P.eI[b]);
            for (int E = 0; E < 12; ++E) {
                double v = 0;
                for (size_t b = 0; b < eB.size(); ++b) v += M(P.eI[a], eB[b]) * UBn((int)b, E);
                P.Fn[sl](a, E) = v;   // M_IB u_B
            }
        }
        for (int E = 0; E < 12; ++E)
            for (int E2 = 0; E2 < 12; ++E2) {
                double v = 0;
                for (size_t a = 0; a < eB.size(); ++a)
                    for (size_t b = 0; b < eB.size(); ++b) v += UBn((int)a, E) * M(eB[a], eB[b]) * UBn((int)b, E2);
                P.Cn[sl](E, E2) = v;   // u_B^T M_BB u_B
            }
    }
    return P;
}

// The weighted local problems of one agglomerate (hex weights wnd / wrt per slot): its
// local prolongator (the shared rows from the reference, the interior ones solved) and
// next-level element.
void kuhn_solve_one(const KuhnPlan& P, const double* wnd, const double* wrt, LocalP& L, CubeElem& el) {
    L = P.ref;
    el = P.ref_el;
    Mat Hw(P.nz, P.nz), hw(P.nz, 6), Cw(6, 6);
    for (int sl = 0; sl < 8; ++sl) {
        for (size_t i = 0; i < Hw.a.size(); ++i) Hw.a[i] += wrt[sl] * P.H[sl].a[i];
        for (size_t i = 0; i < hw.a.size(); ++i) hw.a[i] += wrt[sl] * P.h[sl].a[i];
        for (size_t i = 0; i < Cw.a.size(); ++i) Cw.a[i] += wrt[sl] * P.C[sl].a[i];
    }
    Mat y = hw;
    for (double& v : y.a) v = -v;
    if (P.nz > 0) {
        if (!cholesky(Hw)) fail(AMGE_ERR_NOT_SPD, "local mass not positive definite on the null space");
        chol_solve(Hw, y);
    }
    Mat u = P.up;
    if (P.nz > 0) {
        Mat Z = matmul(P.Q2, y);
        for (size_t i = 0; i < u.a.size(); ++i) u.a[i] += Z.a[i];
    }
    for (int a = 0; a < P.nI; ++a)
        for (int F = 0; F < 6; ++F) L.rt(P.fI[a], F) = u(a, F);
    Mat hy = tmatmul(hw, y);
    for (size_t i = 0; i < Cw.a.size(); ++i) el.rt.a[i] = Cw.a[i] + hy.a[i];
    if (!P.nd) return;
    // ND: G = u C^H - G0, u_p = Wn G, mass M(w) minimised over the null space
    Mat G = matmul(u, P.CH);
    for (size_t i = 0; i < G.a.size(); ++i) G.a[i] -= P.G0.a[i];
    Mat un = matmul(P.Wn, G);
    Mat Mw(P.nIn, P.nIn), Fw(P.nIn, 12), Cnw(12, 12);
    for (int sl = 0; sl < 8; ++sl) {
        for (size_t i = 0; i < Mw.a.size(); ++i) Mw.a[i] += wnd[sl] * P.Mn[sl].a[i];
        for (size_t i = 0; i < Fw.a.size(); ++i) Fw.a[i] += wnd[sl] * P.Fn[sl].a[i];
        for (size_t i = 0; i < Cnw.a.size(); ++i) Cnw.a[i] += wnd[sl] * P.Cn[sl].a[i];
    }
    if (P.nzn > 0) {
        Mat R = matmul(Mw, un);
        for (size_t i = 0; i < R.a.size(); ++i) R.a[i] += Fw.a[i];
        Mat yn = tmatmul(P.Q2n, R);
        for (double& v : yn.a) v = -v;
        Mat Hn = tmatmul(P.Q2n, matmul(Mw, P.Q2n));
        if (!cholesky(Hn)) fail(AMGE_ERR_NOT_SPD, "local mass not positive definite on the null space");
        chol_solve(Hn, yn);
        Mat Z = matmul(P.Q2n, yn);
        for (size_t i = 0; i < un.a.size(); ++i) un.a[i] += Z.a[i];
    }
    for (int a = 0; a < P.nIn; ++a)
        for (int E = 0; E < 12; ++E) L.nd(P.eI[a], E) = un(a, E);
    // el.nd = u^T M_II u + u^T F + F^T u + u_B^T M_BB u_B with M = M(w)
    Mat uMu = tmatmul(un, matmul(Mw, un)), uF = tmatmul(un, Fw);
    for (int E = 0; E < 12; ++E)
        for (int E2 = 0; E2 < 12; ++E2) el.nd(E, E2) = uMu(E, E2) + uF(E, E2) + uF(E2, E) + Cnw(E, E2);
}

// ------------------------------------------------------------------ global assembly
struct Problem {
    int kind, n, nlevels;
    std::vector<Csr> A, D, P;
};

// Fine system matrix, eq. (2.2).
Csr fine_matrix(const Kuhn& K, int kind, const double* alpha, const double* beta) {
    // the tetrahedra are translates of the six of the cube at the origin (tetrahedron t
    // is cube t / 6's copy of type t % 6, with the same local vertex order and face
    // orientations), so their unit-coefficient element matrices are computed once
    const int n = K.n;
    const double h = 1.0 / n;
    const int64_t nt = (int64_t)K.T.size();
    const int per = kind == AMGE_CURL ? 36 : 16;
    const int32_t ndof = kind == AMGE_CURL ? (int32_t)K.E.size() : (int32_t)K.F.size();
    double Ka[6][36], Mb[6][36];   // per type: the alpha and beta parts, row-major
    {
        Kuhn C = build_kuhn(1);
        for (int p = 0; p < 6; ++p) {
            Tet g = kuhn_tet(C, p, h);
            if (kind == AMGE_CURL) {
                double M[6][6], Kc[6][6];
                nd_mass(g, M);
                curlcurl(g, Kc);
                for (int a = 0; a < 6; ++a)
                    for (int b = 0; b < 6; ++b) {
                        Ka[p][a * 6 + b] = Kc[a][b];
                        Mb[p][a * 6 + b] = M[a][b];
                    }
            } else {
                double M[4][4];
                rt_mass(g, M);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        Ka[p][a * 4 + b] = g.s[a] * g.s[b] / g.vol;
                        Mb[p][a * 4 + b] = M[a][b];
                    }
            }
        }
    }
    // written in full (and first touched) by the parallel loop
    std::unique_ptr<int64_t[]> keys(new int64_t[nt * per + 1]);
    std::unique_ptr<double[]> vals(new double[nt * per + 1]);
    parallel_for(nt, [&](int64_t s, int64_t e) {
        for (int64_t t = s; t < e; ++t) {
            const int p = (int)(t % 6);
            const int64_t hx = t / 6;   // cube index i + n (j + n k), as the coefficients
            const double al = alpha[hx], be = beta[hx];
            int64_t o = t * per;
            const int w = kind == AMGE_CURL ? 6 : 4;
            const int32_t* dof = kind == AMGE_CURL ? K.te[t].data() : K.tf[t].data();
            for (int a = 0; a < w; ++a)
                for (int b = 0; b < w; ++b) {
                    keys[o] = (int64_t)dof[a] * ndof + dof[b];
                    vals[o++] = al * Ka[p][a * w + b] + be * Mb[p][a * w + b];
                }
        }
    });
    return from_triplets(ndof, ndof, keys.get(), vals.get(), nt * per, true);
}

Csr kuhn_grad(const Kuhn& K) {
    Csr G;
    G.nrows = (int32_t)K.E.size();
    G.ncols = (int32_t)K.nv;
    for (auto& e : K.E) {
        G.col.push_back(e[0]); G.val.push_back(-1.0);
        G.col.push_back(e[1]); G.val.push_back(1.0);
        G.rowptr.push_back((int32_t)G.col.size());
    }
    return G;
}

Csr kuhn_curl(const Kuhn& K) {
    std::vector<int64_t> keys;
    std::vector<double> vals;
    int32_t nE = (int32_t)K.E.size();
    for (size_t f = 0; f < K.F.size(); ++f) {
        double sg[3] = {1, -1, 1};
        for (int t = 0; t < 3; ++t) { keys.push_back((int64_t)f * nE + K.fe[f][t]); vals.push_back(sg[t]); }
    }
    return from_triplets((int32_t)K.F.size(), nE, keys, vals, true);
}

// Place the local prolongators at every agglomerate.  local_of(t) is the block
// prolongator of agglomerate t (coarse cube t = i + Nc (j + Nc k)); `fine_index(q,
// local)` maps a block entity of the agglomerate with base q to its global index on the
// finer level; coarse entities (unit-cube local order) map to the coarser cube complex.
// Entries that vanish up to rounding (below 1e-14 of the local prolongator's largest) are
// not stored.
template <class FineIndex, class LocalOf>
Csr stamp(const LocalOf& local_of, int kind_dim, int Nc, int32_t nfine, const FineIndex& fine_index) {
    Cubes coarse(Nc);
    Unit U;
    // unit-cube entity (o, a) -> global coarse entity (q + o, a)
    std::vector<std::array<int, 4>> udesc(kind_dim == 1 ? 12 : 6);
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            for (int r = 0; r < 2; ++r) {
                if (kind_dim == 1) {
                    int o[3] = {0, 0, 0};
                    o[(a + 1) % 3] = s; o[(a + 2) % 3] = r;
                    udesc[U.edge(o, a)] = {o[0], o[1], o[2], a};
                } else if (r == 0) {
                    int o[3] = {0, 0, 0};
                    o[a] = s;
                    udesc[U.face(o, a)] = {o[0], o[1], o[2], a};
                }
            }
    int32_t ncoarse = kind_dim == 1 ? coarse.nE : coarse.nF;
    int64_t ncube = (int64_t)Nc * Nc * Nc;
    // per chunk of agglomerates, in agglomerate order (first-kept duplicates are then
    // independent of the threading)
    std::map<int64_t, std::pair<std::vector<int64_t>, std::vector<double>>> parts;
    std::mutex mu;
    parallel_for(ncube, [&](int64_t s, int64_t e) {
        std::vector<int64_t> keys;
        std::vector<double> vals;
        std::vector<int32_t> fi, ci;
        for (int64_t t = s; t < e; ++t) {
            const Mat& Pl = local_of(t);
            double mx = 0;
            for (double v : Pl.a) mx = std::max(mx, std::fabs(v));
            const double tiny = 1e-14 * mx;
            int q[3] = {(int)(t % Nc), (int)((t / Nc) % Nc), (int)(t / ((int64_t)Nc * Nc))};
            fi.resize(Pl.r);
            ci.resize(Pl.c);
            for (int i = 0; i < Pl.r; ++i) fi[i] = fine_index(q, i);
            for (int j = 0; j < Pl.c; ++j) {
                int g[3] = {q[0] + udesc[j][0], q[1] + udesc[j][1], q[2] + udesc[j][2]};
                ci[j] = kind_dim == 1 ? coarse.edge(g, udesc[j][3]) : coarse.face(g, udesc[j][3]);
            }
            for (int i = 0; i < Pl.r; ++i)
                for (int j = 0; j < Pl.c; ++j)
                    if (std::fabs(Pl(i, j)) > tiny) {
                        keys.push_back((int64_t)fi[i] * ncoarse + ci[j]);
                        vals.push_back(Pl(i, j));
                    }
        }
        std::lock_guard<std::mutex> lk(mu);
        parts[s] = {std::move(keys), std::move(vals)};
    });
    std::vector<int64_t> keys;
    std::vector<double> vals;
    for (auto& kv : parts) {
        keys.insert(keys.end(), kv.second.first.begin(), kv.second.first.end());
        vals.insert(vals.end(), kv.second.second.begin(), kv.second.second.end());
    }
    return from_triplets(nfine, ncoarse, keys, vals, false);
}

// Weights of a cell's element masses in the extension problems (coefficient-aware
// extensions): the ND masses carry nd, the RT masses rt; ex >= 0 names an explicit
// element (from a non-uniform agglomerate below), whose masses already carry them.
struct CellW {
    double nd = 1.0, rt = 1.0;
    int32_t ex = -1;
};

// An agglomerate whose eight cells carry the same scalar weights: each of its local
// problems is the reference one with its mass scaled, which has the same minimiser.
bool uniform_cells(const CellW* const c[8]) {
    for (int i = 0; i < 8; ++i)
        if (c[i]->ex >= 0 || c[i]->nd != c[0]->nd || c[i]->rt != c[0]->rt) return false;
    return true;
}

// Essential boundary conditions: keep the entities not lying in the boundary of the
// cube.  map[i] = new index of a kept entity, -1 for a boundary one.
std::vector<int32_t> renumber(const std::vector<char>& bnd) {
    std::vector<int32_t> m(bnd.size());
    int32_t k = 0;
    for (size_t i = 0; i < bnd.size(); ++i) m[i] = bnd[i] ? -1 : k++;
    return m;
}

Csr restrict_csr(const Csr& A, const std::vector<int32_t>& rmap, const std::vector<int32_t>& cmap) {
    Csr B;
    B.ncols = 0;
    for (int32_t v : cmap) B.ncols += v >= 0;
    B.nrows = 0;
    for (int32_t i = 0; i < A.nrows; ++i) {
        if (rmap[i] < 0) continue;
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q)
            if (cmap[A.col[q]] >= 0) {
                B.col.push_back(cmap[A.col[q]]);
                B.val.push_back(A.val[q]);
            }
        B.rowptr.push_back((int32_t)B.col.size());
        ++B.nrows;
    }
    return B;
}

// Boundary masks of the fine Kuhn mesh: vertices (d = 0), edges (1), faces (2) whose
// vertices all lie on one face of the cube (a shared coordinate 0 or n).
std::vector<char> kuhn_boundary(const Kuhn& K, int d) {
    auto on = [&](const std::vector<std::array<int, 3>>& X) {
        for (int a = 0; a < 3; ++a) {
            bool lo = true, hi = true;
            for (auto& x : X) { lo &= x[a] == 0; hi &= x[a] == K.n; }
            if (lo || hi) return true;
        }
        return false;
    };
    std::vector<char> m;
    if (d == 0)
        for (int64_t v = 0; v < K.nv; ++v) m.push_back(on({K.coord(v)}));
    else if (d == 1)
        for (auto& e : K.E) m.push_back(on({K.coord(e[0]), K.coord(e[1])}));
    else
        for (auto& f : K.F) m.push_back(on({K.coord(f[0]), K.coord(f[1]), K.coord(f[2])}));
    return m;
}

// Boundary masks of the cube complex with N cells per side: a vertex with a coordinate
// 0 or N; an edge (p, a) with such a coordinate off its axis; a face (p, a) with p_a = 0
// or N.
std::vector<char> cubes_boundary(const Cubes& C, int d) {
    const int N = C.N;
    auto edgeb = [&](int p) { return p == 0 || p == N; };
    std::vector<char> m(d == 0 ? C.nV : d == 1 ? C.nE : C.nF, 0);
    for (int64_t v = 0; v < C.nV; ++v) {
        int p[3] = {(int)(v % C.M), (int)((v / C.M) % C.M), (int)(v / (C.M * C.M))};
        if (d == 0) m[v] = edgeb(p[0]) || edgeb(p[1]) || edgeb(p[2]);
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            if (d == 1 && Cubes::edge_ok(N, p, a)) m[C.edge(p, a)] = edgeb(p[b]) || edgeb(p[c]);
            if (d == 2 && Cubes::face_ok(N, p, a)) m[C.face(p, a)] = edgeb(p[a]);
        }
    }
    return m;
}

// Wall-clock phases of the build, printed with AMGE_VERBOSE.
struct BuildClock {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    std::map<std::string, double> ms;
    void lap(const char* name) {
        auto now = std::chrono::steady_clock::now();
        ms[name] += std::chrono::duration<double, std::milli>(now - t).count();
        t = now;
    }
    ~BuildClock() {
        const char* e = getenv("AMGE_VERBOSE");
        if (!e || !*e || *e == '0') return;
        for (auto& kv : ms) fprintf(stderr, "[amge build] %-28s %9.1f ms\n", kv.first.c_str(), kv.second);
    }
};

Problem build(int kind, int n, int nlevels, const double* alpha, const double* beta, int flags) {
    BuildClock clk;
    if (kind != AMGE_CURL && kind != AMGE_DIV) fail(AMGE_ERR_ARG, "kind must be AMGE_CURL or AMGE_DIV");
    if (n < 1 || nlevels < 1) fail(AMGE_ERR_ARG, "n and nlevels must be positive");
    if (nlevels > 1 && (n % (1 << (nlevels - 1))) != 0) fail(AMGE_ERR_ARG, "n not divisible by 2^(nlevels-1)");
    if (!alpha || !beta) fail(AMGE_ERR_ARG, "null coefficient array");
    if (flags & ~(AMGE_BUILD_ESSENTIAL | AMGE_BUILD_COEFFICIENT | AMGE_BUILD_DEVICE))
        fail(AMGE_ERR_ARG, "unknown build flags");
    for (int64_t i = 0; i < (int64_t)n * n * n; ++i)
        if (!(alpha[i] > 0) || !(beta[i] > 0) || !std::isfinite(alpha[i]) || !std::isfinite(beta[i]))
            fail(AMGE_ERR_ARG, "coefficients must be positive and finite");
    const bool curl = kind == AMGE_CURL;
    const int sdim = curl ? 1 : 2;
    Problem pr;
    pr.kind = kind; pr.n = n; pr.nlevels = nlevels;
    Kuhn K = build_kuhn(n);
    clk.lap("Kuhn mesh");
    pr.A.push_back(fine_matrix(K, kind, alpha, beta));
    pr.D.push_back(curl ? kuhn_grad(K) : kuhn_curl(K));
    clk.lap("fine matrix, derivative");
    Unit U;
    // extension weights per cell of the current level: the system space's masses carry
    // beta, the next space's (RT for H(curl)) alpha; all 1 for unweighted extensions
    const bool coef = (flags & AMGE_BUILD_COEFFICIENT) != 0;
    std::vector<CellW> cw((size_t)n * n * n);
    if (coef)
        for (size_t i = 0; i < cw.size(); ++i) {
            cw[i].nd = curl ? beta[i] : 1.0;
            cw[i].rt = curl ? alpha[i] : beta[i];
        }
    std::vector<CubeElem> ex;   // explicit elements of the current level (non-uniform cells)
    // Per agglomerate of the step from `Nf` cells per side: its eight cells' weights, and
    // whether it is uniform.
    auto children = [&](int Nf, int64_t t, const CellW* c[8]) {
        const int Nc = Nf / 2;
        int q[3] = {(int)(t % Nc), (int)((t / Nc) % Nc), (int)(t / ((int64_t)Nc * Nc))};
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) {
                    int64_t cell = (2 * q[0] + i) + (int64_t)Nf * ((2 * q[1] + j) + (int64_t)Nf * (2 * q[2] + k));
                    c[i + 2 * j + 4 * k] = &cw[cell];
                }
    };
    // level 1 -> 2: reference Kuhn block (unit weights); non-uniform agglomerates solve
    // their own weighted block
    CubeElem el;   // reference element of the current level (unit weights)
    if (nlevels > 1) {
        Kuhn B = build_kuhn(2);
        Block blk = kuhn_block(1.0 / n, B, U);
        LocalP L = solve_block(blk, U, curl);
        el = next_elem(blk, L, U, curl);
        const int Nc = n / 2;
        const int64_t nagg = (int64_t)Nc * Nc * Nc;
        std::vector<int32_t> own(nagg, -1);   // explicit local solution per agglomerate
        std::vector<int64_t> todo;
        std::vector<CellW> next(nagg);
        for (int64_t t = 0; t < nagg; ++t) {
            const CellW* c[8];
            children(n, t, c);
            if (uniform_cells(c)) {
                next[t].nd = c[0]->nd;
                next[t].rt = c[0]->rt;
            } else {
                own[t] = (int32_t)todo.size();
                next[t].ex = (int32_t)todo.size();
                todo.push_back(t);
            }
        }
        std::vector<LocalP> Ls(todo.size());
        std::vector<CubeElem> nex(todo.size());
        if (!todo.empty()) {
            // the shared plan of the step, then every non-uniform agglomerate's weighted
            // problems from its hex weights: on the host, or (AMGE_BUILD_DEVICE) one
            // workgroup per agglomerate on the GPU
            const KuhnPlan plan = kuhn_plan(1.0 / n, B, U, curl);
            const int64_t na = (int64_t)todo.size();
            if (flags & AMGE_BUILD_DEVICE) {
                std::vector<double> w((size_t)na * 16);
                for (int64_t u = 0; u < na; ++u) {
                    const CellW* c[8];
                    children(n, todo[u], c);
                    for (int i = 0; i < 8; ++i) {
                        w[u * 16 + i] = c[i]->nd;
                        w[u * 16 + 8 + i] = c[i]->rt;
                    }
                }
                auto cat = [](const Mat* m, int k) {
                    std::vector<double> v;
                    for (int i = 0; i < k; ++i) v.insert(v.end(), m[i].a.begin(), m[i].a.end());
                    return v;
                };
                const std::vector<double> H = cat(plan.H, 8), h = cat(plan.h, 8), C = cat(plan.C, 8);
                const std::vector<double> Mn = curl ? cat(plan.Mn, 8) : std::vector<double>(),
                                          Fn = curl ? cat(plan.Fn, 8) : std::vector<double>(),
                                          Cn = curl ? cat(plan.Cn, 8) : std::vector<double>();
                KuhnPlanView v{curl ? 1 : 0, plan.nI, plan.nz, plan.nIn, plan.nzn, H.data(), h.data(), C.data(),
                               plan.up.a.data(), plan.Q2.a.data(), plan.CH.a.data(), plan.G0.a.data(),
                               plan.Wn.a.data(), plan.Q2n.a.data(), Mn.data(), Fn.data(), Cn.data()};
                std::vector<double> Uo((size_t)na * plan.nI * 6), er((size_t)na * 36);
                std::vector<double> Uno(curl ? (size_t)na * plan.nIn * 12 : 1), en(curl ? (size_t)na * 144 : 1);
                kuhn_local_device(v, w.data(), na, Uo.data(), er.data(), Uno.data(), en.data());
                parallel_for(na, [&](int64_t s, int64_t e) {
                    for (int64_t u = s; u < e; ++u) {
                        Ls[u] = plan.ref;
                        nex[u] = plan.ref_el;
                        for (int a = 0; a < plan.nI; ++a)
                            for (int F = 0; F < 6; ++F) Ls[u].rt(plan.fI[a], F) = Uo[((size_t)u * plan.nI + a) * 6 + F];
                        std::copy(er.begin() + u * 36, er.begin() + (u + 1) * 36, nex[u].rt.a.begin());
                        if (!curl) continue;
                        for (int a = 0; a < plan.nIn; ++a)
                            for (int E = 0; E < 12; ++E)
                                Ls[u].nd(plan.eI[a], E) = Uno[((size_t)u * plan.nIn + a) * 12 + E];
                        std::copy(en.begin() + u * 144, en.begin() + (u + 1) * 144, nex[u].nd.a.begin());
                    }
                });
            } else {
                parallel_for(na, [&](int64_t s, int64_t e) {
                    for (int64_t u = s; u < e; ++u) {
                        const CellW* c[8];
                        children(n, todo[u], c);
                        double wnd[8], wrt[8];
                        for (int i = 0; i < 8; ++i) { wnd[i] = c[i]->nd; wrt[i] = c[i]->rt; }
                        kuhn_solve_one(plan, wnd, wrt, Ls[u], nex[u]);
                    }
                });
            }
        }
        int32_t nfine = curl ? (int32_t)K.E.size() : (int32_t)K.F.size();
        auto fine_index = [&](const int q[3], int i) -> int32_t {
            int64_t off[3] = {2 * q[0], 2 * q[1], 2 * q[2]};
            auto gv = [&](int32_t bv) {
                auto c = B.coord(bv);
                return K.vid((int)(c[0] + off[0]), (int)(c[1] + off[1]), (int)(c[2] + off[2]));
            };
            if (curl) return K.edge(gv(B.E[i][0]), gv(B.E[i][1]));
            return K.face(gv(B.F[i][0]), gv(B.F[i][1]), gv(B.F[i][2]));
        };
        auto local_of = [&](int64_t t) -> const Mat& {
            const LocalP& lp = own[t] < 0 ? L : Ls[own[t]];
            return curl ? lp.nd : lp.rt;
        };
        clk.lap("local problems");
        pr.P.push_back(stamp(local_of, sdim, Nc, nfine, fine_index));
        clk.lap("prolongator assembly");
        cw.swap(next);
        ex.swap(nex);
    }
    // coarser levels: reference cube-complex block, and non-uniform agglomerates
    for (int k = 2; k < nlevels; ++k) {
        int Nf = n >> (k - 1);      // cubes per side on level k
        const CubeElem* ref8[8];
        std::array<double, 2> one8[8];
        for (int i = 0; i < 8; ++i) { ref8[i] = &el; one8[i] = {1.0, 1.0}; }
        Block blk = cube_block(ref8, one8, el, U);
        LocalP L = solve_block(blk, U, curl);
        CubeElem next_ref = next_elem(blk, L, U, curl);
        const int Nc = Nf / 2;
        const int64_t nagg = (int64_t)Nc * Nc * Nc;
        std::vector<int32_t> own(nagg, -1);
        std::vector<int64_t> todo;
        std::vector<CellW> next(nagg);
        for (int64_t t = 0; t < nagg; ++t) {
            const CellW* c[8];
            children(Nf, t, c);
            if (uniform_cells(c)) {
                next[t].nd = c[0]->nd;
                next[t].rt = c[0]->rt;
            } else {
                own[t] = (int32_t)todo.size();
                next[t].ex = (int32_t)todo.size();
                todo.push_back(t);
            }
        }
        std::vector<LocalP> Ls(todo.size());
        std::vector<CubeElem> nex(todo.size());
        parallel_for((int64_t)todo.size(), [&](int64_t s, int64_t e) {
            for (int64_t u = s; u < e; ++u) {
                const CellW* c[8];
                children(Nf, todo[u], c);
                const CubeElem* ce[8];
                std::array<double, 2> w[8];
                for (int i = 0; i < 8; ++i) {
                    if (c[i]->ex >= 0) { ce[i] = &ex[c[i]->ex]; w[i] = {1.0, 1.0}; }
                    else { ce[i] = &el; w[i] = {c[i]->nd, c[i]->rt}; }
                }
                Block b2 = cube_block(ce, w, el, U);
                Ls[u] = solve_block(b2, U, curl);
                nex[u] = next_elem(b2, Ls[u], U, curl);
            }
        });
        Cubes fineC(Nf), c2(2);
        // block entity descriptors (base, axis) in the 2x2x2 block's canonical order
        std::vector<std::array<int, 4>> bdesc;
        for (int64_t v = 0; v < c2.nV; ++v) {
            int p[3] = {(int)(v % 3), (int)((v / 3) % 3), (int)(v / 9)};
            if (curl) {
                for (int a = 0; a < 3; ++a) if (p[a] < 2) bdesc.push_back({p[0], p[1], p[2], a});
            } else {
                for (int a = 2; a >= 0; --a) if (Cubes::face_ok(2, p, a)) bdesc.push_back({p[0], p[1], p[2], a});
            }
        }
        auto fine_index = [&](const int q[3], int i) -> int32_t {
            int g[3] = {2 * q[0] + bdesc[i][0], 2 * q[1] + bdesc[i][1], 2 * q[2] + bdesc[i][2]};
            return curl ? fineC.edge(g, bdesc[i][3]) : fineC.face(g, bdesc[i][3]);
        };
        auto local_of = [&](int64_t t) -> const Mat& {
            const LocalP& lp = own[t] < 0 ? L : Ls[own[t]];
            return curl ? lp.nd : lp.rt;
        };
        clk.lap("local problems");
        pr.P.push_back(stamp(local_of, sdim, Nc, curl ? fineC.nE : fineC.nF, fine_index));
        clk.lap("prolongator assembly");
        el = next_ref;
        cw.swap(next);
        ex.swap(nex);
    }
    // Galerkin coarse matrices and coarse derivatives
    for (int k = 1; k < nlevels; ++k) {
        const Csr& P = pr.P[k - 1];
        if (flags & AMGE_BUILD_DEVICE) {
            pr.A.push_back(triple_on_device(transpose(P), pr.A[k - 1], P, nullptr));
        } else {
            Csr AP = spgemm(pr.A[k - 1], P);
            pr.A.push_back(spgemm(transpose(P), AP));
        }
        Cubes c(n >> k);
        pr.D.push_back(curl ? c.grad() : c.curl());
    }
    clk.lap("Galerkin products");
    if (flags & AMGE_BUILD_ESSENTIAL) {
        // every level restricted to the entities off the boundary: the system space (rows
        // and columns of A, rows of P and D) and the derivative's domain (columns of D)
        std::vector<std::vector<int32_t>> sm(nlevels), dm(nlevels);
        sm[0] = renumber(kuhn_boundary(K, sdim));
        dm[0] = renumber(kuhn_boundary(K, sdim - 1));
        for (int k = 1; k < nlevels; ++k) {
            Cubes c(n >> k);
            sm[k] = renumber(cubes_boundary(c, sdim));
            dm[k] = renumber(cubes_boundary(c, sdim - 1));
        }
        for (int k = 0; k < nlevels; ++k) {
            pr.A[k] = restrict_csr(pr.A[k], sm[k], sm[k]);
            pr.D[k] = restrict_csr(pr.D[k], sm[k], dm[k]);
            if (k + 1 < nlevels) pr.P[k] = restrict_csr(pr.P[k], sm[k], sm[k + 1]);
        }
    }
    return pr;
}

}  // namespace
}  // namespace amge

struct amge_problem {
    amge::Problem p;
    amge::Csr empty;
};

extern "C" amge_status amge_kuhn_build(int32_t kind, int32_t n, int32_t nlevels, const double* alpha_hex,
                                       const double* beta_hex, int32_t flags, amge_problem** out) {
    try {
        if (!out) amge::fail(AMGE_ERR_ARG, "null output pointer");
        auto* pp = new amge_problem;
        try {
            pp->p = amge::build(kind, n, nlevels, alpha_hex, beta_hex, flags);
        } catch (...) {
            delete pp;
            throw;
        }
        pp->empty.nrows = 0;
        pp->empty.ncols = 0;
        *out = pp;
        return AMGE_OK;
    } catch (const amge::Error& e) {
        amge::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        amge::set_last_error("host allocation failed");
        return AMGE_ERR_OOM;
    } catch (const std::exception& e) {
        amge::set_last_error(e.what());
        return AMGE_ERR_ARG;
    }
}

extern "C" int32_t amge_problem_nlevels(const amge_problem* p) { return p ? p->p.nlevels : 0; }

extern "C" amge_status amge_problem_levels(const amge_problem* p, amge_level* levels) {
    if (!p || !levels) {
        amge::set_last_error("null argument");
        return AMGE_ERR_ARG;
    }
    for (int k = 0; k < p->p.nlevels; ++k) {
        levels[k].A = p->p.A[k].view();
        levels[k].D = p->p.D[k].view();
        levels[k].P = k + 1 < p->p.nlevels ? p->p.P[k].view() : p->empty.view();
        if (k + 1 == p->p.nlevels) levels[k].P.ncols = 0;
    }
    return AMGE_OK;
}

extern "C" void amge_problem_free(amge_problem* p) { delete p; }
