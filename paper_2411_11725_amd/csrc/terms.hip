// Term generator: element matrices of the quadratic energy terms, integrated
// from the Q1 basis by Gauss quadrature, reduced to the neighbour weights the
// fused node kernel applies (Sec. 5.1: the paper's form compiler turns a
// term's weak form into per-cell tensor operations by Gauss quadrature over
// the element; here the same integration produces the small tables a
// hand-written gather kernel needs).
//
// On a cuboid cell of edges h the trilinear functions phi_a (a in {0,1}^3)
// and the 2-point Gauss rule per axis (exact for every product of two Q1
// functions or their derivatives) give
//   M_ab   = int phi_a phi_b                      (mass: anisotropy, lumping)
//   K_ab   = int grad phi_a . grad phi_b          (exchange)
//   G^k_ab = int phi_a d_k phi_b,  A^k = G^k - G^k^T   (antisymmetric exchange)
// The node kernel gathers node n's gradient from its 26 neighbours, so each
// matrix must reduce to numbers indexed by the neighbour offset d = b - a:
//   M_ab, K_ab   depend only on which axes differ (mask = a ^ b)   -> Mp[8], Kp[8]
//   A^k_ab       = d_k times a number set by which other axes differ -> g_k[4]
// The generator checks every pair (a, b) against that reduction and fails if
// a term does not have the structure the kernel assumes.  It also emits the
// 1D basis values at the Gauss points and the point weight, which the kernel
// uses to integrate the quartic cubic-anisotropy density.
#include <cmath>
#include <string>

#include "nm_internal.h"

namespace nm {

namespace {

// 1D linear hat on [0, h]: psi_0 = 1 - x/h, psi_1 = x/h
double psi(int i, double x, double h) { return i ? x / h : 1.0 - x / h; }
double dpsi(int i, double h) { return i ? 1.0 / h : -1.0 / h; }

bool close(double a, double b, double scale) { return std::fabs(a - b) <= 1e-12 * scale; }

}  // namespace

bool generate_element_tables(const double h[3], ElementTables *out, std::string *why) {
    const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    double M[8][8] = {}, K[8][8] = {}, G[3][8][8] = {};
    const double w = h[0] * h[1] * h[2] / 8.0;   // Gauss weight per point
    for (int g = 0; g < 8; ++g) {
        const double x[3] = {gp[g & 1] * h[0], gp[(g >> 1) & 1] * h[1], gp[g >> 2] * h[2]};
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) {
                double pa[3], pb[3];
                for (int k = 0; k < 3; ++k) {
                    pa[k] = psi((a >> k) & 1, x[k], h[k]);
                    pb[k] = psi((b >> k) & 1, x[k], h[k]);
                }
                const double fa = pa[0] * pa[1] * pa[2], fb = pb[0] * pb[1] * pb[2];
                M[a][b] += w * fa * fb;
                for (int k = 0; k < 3; ++k) {
                    // d_k phi = psi' along k times the other two factors
                    double da = dpsi((a >> k) & 1, h[k]), db = dpsi((b >> k) & 1, h[k]);
                    for (int l = 0; l < 3; ++l)
                        if (l != k) {
                            da *= pa[l];
                            db *= pb[l];
                        }
                    K[a][b] += w * da * db;
                    G[k][a][b] += w * fa * db;
                }
            }
    }
    double smax = 0.0, kmax = 0.0, gmax = 0.0;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            smax = std::fmax(smax, std::fabs(M[a][b]));
            kmax = std::fmax(kmax, std::fabs(K[a][b]));
            for (int k = 0; k < 3; ++k) gmax = std::fmax(gmax, std::fabs(G[k][a][b]));
        }
    // reduction by axis-difference pattern (first pair of each pattern sets it)
    bool set[8] = {};
    double Kp[8] = {}, Mp[8] = {}, gk[3][4] = {};
    bool gset[3][4] = {};
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            const int mask = a ^ b;
            if (!set[mask]) {
                Kp[mask] = K[a][b];
                Mp[mask] = M[a][b];
                set[mask] = true;
            } else if (!close(K[a][b], Kp[mask], kmax) || !close(M[a][b], Mp[mask], smax)) {
                if (why) *why = "element matrices are not functions of the axis-difference pattern";
                return false;
            }
            for (int k = 0; k < 3; ++k) {
                const double A = G[k][a][b] - G[k][b][a];
                const int dk = ((b >> k) & 1) - ((a >> k) & 1);
                const int l1 = (k + 1) % 3, l2 = (k + 2) % 3;
                // which of the two other axes differ, in increasing axis order
                const int lo = l1 < l2 ? l1 : l2, hi = l1 < l2 ? l2 : l1;
                const int i = ((mask >> lo) & 1) + 2 * ((mask >> hi) & 1);
                if (dk == 0) {
                    if (!close(A, 0.0, gmax)) {
                        if (why) *why = "antisymmetric part does not vanish between equal coordinates";
                        return false;
                    }
                    continue;
                }
                const double v = A / dk;
                if (!gset[k][i]) {
                    gk[k][i] = v;
                    gset[k][i] = true;
                } else if (!close(v, gk[k][i], gmax)) {
                    if (why) *why = "antisymmetric part is not d_k times a pattern factor";
                    return false;
                }
            }
        }
    for (int i = 0; i < 8; ++i) {
        out->Kp[i] = (float)Kp[i];
        out->Mp[i] = (float)Mp[i];
    }
    for (int i = 0; i < 4; ++i) {
        out->gx[i] = (float)gk[0][i];
        out->gy[i] = (float)gk[1][i];
        out->gz[i] = (float)gk[2][i];
    }
    out->gq[0] = (float)gp[0];
    out->gq[1] = (float)gp[1];
    out->gw = (float)w;
    return true;
}

}  // namespace nm
