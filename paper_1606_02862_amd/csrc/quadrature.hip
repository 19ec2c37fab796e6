// 64-point Gauss-Laguerre rule (weight e^{-x} on [0, inf)) for the
// Maxwellian average of the Lotz cross-section, computed on the host.
//
// Golub & Welsch (Math. Comp. 23, 1969): the nodes are the eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the Laguerre recurrence (diagonal
// 2k+1, off-diagonal k) and the weights the squared first components of its
// normalised eigenvectors.  The eigenproblem is solved by the implicit-shift
// QL algorithm for symmetric tridiagonal matrices (Bowdler, Martin, Reinsch &
// Wilkinson, Numer. Math. 11, 1968; EISPACK tql1/tql2): Wilkinson shift from
// the leading 2x2 block, a sweep of plane rotations that chases the bulge,
// and a restart where an off-diagonal element underflows.  Only the first row
// of the accumulated rotations is kept, which is all the weights need.  Each node
// is then polished by Newton steps on L_n evaluated with the three-term
// recurrence, and the weights are recomputed as x / ((n+1) L_{n+1}(x))^2,
// which keeps full relative accuracy for the tiny weights of the large nodes.
#include <cmath>
#include <mutex>

#include "ionize_internal.hpp"

namespace pic {
namespace {

typedef long double ld;

// L_n(x) and L_{n-1}(x) by (k+1) L_{k+1} = (2k+1-x) L_k - k L_{k-1}.
void laguerre(int n, ld x, ld* ln, ld* lnm1)
{
    ld a = 1.0L, b = 1.0L - x;  // L_0, L_1
    if (n == 0) { *ln = a; *lnm1 = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
        const ld c = ((2 * k + 1 - x) * b - k * a) / (k + 1);
        a = b;
        b = c;
    }
    *ln = b;
    *lnm1 = a;
}

void golub_welsch(int n, ld* d, ld* z)
{
    ld e[GL_NODES];
    for (int i = 0; i < n; ++i) {
        d[i] = 2 * i + 1;
        e[i] = (i + 1 < n) ? (ld)(i + 1) : 0.0L;
        z[i] = (i == 0) ? 1.0L : 0.0L;
    }
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                const ld dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-19L * dd) break;
            }
            if (m == l) break;
            // Wilkinson-like shift from the leading 2x2 block
            ld g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            ld r = std::hypot(g, 1.0L);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            ld s = 1.0L, c = 1.0L, p = 0.0L;
            int i = m - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                ld f = s * e[i];
                const ld b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {
                    d[i + 1] -= p;
                    e[m] = 0.0L;
                    underflow = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // first row of the accumulated rotations
                f = z[i + 1];
                z[i + 1] = s * z[i] + c * f;
                z[i] = c * z[i] - s * f;
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0L;
        }
    }
}

struct Rule {
    double x[GL_NODES], w[GL_NODES];
};

Rule compute_rule()
{
    const int n = GL_NODES;
    ld d[GL_NODES], z[GL_NODES];
    golub_welsch(n, d, z);
    // sort ascending (with the eigenvector components)
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && d[j - 1] > d[j]; --j) {
            std::swap(d[j - 1], d[j]);
            std::swap(z[j - 1], z[j]);
        }
    Rule r;
    for (int i = 0; i < n; ++i) {
        ld x = d[i];
        for (int it = 0; it < 4; ++it) {
            ld ln, lm;
            laguerre(n, x, &ln, &lm);
            const ld dln = n * (ln - lm) / x;  // x L_n' = n (L_n - L_{n-1})
            x -= ln / dln;
        }
        ld ln1, ln;
        laguerre(n + 1, x, &ln1, &ln);
        r.x[i] = (double)x;
        r.w[i] = (double)(x / ((ld)(n + 1) * (n + 1) * ln1 * ln1));
    }
    return r;
}

}  // namespace

const double* gauss_laguerre_nodes(const double** weights)
{
    static Rule rule;
    static std::once_flag once;
    std::call_once(once, [] { rule = compute_rule(); });
    *weights = rule.w;
    return rule.x;
}

}  // namespace pic

extern "C" int pic_gauss_laguerre64(double* nodes, double* weights)
{
    if (!nodes || !weights) return PIC_ERR_ARG;
    const double* w;
    const double* x = pic::gauss_laguerre_nodes(&w);
    for (int i = 0; i < pic::GL_NODES; ++i) {
        nodes[i] = x[i];
        weights[i] = w[i];
    }
    return PIC_OK;
}
