// Translation operators of the solid-harmonic FMM, built once per key in FP64 on the
// host and kept on the device for the life of the process (Sec. 2.2: translation
// operators stored as matrices acting on coefficient vectors, precomputed; boxes with
// the same relative position share one operator).
//
// Basis (scaled complex solid harmonics, m = -l..l):
//   R_00 = 1,  R_mm = -(x + i y)/(2m) R_{m-1,m-1},
//   R_{l+1,m} = ((2l+1) z R_lm - r^2 R_{l-1,m}) / ((l+m+1)(l-m+1))
//   I_00 = 1/r, I_mm = -(2m-1)(x + i y)/r^2 I_{m-1,m-1},
//   I_{l+1,m} = ((2l+1) z I_lm - (l^2 - m^2) I_{l-1,m}) / r^2
//   X_{l,-m} = (-1)^m conj(X_lm) for both.
// With these, for |s| < |D|:
//   1/|t - s|  = sum_lm conj(R_lm(s)) I_lm(t)
//   R_lm(a + b) = sum_jk R_jk(a) R_{l-j,m-k}(b)
//   I_jk(D + s) = sum_lm (-1)^l conj(R_lm(s)) I_{j+l,k+m}(D)
// Multipole of a cell c with side s_c:  Mt_lm = sum_i q_i conj(R_lm((x_i - c)/s_c))
//   (the field is sum_lm s_c^l Mt_lm I_lm(x - c)).
// Local expansion: phi(c + t) = (1/s_c) sum_jk Lt_jk conj(R_jk(t/s_c)).
// In this scaled basis
//   M2L (B -> A, D = c_B - c_A): Lt_jk = sum_lm (-1)^l s_A^(j+1) s_B^l I_{j+l,k+m}(D) Mt_lm
//   M2M (child c -> parent P, d = c_c - c_P): Mt_P,lm = sum_jk conj(R_jk(d/s_P)) 2^-(l-j) Mt_c,(l-j)(m-k)
//   L2L (parent P -> child c, d = c_c - c_P): Lt_c,ab = sum_jk Lt_P,jk conj(R_{j-a,k-b}(d/s_P)) 2^-(a+1)
// The M2L factor depends only on the level difference and on D in units of the finer
// cell's half side h, because s_A, s_B and D all scale with h; so one matrix serves
// every level (translation invariance).  M2M/L2L need eight matrices (one per octant).
//
// Real storage of a coefficient vector of order p, (p+1)^2 reals: degree l occupies
// [l^2, (l+1)^2): Re X_l0, then (Re X_lm, Im X_lm) for m = 1..l.  Negative orders are
// implied by the symmetry above (the fields are real).
#include <algorithm>
#include <complex>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "fmm_internal.h"

namespace fmm {
namespace {

using cd = std::complex<double>;

inline int tri(int l, int m) { return l * (l + 1) / 2 + m; }

struct Harm {
    int P;
    std::vector<cd> v;   // tri(l, m), m >= 0
    cd get(int l, int m) const {
        if (l < 0 || m > l || -m > l) return 0.0;
        if (m >= 0) return v[tri(l, m)];
        cd c = std::conj(v[tri(l, -m)]);
        return (m & 1) ? -c : c;
    }
};

Harm regular(double x, double y, double z, int P) {
    Harm h{P, std::vector<cd>(tri(P, P) + 1)};
    double r2 = x * x + y * y + z * z;
    h.v[0] = 1.0;
    for (int m = 1; m <= P; ++m) h.v[tri(m, m)] = -cd(x, y) / (2.0 * m) * h.v[tri(m - 1, m - 1)];
    for (int m = 0; m < P; ++m) {
        h.v[tri(m + 1, m)] = z * h.v[tri(m, m)];
        for (int l = m + 1; l < P; ++l)
            h.v[tri(l + 1, m)] = ((2.0 * l + 1) * z * h.v[tri(l, m)] - r2 * h.v[tri(l - 1, m)]) /
                                 (double((l + m + 1) * (l - m + 1)));
    }
    return h;
}

Harm irregular(double x, double y, double z, int P) {
    Harm h{P, std::vector<cd>(tri(P, P) + 1)};
    double r2 = x * x + y * y + z * z;
    h.v[0] = 1.0 / std::sqrt(r2);
    for (int m = 1; m <= P; ++m) h.v[tri(m, m)] = -(2.0 * m - 1) * cd(x, y) / r2 * h.v[tri(m - 1, m - 1)];
    for (int m = 0; m < P; ++m) {
        h.v[tri(m + 1, m)] = (2.0 * m + 1) * z * h.v[tri(m, m)] / r2;
        for (int l = m + 1; l < P; ++l)
            h.v[tri(l + 1, m)] = ((2.0 * l + 1) * z * h.v[tri(l, m)] - double(l * l - m * m) * h.v[tri(l - 1, m)]) / r2;
    }
    return h;
}

inline int ridx(int l, int m, int im) { return m == 0 ? l * l : l * l + 2 * m - 1 + im; }

// Build the real matrix of a complex-linear map given as: for an input basis
// element with nonzero entries at (l, m) and (l, -m), `apply(l, m, val)` adds
// val * (column of the complex map for input (l, m)) into Y (indexed tri(j,k), k >= 0).
template <class Col>
void real_matrix(int p, int RP, int KP, bool transposed, std::vector<double> &A, Col col) {
    A.assign((size_t)RP * KP, 0.0);
    std::vector<cd> Y(tri(p, p) + 1);
    for (int l = 0; l <= p; ++l)
        for (int m = 0; m <= l; ++m)
            for (int im = 0; im < (m == 0 ? 1 : 2); ++im) {
                std::fill(Y.begin(), Y.end(), cd(0.0));
                cd xv = im ? cd(0, 1) : cd(1, 0);
                col(l, m, xv, Y);
                if (m > 0) {
                    cd xn = std::conj(xv);
                    if (m & 1) xn = -xn;
                    col(l, -m, xn, Y);
                }
                int c = ridx(l, m, im);
                for (int j = 0; j <= p; ++j)
                    for (int k = 0; k <= j; ++k) {
                        int r = ridx(j, k, 0);
                        double vr = Y[tri(j, k)].real();
                        if (transposed) A[(size_t)c * RP + r] = vr; else A[(size_t)r * KP + c] = vr;
                        if (k > 0) {
                            double vi = Y[tri(j, k)].imag();
                            if (transposed) A[(size_t)c * RP + r + 1] = vi; else A[(size_t)(r + 1) * KP + c] = vi;
                        }
                    }
            }
}

// FP32 copy of a KP x KP operator in the layout the MFMA GEMM reads: inside every
// 16-wide chunk of columns, position 16 c + 4 a + b holds column 16 c + 4 b + a (a 4 x 4
// transpose), so that each of the GEMM's four k steps of a chunk covers four consecutive
// columns and a step whose columns are all padding can be left out.
void to_gemm_layout(const std::vector<double> &A, int KP, float *dst) {
    for (int r = 0; r < KP; ++r)
        for (int c = 0; c < KP; c += 16)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    dst[(size_t)r * KP + c + 4 * a + b] = (float)A[(size_t)r * KP + c + 4 * b + a];
}

void build_m2l(int p, uint64_t key, std::vector<double> &A) {
    int dl;
    int64_t nx, ny, nz;
    unpack_key(key, dl, nx, ny, nz);
    // sigma = side / h for each cell: the finer cell has side 2h.
    double sA = dl >= 0 ? std::ldexp(1.0, dl + 1) : 2.0;    // dl = level(B) - level(A)
    double sB = dl <= 0 ? std::ldexp(1.0, -dl + 1) : 2.0;
    Harm I = irregular((double)nx, (double)ny, (double)nz, 2 * p);
    int KP = ncoef_pad(p);
    std::vector<double> pa(p + 2), pb(2 * p + 2);
    for (int j = 0; j <= p + 1; ++j) pa[j] = std::pow(sA, j);
    for (int l = 0; l <= p; ++l) pb[l] = std::pow(sB, l);
    real_matrix(p, KP, KP, false, A, [&](int l, int m, cd xv, std::vector<cd> &Y) {
        double sgn = (l & 1) ? -1.0 : 1.0;
        for (int j = 0; j <= p; ++j)
            for (int k = 0; k <= j; ++k)
                Y[tri(j, k)] += sgn * pa[j + 1] * pb[l] * xv * I.get(j + l, k + m);
    });
}

void build_m2m(int p, int oct, std::vector<double> &A) {
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = ((oct >> (2 - a)) & 1) ? 0.25 : -0.25;
    Harm R = regular(d[0], d[1], d[2], p);
    int KP = ncoef_pad(p);
    real_matrix(p, KP, KP, false, A, [&](int lc, int mc, cd xv, std::vector<cd> &Y) {
        double sc = std::ldexp(1.0, -lc);
        for (int l = lc; l <= p; ++l)
            for (int m = 0; m <= l; ++m) Y[tri(l, m)] += std::conj(R.get(l - lc, m - mc)) * sc * xv;
    });
}

void build_l2l(int p, int oct, std::vector<double> &A) {
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = ((oct >> (2 - a)) & 1) ? 0.25 : -0.25;
    Harm R = regular(d[0], d[1], d[2], p);
    int KP = ncoef_pad(p);
    real_matrix(p, KP, KP, false, A, [&](int j, int k, cd xv, std::vector<cd> &Y) {
        for (int a = 0; a <= j; ++a) {
            double sc = std::ldexp(1.0, -(a + 1));
            for (int b = 0; b <= a; ++b) Y[tri(a, b)] += xv * std::conj(R.get(j - a, k - b)) * sc;
        }
    });
}

void transpose_into(const std::vector<double> &A, int KP, double *out) {
    for (int r = 0; r < KP; ++r)
        for (int c = 0; c < KP; ++c) out[(size_t)c * KP + r] = A[(size_t)r * KP + c];
}

// Normalisation of the multipole coefficients for FP16: nu_lm = sqrt((l+m)! (l-m)!)
// brings every |nu_lm R_lm(u)| below |u|^l <= 1 (applied to Re and Im alike).
double nu_coef(int l, int m) { return std::sqrt(std::tgamma(l + m + 1.0) * std::tgamma(l - m + 1.0)); }

std::vector<double> nu_vector(int p, int KP) {
    std::vector<double> nu(KP, 1.0);
    for (int l = 0; l <= p; ++l)
        for (int m = 0; m <= l; ++m) {
            nu[ridx(l, m, 0)] = nu_coef(l, m);
            if (m > 0) nu[ridx(l, m, 1)] = nu_coef(l, m);
        }
    return nu;
}

// Split-FP16 form of an M2L operator A ([KP][KP], row-major, acting on the FP32 basis):
// with the multipoles normalised as Mh = nu * M, A M = diag(rs) (H + Lo) Mh where
// A' = diag(1/rs) A diag(1/nu), rs = power of two bringing each row maximum into [1, 2),
// H = fp16(A'), Lo = fp16(A' - H).  Layout: H [KP][KP] half, Lo [KP][KP] half, rs [KP] float.
size_t split16_bytes(int KP) { return (size_t)KP * KP * 2 * sizeof(_Float16) + (size_t)KP * sizeof(float); }

void split16(const std::vector<double> &A, int p, int KP, std::vector<char> &out) {
    out.assign(split16_bytes(KP), 0);
    std::vector<double> nu = nu_vector(p, KP), rs(KP, 1.0), B(A);
    auto pow2floor = [](double v) { int e; std::frexp(v, &e); return std::ldexp(1.0, e - 1); };
    for (int r = 0; r < KP; ++r) {
        double m = 0;
        for (int c = 0; c < KP; ++c) {
            B[(size_t)r * KP + c] /= nu[c];
            m = std::max(m, std::fabs(B[(size_t)r * KP + c]));
        }
        if (m > 0) rs[r] = pow2floor(m);
        for (int c = 0; c < KP; ++c) B[(size_t)r * KP + c] /= rs[r];
    }
    _Float16 *H = reinterpret_cast<_Float16 *>(out.data());
    _Float16 *Lo = H + (size_t)KP * KP;
    float *rsf = reinterpret_cast<float *>(Lo + (size_t)KP * KP);
    for (size_t i = 0; i < (size_t)KP * KP; ++i) {
        _Float16 h = (_Float16)B[i];
        H[i] = h;
        Lo[i] = (_Float16)(B[i] - (double)h);
    }
    for (int i = 0; i < KP; ++i) rsf[i] = (float)rs[i];
}

// Size of every 16 x 16 block of an M2L operator A ([KP][KP], rows = local coefficient of
// the target, columns = multipole coefficient of the source), measured by what the block
// can add to a potential: a multipole coefficient of degree n is at most h^n / nu_nm
// times the source cell's total |charge| (its bodies lie within h = sqrt(3)/2 of the
// centre, in units of the side), and a local coefficient of degree j reaches the
// potential with a weight of at most h^j / nu_jk.  Returned: for every block, the sum of
// |w_r A_rc w_c| over the block, divided by |w_0 A_00 w_0| (the monopole-to-monopole
// term, i.e. the size of the whole interaction).
// Bound weights of the coefficients: h^l / nu_lm (h = sqrt(3)/2), zero on the padding.
std::vector<double> bound_weights(int p, int KP) {
    const double h = std::sqrt(3.0) / 2;
    std::vector<double> nu = nu_vector(p, KP), w(KP, 0.0);
    for (int l = 0; l <= p; ++l)
        for (int m = 0; m <= l; ++m) {
            w[ridx(l, m, 0)] = std::pow(h, l) / nu[ridx(l, m, 0)];
            if (m > 0) w[ridx(l, m, 1)] = std::pow(h, l) / nu[ridx(l, m, 1)];
        }
    return w;
}

std::vector<float> block_sums(const std::vector<double> &A, int p, int KP) {
    const int NB = KP / 16;
    std::vector<double> w = bound_weights(p, KP);
    std::vector<double> b((size_t)NB * NB, 0.0);
    for (int r = 0; r < KP; ++r)
        for (int c = 0; c < KP; ++c) b[(size_t)(r / 16) * NB + c / 16] += std::fabs(w[r] * A[(size_t)r * KP + c] * w[c]);
    const double ref = std::fabs(A[0]);
    std::vector<float> out(b.size());
    for (size_t i = 0; i < b.size(); ++i) out[i] = ref > 0 ? (float)(b[i] / ref) : 1.f;
    return out;
}

// ------------------------------------------------------------------ SVD-compressed M2L
// Low-rank form of an M2L operator (Sec. 2.2: an SVD of the translation matrices gives what
// expansions of varying order give, systematically).  The SVD is taken of the weighted
// operator B = W A W, W = diag(bound weights): a multipole coefficient of degree n is at most
// h^n / nu_nm times the source's total |charge| and a local coefficient of degree j reaches
// the potential with at most the same weight, so B's singular values measure what each
// direction can add to a potential.  Singular values at or below tol * sigma_1 are dropped;
// A ~ (W^-1 U_r Sigma_r) (V_r^T W^-1) = Pf Qf, applied as two skinny products: Y = Qf M
// (r x KP times KP), then L += Pf Y.
//
// The SVD: Householder QR with column pivoting of B, stopped once every remaining column
// is below tol * (largest column norm) / sqrt(n) (so the dropped part is below tol * sigma_1),
// then one-sided Jacobi (Hestenes) rotations on the transposed triangular factor.
struct SvdFactor {
    int r = 0;                     // rank kept
    std::vector<double> Pf, Qf;    // [n][r] and [r][n] (n = coefficient count)
};

SvdFactor svd_factor(const std::vector<double> &A, int p, int KP, double tol) {
    const int n = ncoef(p);
    std::vector<double> w = bound_weights(p, KP);
    // B column-major (n x n)
    std::vector<double> B((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) B[i + (size_t)j * n] = w[i] * A[(size_t)i * KP + j] * w[j];
    std::vector<int> piv(n);
    for (int j = 0; j < n; ++j) piv[j] = j;
    std::vector<double> cn(n);
    auto colnorm2 = [&](int j, int from) {
        double t = 0;
        for (int i = from; i < n; ++i) t += B[i + (size_t)j * n] * B[i + (size_t)j * n];
        return t;
    };
    double cmax = 0;
    for (int j = 0; j < n; ++j) { cn[j] = colnorm2(j, 0); cmax = std::max(cmax, cn[j]); }
    const double stop2 = (tol * std::sqrt(cmax)) * (tol * std::sqrt(cmax)) / n;
    std::vector<std::vector<double>> refl;   // Householder vectors (length n - j), beta folded in
    std::vector<double> betas;
    int k = 0;
    for (int j = 0; j < n; ++j) {
        int pc = j;
        for (int c = j + 1; c < n; ++c)
            if (cn[c] > cn[pc]) pc = c;
        if (cn[pc] <= stop2 || cn[pc] == 0) break;
        if (pc != j) {
            for (int i = 0; i < n; ++i) std::swap(B[i + (size_t)j * n], B[i + (size_t)pc * n]);
            std::swap(cn[j], cn[pc]);
            std::swap(piv[j], piv[pc]);
        }
        // reflector zeroing B(j+1:n, j)
        std::vector<double> v(n - j);
        double alpha = 0;
        for (int i = j; i < n; ++i) { v[i - j] = B[i + (size_t)j * n]; alpha += v[i - j] * v[i - j]; }
        alpha = std::sqrt(alpha);
        if (v[0] > 0) alpha = -alpha;
        v[0] -= alpha;
        double vn = 0;
        for (double x : v) vn += x * x;
        const double beta = vn > 0 ? 2.0 / vn : 0.0;
        for (int c = j; c < n; ++c) {
            double d = 0;
            for (int i = j; i < n; ++i) d += v[i - j] * B[i + (size_t)c * n];
            d *= beta;
            for (int i = j; i < n; ++i) B[i + (size_t)c * n] -= d * v[i - j];
        }
        refl.push_back(std::move(v));
        betas.push_back(beta);
        for (int c = j + 1; c < n; ++c) cn[c] = colnorm2(c, j + 1);
        k = j + 1;
    }
    SvdFactor f;
    if (k == 0) return f;
    // explicit Q (n x k, column-major): reflectors applied to the first k unit columns
    std::vector<double> Q((size_t)n * k, 0.0);
    for (int c = 0; c < k; ++c) {
        Q[c + (size_t)c * n] = 1.0;
        for (int j = k - 1; j >= 0; --j) {
            const std::vector<double> &v = refl[j];
            double d = 0;
            for (int i = j; i < n; ++i) d += v[i - j] * Q[i + (size_t)c * n];
            d *= betas[j];
            for (int i = j; i < n; ++i) Q[i + (size_t)c * n] -= d * v[i - j];
        }
    }
    // X = R^T (n x k, column-major; row index = pivoted column position), V = I (k x k)
    std::vector<double> X((size_t)n * k, 0.0), V((size_t)k * k, 0.0);
    for (int c = 0; c < k; ++c)
        for (int i = c; i < n; ++i) X[i + (size_t)c * n] = B[c + (size_t)i * n];
    for (int c = 0; c < k; ++c) V[c + (size_t)c * k] = 1.0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool rotated = false;
        for (int a = 0; a < k - 1; ++a)
            for (int b = a + 1; b < k; ++b) {
                double al = 0, be = 0, ga = 0;
                for (int i = 0; i < n; ++i) {
                    const double xa = X[i + (size_t)a * n], xb = X[i + (size_t)b * n];
                    al += xa * xa;
                    be += xb * xb;
                    ga += xa * xb;
                }
                if (std::fabs(ga) <= 1e-15 * std::sqrt(al * be) || ga == 0) continue;
                rotated = true;
                const double zeta = (be - al) / (2 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
                const double cs = 1 / std::sqrt(1 + t * t), sn = cs * t;
                for (int i = 0; i < n; ++i) {
                    const double xa = X[i + (size_t)a * n], xb = X[i + (size_t)b * n];
                    X[i + (size_t)a * n] = cs * xa - sn * xb;
                    X[i + (size_t)b * n] = sn * xa + cs * xb;
                }
                for (int i = 0; i < k; ++i) {
                    const double va = V[i + (size_t)a * k], vb = V[i + (size_t)b * k];
                    V[i + (size_t)a * k] = cs * va - sn * vb;
                    V[i + (size_t)b * k] = sn * va + cs * vb;
                }
            }
        if (!rotated) break;
    }
    // X V = U Sigma: sigma_c = |X_c|; R = V Sigma U^T; B ~ (Q V) Sigma (Pi U)^T
    std::vector<std::pair<double, int>> sig(k);
    for (int c = 0; c < k; ++c) {
        double t = 0;
        for (int i = 0; i < n; ++i) t += X[i + (size_t)c * n] * X[i + (size_t)c * n];
        sig[c] = {std::sqrt(t), c};
    }
    std::sort(sig.begin(), sig.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first > y.first;
    });
    int r = 0;
    while (r < k && sig[r].first > tol * sig[0].first) ++r;
    f.r = r;
    f.Pf.assign((size_t)n * r, 0.0);
    f.Qf.assign((size_t)r * n, 0.0);
    for (int q = 0; q < r; ++q) {
        const int c = sig[q].second;
        const double sv = sig[q].first;
        // left vector: Q V_c (n), scaled by sigma and un-weighted
        for (int i = 0; i < n; ++i) {
            double t = 0;
            for (int j = 0; j < k; ++j) t += Q[i + (size_t)j * n] * V[j + (size_t)c * k];
            f.Pf[(size_t)i * r + q] = t * sv / w[i];
        }
        // right vector: U_c = X_c / sigma in pivoted positions, back to column order, un-weighted
        for (int i = 0; i < n; ++i) f.Qf[(size_t)q * n + piv[i]] = X[i + (size_t)c * n] / sv / w[piv[i]];
    }
    return f;
}

// GEMM layouts of a factor pair with the rank padded to rp (a multiple of 16): Qf as
// [rp][KP] and Pf as [KP][rp], both with the 4 x 4 transpose inside every 16-wide chunk of
// columns (see to_gemm_layout); padding is zero.
void svd_gemm_layout(const SvdFactor &f, int p, int KP, int rp, float *dst) {
    const int n = ncoef(p), r = f.r;
    float *q = dst, *pp = dst + (size_t)rp * KP;
    std::fill(dst, dst + (size_t)2 * rp * KP, 0.f);
    auto tpos = [](int c) { return 16 * (c / 16) + 4 * (c % 4) + (c % 16) / 4; };
    for (int a = 0; a < r; ++a)
        for (int c = 0; c < n; ++c) q[(size_t)a * KP + tpos(c)] = (float)f.Qf[(size_t)a * n + c];
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < r; ++a) pp[(size_t)i * rp + tpos(a)] = (float)f.Pf[(size_t)i * r + a];
}

// ------------------------------------------------------------------ device store
constexpr int kChunk = 64;   // matrices per device allocation (never moved)

// Device memory for operators, handed out in fixed-size blocks from chunks that are
// never moved or freed (pointers stay valid for the process).
struct BlockPool {
    size_t block_bytes = 0;
    std::vector<char *> chunks;
    int used = kChunk;
    // `fresh` (if given) tells whether the block opens a new chunk
    void *take(bool *fresh = nullptr) {
        if (fresh) *fresh = used == kChunk;
        if (used == kChunk) {
            char *c = nullptr;
            HIP_CHECK(hipMalloc(&c, block_bytes * kChunk));
            chunks.push_back(c);
            used = 0;
        }
        return chunks.back() + block_bytes * (used++);
    }
};

// Device memory for variable-size blocks (SVD factors): bump allocation inside 64 MB
// chunks that are never moved or freed.
struct Arena {
    std::vector<char *> chunks;
    size_t used = 0, cap = 0;
    void *take(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        if (chunks.empty() || used + bytes > cap) {
            const size_t sz = std::max(bytes, size_t(64) << 20);
            char *c = nullptr;
            HIP_CHECK(hipMalloc(&c, sz));
            chunks.push_back(c);
            used = 0;
            cap = sz;
        }
        void *r = chunks.back() + used;
        used += bytes;
        return r;
    }
};

struct SvdEntry {
    uint64_t q = 0, pp = 0;   // device pointers of Qf [rp][KP] and Pf [KP][rp]
    int32_t r = 0, rp = 0;
};

struct Store {
    int p = -1;
    size_t mat_floats = 0;
    std::map<std::pair<uint64_t, double>, SvdEntry> svd;   // (key, tolerance) -> factors
    Arena svd_arena;
    std::unordered_map<uint64_t, uint64_t> f32;   // key -> device pointer
    std::unordered_map<uint64_t, uint64_t> f16;   // key -> device pointer (split FP16 form)
    std::unordered_map<uint64_t, uint64_t> f64;   // key -> device pointer (FP64, transposed)
    std::unordered_map<uint64_t, std::vector<float>> bsum;   // key -> weighted block sums (see block_sums)
    BlockPool pool32, pool16, pool64;
    OpTables tables;
    float *alloc_matrix(bool *fresh = nullptr) { return static_cast<float *>(pool32.take(fresh)); }
};

std::mutex g_mu;
std::unordered_map<int, Store> g_store;   // (device * 32 + p) -> store

Store &store_for(int p) {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    Store &s = g_store[dev * 32 + p];
    if (s.p < 0) {
        s.p = p;
        int KP = ncoef_pad(p);
        s.mat_floats = (size_t)KP * KP;
        s.pool32.block_bytes = sizeof(float) * s.mat_floats;
        s.pool16.block_bytes = split16_bytes(KP);
        s.pool64.block_bytes = sizeof(double) * s.mat_floats;
        std::vector<double> A;
        std::vector<float> host((size_t)8 * KP * KP);
        float *m2m = nullptr, *l2l = nullptr;
        uint64_t *ptrs = nullptr;
        HIP_CHECK(hipMalloc(&m2m, sizeof(float) * host.size()));
        HIP_CHECK(hipMalloc(&l2l, sizeof(float) * host.size()));
        HIP_CHECK(hipMalloc(&ptrs, sizeof(uint64_t) * 16));
        for (int o = 0; o < 8; ++o) {
            build_m2m(p, o, A);
            to_gemm_layout(A, KP, host.data() + (size_t)o * KP * KP);
        }
        HIP_CHECK(hipMemcpy(m2m, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice));
        for (int o = 0; o < 8; ++o) {
            build_l2l(p, o, A);
            to_gemm_layout(A, KP, host.data() + (size_t)o * KP * KP);
        }
        HIP_CHECK(hipMemcpy(l2l, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice));
        uint64_t hp[16];
        for (int o = 0; o < 8; ++o) {
            hp[o] = (uint64_t)(uintptr_t)(m2m + (size_t)o * KP * KP);
            hp[8 + o] = (uint64_t)(uintptr_t)(l2l + (size_t)o * KP * KP);
        }
        HIP_CHECK(hipMemcpy(ptrs, hp, sizeof(hp), hipMemcpyHostToDevice));
        s.tables.p = p;
        s.tables.m2m_ptrs = ptrs;
        s.tables.l2l_ptrs = ptrs + 8;
        // FP64 octant operators, transposed ([KP in][KP out]), for the root levels
        std::vector<double> h64((size_t)8 * KP * KP);
        double *m2m64 = nullptr, *l2l64 = nullptr;
        HIP_CHECK(hipMalloc(&m2m64, sizeof(double) * h64.size()));
        HIP_CHECK(hipMalloc(&l2l64, sizeof(double) * h64.size()));
        for (int o = 0; o < 8; ++o) {
            build_m2m(p, o, A);
            transpose_into(A, KP, h64.data() + (size_t)o * KP * KP);
        }
        HIP_CHECK(hipMemcpy(m2m64, h64.data(), sizeof(double) * h64.size(), hipMemcpyHostToDevice));
        for (int o = 0; o < 8; ++o) {
            build_l2l(p, o, A);
            transpose_into(A, KP, h64.data() + (size_t)o * KP * KP);
        }
        HIP_CHECK(hipMemcpy(l2l64, h64.data(), sizeof(double) * h64.size(), hipMemcpyHostToDevice));
        s.tables.m2m64_t = m2m64;
        s.tables.l2l64_t = l2l64;
        uint64_t hp64[16];
        for (int o = 0; o < 8; ++o) {
            hp64[o] = (uint64_t)(uintptr_t)(m2m64 + (size_t)o * KP * KP);
            hp64[8 + o] = (uint64_t)(uintptr_t)(l2l64 + (size_t)o * KP * KP);
        }
        uint64_t *ptrs64 = nullptr;
        HIP_CHECK(hipMalloc(&ptrs64, sizeof(hp64)));
        HIP_CHECK(hipMemcpy(ptrs64, hp64, sizeof(hp64), hipMemcpyHostToDevice));
        s.tables.m2m64_ptrs = ptrs64;
        s.tables.l2l64_ptrs = ptrs64 + 8;
        std::vector<double> nu = nu_vector(p, KP);
        std::vector<float> nuf(KP);
        for (int i = 0; i < KP; ++i) nuf[i] = i < ncoef(p) ? (float)nu[i] : 0.f;
        float *dnu = nullptr;
        HIP_CHECK(hipMalloc(&dnu, sizeof(float) * KP));
        HIP_CHECK(hipMemcpy(dnu, nuf.data(), sizeof(float) * KP, hipMemcpyHostToDevice));
        s.tables.nu = dnu;
    }
    return s;
}

}  // namespace

const OpTables &op_tables(int p) {
    std::lock_guard<std::mutex> lk(g_mu);
    return store_for(p).tables;
}

// Device copies of host blocks of `bytes` each: consecutive blocks of one pool chunk (adjacent
// on the device, and no block opens a new chunk: two chunks may be adjacent too, but a copy
// must stay inside one allocation) go in one copy.
static void upload_blocks(const std::vector<void *> &dst, const std::vector<char> &fresh, const char *src,
                          size_t bytes) {
    size_t j = 0;
    while (j < dst.size()) {
        size_t k = j + 1;
        while (k < dst.size() && !fresh[k] && static_cast<char *>(dst[k]) == static_cast<char *>(dst[k - 1]) + bytes) ++k;
        HIP_CHECK(hipMemcpy(dst[j], src + j * bytes, (k - j) * bytes, hipMemcpyHostToDevice));
        j = k;
    }
}

void m2l_operator_ptrs(int p, const std::vector<uint64_t> &keys, std::vector<uint64_t> &f32_ptrs,
                       std::vector<uint64_t> &f16_ptrs, bool need_f16) {
    std::lock_guard<std::mutex> lk(g_mu);
    Store &s = store_for(p);
    const int KP = ncoef_pad(p);
    f32_ptrs.resize(keys.size());
    f16_ptrs.assign(keys.size(), 0);
    // operators missing from the cache: built on all host cores, then uploaded in runs
    std::vector<size_t> miss32, miss16;
    for (size_t i = 0; i < keys.size(); ++i) {
        if (!s.f32.count(keys[i])) miss32.push_back(i);
        if (need_f16 && !s.f16.count(keys[i])) miss16.push_back(i);
    }
    if (!miss32.empty() || !miss16.empty()) {
        std::vector<size_t> todo = miss32;   // keys to build: the union of the two lists
        todo.insert(todo.end(), miss16.begin(), miss16.end());
        std::sort(todo.begin(), todo.end());
        todo.erase(std::unique(todo.begin(), todo.end()), todo.end());
        std::vector<int> pos32(keys.size(), -1), pos16(keys.size(), -1);
        for (size_t j = 0; j < miss32.size(); ++j) pos32[miss32[j]] = (int)j;
        for (size_t j = 0; j < miss16.size(); ++j) pos16[miss16[j]] = (int)j;
        std::vector<float> h32(miss32.size() * s.mat_floats);
        std::vector<std::vector<float>> bs(miss32.size());
        std::vector<std::vector<char>> blobs(miss16.size());
        const unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 64));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                std::vector<double> A;
                for (size_t j = t; j < todo.size(); j += nt) {
                    const size_t i = todo[j];
                    build_m2l(p, keys[i], A);
                    if (pos32[i] >= 0) {
                        to_gemm_layout(A, KP, h32.data() + (size_t)pos32[i] * s.mat_floats);
                        bs[pos32[i]] = block_sums(A, p, KP);
                    }
                    if (pos16[i] >= 0) split16(A, p, KP, blobs[pos16[i]]);
                }
            });
        for (auto &x : th) x.join();
        std::vector<void *> d32(miss32.size());
        std::vector<char> f32(miss32.size());
        for (size_t j = 0; j < miss32.size(); ++j) {
            bool fr = false;
            d32[j] = s.alloc_matrix(&fr);
            f32[j] = fr;
            s.f32.emplace(keys[miss32[j]], (uint64_t)(uintptr_t)d32[j]);
            s.bsum[keys[miss32[j]]] = std::move(bs[j]);
        }
        upload_blocks(d32, f32, reinterpret_cast<const char *>(h32.data()), sizeof(float) * s.mat_floats);
        if (!miss16.empty()) {
            const size_t bb = blobs[0].size();
            std::vector<char> h16(miss16.size() * bb);
            std::vector<void *> d16(miss16.size());
            std::vector<char> f16(miss16.size());
            for (size_t j = 0; j < miss16.size(); ++j) {
                if (blobs[j].size() != bb) fail(FMM_EDEVICE, "internal: FP16 operator blobs differ in size");
                std::memcpy(h16.data() + j * bb, blobs[j].data(), bb);
                bool fr = false;
                d16[j] = s.pool16.take(&fr);
                f16[j] = fr;
                s.f16.emplace(keys[miss16[j]], (uint64_t)(uintptr_t)d16[j]);
            }
            upload_blocks(d16, f16, h16.data(), bb);
        }
    }
    for (size_t i = 0; i < keys.size(); ++i) {
        f32_ptrs[i] = s.f32.at(keys[i]);
        if (need_f16) f16_ptrs[i] = s.f16.at(keys[i]);
    }
}

void m2l_block_rows(int p, const std::vector<uint64_t> &keys, double tol, std::vector<uint32_t> &rows,
                    std::vector<float> &kept) {
    std::lock_guard<std::mutex> lk(g_mu);
    Store &s = store_for(p);
    const int NB = ncoef_pad(p) / 16;
    rows.assign(keys.size() * (NB + 1), 0u);
    kept.assign(keys.size(), 1.f);
    std::vector<std::pair<float, int>> order;
    for (size_t i = 0; i < keys.size(); ++i) {
        const std::vector<float> &b = s.bsum.at(keys[i]);
        order.clear();
        for (int q = 0; q < NB * NB; ++q) order.emplace_back(b[q], q);
        std::sort(order.begin(), order.end());
        // drop the smallest blocks while their total stays within tol
        double dropped = 0;
        size_t nd = 0;
        while (nd < order.size() && dropped + order[nd].first <= tol) dropped += order[nd++].first;
        for (size_t q = nd; q < order.size(); ++q) {
            const int blk = order[q].second;
            rows[i * (NB + 1) + blk / NB] |= 1u << (blk % NB);
            rows[i * (NB + 1) + NB] |= 1u << (blk % NB);      // chunks used by any row block
        }
        kept[i] = (float)(order.size() - nd) / (float)order.size();
    }
}

void m2l_svd_ptrs(int p, const std::vector<uint64_t> &keys, double tol, std::vector<uint64_t> &ptrs,
                  std::vector<int32_t> &rank_pad, std::vector<int32_t> &rank) {
    std::lock_guard<std::mutex> lk(g_mu);
    Store &s = store_for(p);
    const int KP = ncoef_pad(p);
    const size_t nk = keys.size();
    // factors missing from the cache, computed on all host cores
    std::vector<size_t> todo;
    for (size_t i = 0; i < nk; ++i)
        if (!s.svd.count({keys[i], tol})) todo.push_back(i);
    std::vector<SvdFactor> fac(todo.size());
    {
        const unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 64));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                std::vector<double> A;
                for (size_t j = t; j < todo.size(); j += nt) {
                    build_m2l(p, keys[todo[j]], A);
                    fac[j] = svd_factor(A, p, KP, tol);
                }
            });
        for (auto &x : th) x.join();
    }
    std::vector<float> host;
    for (size_t j = 0; j < todo.size(); ++j) {
        SvdEntry e;
        e.r = fac[j].r;
        e.rp = std::max(16, (e.r + 15) / 16 * 16);
        host.assign((size_t)2 * e.rp * KP, 0.f);
        svd_gemm_layout(fac[j], p, KP, e.rp, host.data());
        char *d = static_cast<char *>(s.svd_arena.take(sizeof(float) * host.size()));
        HIP_CHECK(hipMemcpy(d, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice));
        e.q = (uint64_t)(uintptr_t)d;
        e.pp = (uint64_t)(uintptr_t)(d + sizeof(float) * (size_t)e.rp * KP);
        s.svd[{keys[todo[j]], tol}] = e;
    }
    ptrs.resize(2 * nk);
    rank_pad.resize(nk);
    rank.resize(nk);
    for (size_t i = 0; i < nk; ++i) {
        const SvdEntry &e = s.svd.at({keys[i], tol});
        ptrs[2 * i] = e.q;
        ptrs[2 * i + 1] = e.pp;
        rank_pad[i] = e.rp;
        rank[i] = e.r;
    }
}

void m2l_operator_ptrs64(int p, const std::vector<uint64_t> &keys, std::vector<uint64_t> &f64_ptrs) {
    std::lock_guard<std::mutex> lk(g_mu);
    Store &s = store_for(p);
    f64_ptrs.resize(keys.size());
    const int KP = ncoef_pad(p);
    // missing operators built on all host cores, then uploaded in runs
    std::vector<size_t> miss;
    for (size_t i = 0; i < keys.size(); ++i)
        if (!s.f64.count(keys[i])) miss.push_back(i);
    if (!miss.empty()) {
        std::vector<double> h(miss.size() * s.mat_floats);
        const unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 64));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                std::vector<double> A;
                for (size_t j = t; j < miss.size(); j += nt) {
                    build_m2l(p, keys[miss[j]], A);
                    transpose_into(A, KP, h.data() + j * s.mat_floats);
                }
            });
        for (auto &x : th) x.join();
        std::vector<void *> d(miss.size());
        std::vector<char> fresh(miss.size());
        for (size_t j = 0; j < miss.size(); ++j) {
            bool fr = false;
            d[j] = s.pool64.take(&fr);
            fresh[j] = fr;
            s.f64.emplace(keys[miss[j]], (uint64_t)(uintptr_t)d[j]);
        }
        upload_blocks(d, fresh, reinterpret_cast<const char *>(h.data()), sizeof(double) * s.mat_floats);
    }
    for (size_t i = 0; i < keys.size(); ++i) f64_ptrs[i] = s.f64.at(keys[i]);
}

}  // namespace fmm
