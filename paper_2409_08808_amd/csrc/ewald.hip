// Ewald pair matrix on gfx950 (Methodology, "Cluster Expansion of Coulomb
// Energy": periodic point-charge energies by Ewald summation).
//
//   V_ij = k_e [ sum_{m: 0 < |r+mA| < rc} erfc(a|r+mA|)/|r+mA|            (real)
//              + (4 pi/W) sum_{G != 0} e^{-G^2/4a^2}/G^2 cos(G.r)           (reciprocal)
//              - pi/(W a^2) ] - delta_ij k_e 2a/sqrt(pi),   r = r_j - r_i.
//
// Real space: one thread per entry loops over the lattice translations that can
// bring an image within rc (FP64 VALU, erfc). Reciprocal space: G and -G pair up,
// so the sum over the half space with weight w_G = 2 (4 pi/W) e^{-G^2/4a^2}/G^2 is
// sum_G w_G [cos(G.r_i) cos(G.r_j) + sin(G.r_i) sin(G.r_j)] = (T T^T)_ij with
// T_{i,2g} = sqrt(k_e w_g) cos(G_g.r_i), T_{i,2g+1} = sqrt(k_e w_g) sin(G_g.r_i):
// an FP64 matrix-core product added onto the real-space part.
//
// V_ij depends on r_j - r_i only, so a translation t that maps the set of sites
// onto itself gives V_{s(i) s(j)} = V_ij. When the sites are invariant under an
// axis-aligned grid of fractional translations Z_m0 x Z_m1 x Z_m2 (every supercell
// of a crystal is), only one row per orbit of the grid is summed (real space by
// k_ewald_real on those rows, reciprocal space directly as sum_G w_G cos(G.r)) and
// every other row is the relabelled row of its orbit's representative.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace goac {

namespace {
constexpr double kPi = 3.14159265358979323846;

struct Cell {
    double A[3][3];
    double B[3][3];
    double vol;
};

bool cell_setup(const double* lat, Cell& c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.A[i][j] = lat[3 * i + j];
    double cr[3][3];
    for (int i = 0; i < 3; ++i) {
        const double* u = c.A[(i + 1) % 3];
        const double* v = c.A[(i + 2) % 3];
        cr[i][0] = u[1] * v[2] - u[2] * v[1];
        cr[i][1] = u[2] * v[0] - u[0] * v[2];
        cr[i][2] = u[0] * v[1] - u[1] * v[0];
    }
    const double det = c.A[0][0] * cr[0][0] + c.A[0][1] * cr[0][1] + c.A[0][2] * cr[0][2];
    if (!(std::fabs(det) > 1e-12)) return false;
    c.vol = std::fabs(det);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.B[i][j] = 2.0 * kPi * cr[i][j] / det;
    return true;
}

double norm3(const double* v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }
}  // namespace

// Real-space part plus the constant terms. Positions arrive reduced to
// fractional coordinates in [0, 1); r = r_j - r_i is folded to (-1/2, 1/2] per
// axis before the translation loop.
// With rows, output row y holds site rows[y] (the representatives of the symmetric
// build); without, row y is site y.
__global__ void k_ewald_real(int64_t n, const double* __restrict__ frac, const double* __restrict__ A9,
                             const double* __restrict__ trans, int32_t n_trans, double alpha, double rcut,
                             double ke, double cst, double self, const int32_t* __restrict__ rows,
                             double* __restrict__ V) {
    extern __shared__ double s_tr[];
    for (int m = threadIdx.x; m < 3 * n_trans; m += blockDim.x) s_tr[m] = trans[m];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t y = blockIdx.y;
    const int64_t i = rows ? (int64_t)rows[y] : y;
    if (j >= n) return;
    double f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double x = frac[3 * j + d] - frac[3 * i + d];
        x -= rint(x);
        f[d] = x;
    }
    double r[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) r[d] = f[0] * A9[d] + f[1] * A9[3 + d] + f[2] * A9[6 + d];
    const double rc2 = rcut * rcut;
    double s = 0.0;
    for (int m = 0; m < n_trans; ++m) {
        const double x = r[0] + s_tr[3 * m], y = r[1] + s_tr[3 * m + 1], z = r[2] + s_tr[3 * m + 2];
        const double d2 = x * x + y * y + z * z;
        if (d2 < rc2 && d2 > 0.0) {
            const double dd = sqrt(d2);
            s += erfc(alpha * dd) / dd;
        }
    }
    double v = ke * s + cst;
    if (i == j) v -= self;
    V[y * n + j] = v;
}

// Reciprocal part of the representative rows, chunk z of the G list:
// part[z][y][j] = sum_{g in chunk z} w_g cos(G_g.(r_j - r_rows[y])), w_g = s_g^2
// (the table's weight squared); the chunks are summed in order by k_ewald_rows_sum.
__global__ void k_ewald_recip_rows(int64_t n, int32_t K, int32_t chunk, const int32_t* __restrict__ rows,
                                   const double* __restrict__ pos, const double* __restrict__ G,
                                   double* __restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t y = blockIdx.y;
    const int z = blockIdx.z;
    if (j >= n) return;
    const int64_t i = rows[y];
    const double dx = pos[3 * j] - pos[3 * i], dy = pos[3 * j + 1] - pos[3 * i + 1], dz = pos[3 * j + 2] - pos[3 * i + 2];
    const int g0 = z * chunk, g1 = min(K, g0 + chunk);
    double s = 0.0;
    for (int g = g0; g < g1; ++g) {
        const double w = G[4 * g + 3];
        s += (w * w) * cos(G[4 * g] * dx + G[4 * g + 1] * dy + G[4 * g + 2] * dz);
    }
    part[((int64_t)z * gridDim.y + y) * n + j] = s;
}

// Vrep[y][j] += sum over the chunks z (in order) of part[z][y][j]
__global__ void k_ewald_rows_sum(int64_t cnt, int32_t nz, const double* __restrict__ part, double* __restrict__ Vrep) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * cnt + e];
    Vrep[e] += s;
}

// V[i][j] = Vrep[b_i][j'], j' the site translate (g_j - g_i) mod m of representative
// b_j: r_j - r_i = r_j' - r_rep(b_i) modulo the lattice. site_g packs g0 | g1 << 10 | g2 << 20.
__global__ void k_ewald_fill(int64_t n, int32_t ng, int32_t m0, int32_t m1, int32_t m2,
                             const int32_t* __restrict__ site_b, const int32_t* __restrict__ site_g,
                             const int32_t* __restrict__ idx, const double* __restrict__ Vrep,
                             double* __restrict__ V) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    const int gi = site_g[i], gj = site_g[j];
    int d0 = (gj & 1023) - (gi & 1023);
    int d1 = ((gj >> 10) & 1023) - ((gi >> 10) & 1023);
    int d2 = ((gj >> 20) & 1023) - ((gi >> 20) & 1023);
    d0 += d0 < 0 ? m0 : 0;
    d1 += d1 < 0 ? m1 : 0;
    d2 += d2 < 0 ? m2 : 0;
    const int jj = idx[(int64_t)site_b[j] * ng + (d0 * m1 + d1) * m2 + d2];
    V[i * n + j] = Vrep[(int64_t)site_b[i] * n + jj];
}

// T[i][2g] = s_g cos(G_g.r_i), T[i][2g+1] = s_g sin(G_g.r_i), zero padding to ld
__global__ void k_ewald_table(int64_t n, int32_t K, int32_t ld, const double* __restrict__ pos,
                              const double* __restrict__ G, double* __restrict__ T) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * (int64_t)ld / 2) return;
    const int64_t i = idx / (ld / 2);
    const int g = (int)(idx - i * (ld / 2));
    double c = 0.0, s = 0.0;
    if (g < K) {
        const double gr = G[4 * g] * pos[3 * i] + G[4 * g + 1] * pos[3 * i + 1] + G[4 * g + 2] * pos[3 * i + 2];
        const double w = G[4 * g + 3];
        sincos(gr, &s, &c);
        c *= w;
        s *= w;
    }
    T[i * ld + 2 * g] = c;
    T[i * ld + 2 * g + 1] = s;
}

// The grid of axis-aligned fractional translations (1/m0, 0, 0), (0, 1/m1, 0),
// (0, 0, 1/m2) under which the site set is invariant, with each axis's m the largest
// that works, and each site's representative and translate (nb = 0 when the grid is
// trivial or anything does not add up). Positions are hashed on a 2^-20 grid of
// fractional coordinates, each lookup trying the neighbouring keys too, and a match
// must agree within kSymTol in every fractional coordinate: sites that differ by the
// rounding of their coordinates match, a set perturbed by more (noise in the
// input) is not a translate of itself and takes the general build.
constexpr double kSymTol = 1e-10;
static void ewald_symmetry(const std::vector<double>& frac, int64_t n, EwaldPlan& P, std::vector<int32_t>& sym) {
    P.nb = 0;
    P.ng = 0;
    P.m[0] = P.m[1] = P.m[2] = 1;
    sym.clear();
    if (n < 2 || n > ((int64_t)1 << 30)) return;
    constexpr int64_t Q = (int64_t)1 << 20;
    auto qv = [](double f) { return (int64_t)std::llround(f * (double)Q) & (Q - 1); };
    auto key = [](int64_t a, int64_t b, int64_t c) { return (uint64_t)a | ((uint64_t)b << 20) | ((uint64_t)c << 40); };
    std::unordered_map<uint64_t, int32_t> at;
    at.reserve((size_t)n * 2);
    for (int64_t i = 0; i < n; ++i)
        if (!at.emplace(key(qv(frac[3 * i]), qv(frac[3 * i + 1]), qv(frac[3 * i + 2])), (int32_t)i).second) return;
    auto find = [&](double f0, double f1, double f2) -> int32_t {
        const int64_t a = qv(f0), b = qv(f1), c = qv(f2);
        for (int da = -1; da <= 1; ++da)
            for (int db = -1; db <= 1; ++db)
                for (int dc = -1; dc <= 1; ++dc) {
                    const auto it = at.find(key((a + da) & (Q - 1), (b + db) & (Q - 1), (c + dc) & (Q - 1)));
                    if (it == at.end()) continue;
                    const int64_t r = it->second;
                    const double e[3] = {frac[3 * r] - f0, frac[3 * r + 1] - f1, frac[3 * r + 2] - f2};
                    bool close = true;
                    for (int d = 0; d < 3; ++d) close = close && std::fabs(e[d] - std::nearbyint(e[d])) <= kSymTol;
                    if (close) return (int32_t)r;
                }
        return -1;
    };
    int m[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d) {
        std::vector<int64_t> vals(n);
        for (int64_t i = 0; i < n; ++i) vals[i] = qv(frac[3 * i + d]);
        std::sort(vals.begin(), vals.end());
        const int64_t kd = std::unique(vals.begin(), vals.end()) - vals.begin();
        for (int64_t cand = std::min<int64_t>(kd, 1024); cand >= 2; --cand) {
            if (kd % cand) continue;
            const double t = 1.0 / (double)cand;
            bool ok = true;
            for (int64_t i = 0; i < n && ok; ++i) {
                double f[3] = {frac[3 * i], frac[3 * i + 1], frac[3 * i + 2]};
                f[d] += t;
                ok = find(f[0], f[1], f[2]) >= 0;
            }
            if (ok) {
                m[d] = (int)cand;
                break;
            }
        }
    }
    const int64_t ng = (int64_t)m[0] * m[1] * m[2];
    if (ng < 2 || n % ng) return;
    const int64_t nb = n / ng;
    std::vector<int32_t> site_b(n, -1), site_g(n), idx(n, -1), reps;
    std::vector<int32_t> g(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            int64_t gd = (int64_t)std::floor(frac[3 * i + d] * m[d] + 1e-6);
            gd %= m[d];
            if (gd < 0) gd += m[d];
            g[3 * i + d] = (int32_t)gd;
        }
    std::unordered_map<int32_t, int32_t> bof;
    for (int64_t i = 0; i < n; ++i)
        if (g[3 * i] == 0 && g[3 * i + 1] == 0 && g[3 * i + 2] == 0) {
            bof[(int32_t)i] = (int32_t)reps.size();
            reps.push_back((int32_t)i);
        }
    if ((int64_t)reps.size() != nb) return;
    for (int64_t i = 0; i < n; ++i) {
        double f[3];
        for (int d = 0; d < 3; ++d) {
            f[d] = frac[3 * i + d] - (double)g[3 * i + d] / m[d];
            f[d] -= std::floor(f[d]);
        }
        const int32_t r = find(f[0], f[1], f[2]);
        const auto it = r >= 0 ? bof.find(r) : bof.end();
        if (it == bof.end()) return;
        site_b[i] = it->second;
        site_g[i] = g[3 * i] | (g[3 * i + 1] << 10) | (g[3 * i + 2] << 20);
        const int64_t slot = (int64_t)it->second * ng + ((int64_t)g[3 * i] * m[1] + g[3 * i + 1]) * m[2] + g[3 * i + 2];
        if (idx[slot] >= 0) return;
        idx[slot] = (int32_t)i;
    }
    P.nb = (int32_t)nb;
    P.ng = (int32_t)ng;
    for (int d = 0; d < 3; ++d) P.m[d] = m[d];
    sym.reserve(nb + 3 * n);
    sym.insert(sym.end(), reps.begin(), reps.end());
    sym.insert(sym.end(), site_b.begin(), site_b.end());
    sym.insert(sym.end(), site_g.begin(), site_g.end());
    sym.insert(sym.end(), idx.begin(), idx.end());
}

// CODATA 2018: e = 1.602176634e-19 C, eps0 = 8.8541878128e-12 F/m -> eV A
static double coulomb_constant() { return 1.602176634e-19 / (4.0 * kPi * 8.8541878128e-12) * 1e10; }

// The host-side tables of a build (fractional and folded positions, lattice
// translations, half-space G vectors with their weights), laid out as uploaded.
// They depend only on the inputs, so the context keeps the last set and reuses it
// when the same cell and parameters come again.
static goac_status ewald_plan(goac_ctx* ctx, const double* lat, int64_t n, const double* pos,
                              const goac_ewald_params* prm, EwaldPlan& P) {
    const double alpha_in = prm ? prm->alpha : 0.0, rcut_in = prm ? prm->rcut : 0.0;
    const int32_t kmax_in = prm ? prm->kmax : 0;
    const int32_t flags_in = prm ? prm->flags : 0;
    if (P.n == n && P.alpha_in == alpha_in && P.rcut_in == rcut_in && P.kmax_in == kmax_in && P.flags_in == flags_in &&
        std::memcmp(P.lat, lat, sizeof(P.lat)) == 0 && P.pos.size() == (size_t)(3 * n) &&
        std::memcmp(P.pos.data(), pos, (size_t)(3 * n) * sizeof(double)) == 0)
        return GOAC_OK;
    P.n = -1;   // invalid until complete
    Cell c;
    if (!cell_setup(lat, c)) return fail(ctx, GOAC_EINVAL, "build_ewald: singular lattice");
    double alpha = alpha_in, rcut = rcut_in;
    int kmax = kmax_in;
    if (!(alpha > 0.0)) alpha = 5.0 / std::cbrt(c.vol);
    if (!(rcut > 0.0)) rcut = 6.0 / alpha;
    if (kmax <= 0) {
        double amax = 0.0;
        for (int i = 0; i < 3; ++i) amax = std::fmax(amax, norm3(c.A[i]));
        kmax = (int)std::ceil(12.0 * alpha * amax / (2.0 * kPi));
    }
    if (kmax > 200) return fail(ctx, GOAC_EINVAL, "build_ewald: reciprocal index radius above 200");
    const double ke = coulomb_constant();

    // fractional coordinates in [0, 1)
    // inverse of A (rows a_i): f = r A^-1, A^-1 = B^T / (2 pi)
    std::vector<double> frac(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double* r = pos + 3 * i;
            double f = (r[0] * c.B[d][0] + r[1] * c.B[d][1] + r[2] * c.B[d][2]) / (2.0 * kPi);
            f -= std::floor(f);
            frac[3 * i + d] = f;
        }
    // lattice translations whose images of a folded r (|f_d| <= 1/2) can lie within rcut:
    // (|m_d| - 1/2) times the plane spacing of axis d must stay below rcut
    std::vector<double> trans;
    int nm[3];
    double spacing[3];
    for (int d = 0; d < 3; ++d) {
        spacing[d] = 2.0 * kPi / norm3(c.B[d]);
        nm[d] = (int)std::ceil(rcut / spacing[d] + 0.5);
    }
    for (int a = -nm[0]; a <= nm[0]; ++a)
        for (int b = -nm[1]; b <= nm[1]; ++b)
            for (int e = -nm[2]; e <= nm[2]; ++e) {
                const int m[3] = {a, b, e};
                bool skip = false;
                for (int d = 0; d < 3; ++d)
                    if ((std::abs(m[d]) - 0.5) * spacing[d] >= rcut) skip = true;
                if (skip) continue;
                for (int k = 0; k < 3; ++k) trans.push_back(a * c.A[0][k] + b * c.A[1][k] + e * c.A[2][k]);
            }
    if (trans.size() * sizeof(double) > 60 * 1024)
        return fail(ctx, GOAC_EINVAL, "build_ewald: real-space cutoff spans too many cells");
    // half-space reciprocal vectors (first non-zero index positive) with weights
    std::vector<double> G;
    for (int a = -kmax; a <= kmax; ++a)
        for (int b = -kmax; b <= kmax; ++b)
            for (int e = -kmax; e <= kmax; ++e) {
                if (a * a + b * b + e * e > kmax * kmax) continue;
                if (!(a > 0 || (a == 0 && b > 0) || (a == 0 && b == 0 && e > 0))) continue;
                double g[3];
                for (int k = 0; k < 3; ++k) g[k] = a * c.B[0][k] + b * c.B[1][k] + e * c.B[2][k];
                const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                const double w = 2.0 * (4.0 * kPi / c.vol) * std::exp(-g2 / (4.0 * alpha * alpha)) / g2;
                G.insert(G.end(), {g[0], g[1], g[2], std::sqrt(ke * w)});
            }
    P.K = (int32_t)(G.size() / 4);
    P.ld = (int32_t)round_up(2 * (int64_t)std::max(P.K, 1), 16);
    P.ntrans = (int32_t)(trans.size() / 3);
    P.b_frac = round_up(frac.size() * 8, 256);
    P.b_pos = round_up(3 * n * 8, 256);
    P.b_tr = round_up(trans.size() * 8 + 8, 256);
    P.b_G = round_up(G.size() * 8 + 8, 256);
    P.b_A = 256;
    // folded Cartesian positions for the tables (exact phase equivalence mod 2 pi)
    std::vector<double> cpos(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            cpos[3 * i + k] = frac[3 * i] * c.A[0][k] + frac[3 * i + 1] * c.A[1][k] + frac[3 * i + 2] * c.A[2][k];
    // the translation grid (unless the general build is asked for)
    std::vector<int32_t> sym;
    if (!(flags_in & GOAC_EWALD_GENERAL)) ewald_symmetry(frac, n, P, sym);
    else P.nb = 0;
    P.b_sym = round_up(sym.size() * 4 + 4, 256);
    // the tables in the workspace's layout, one copy
    P.img.assign(P.b_frac + P.b_pos + P.b_tr + P.b_G + P.b_A + P.b_sym, 0);
    if (!sym.empty())
        std::memcpy(P.img.data() + P.b_frac + P.b_pos + P.b_tr + P.b_G + P.b_A, sym.data(), sym.size() * 4);
    std::memcpy(P.img.data(), frac.data(), frac.size() * 8);
    std::memcpy(P.img.data() + P.b_frac, cpos.data(), cpos.size() * 8);
    if (!trans.empty()) std::memcpy(P.img.data() + P.b_frac + P.b_pos, trans.data(), trans.size() * 8);
    if (!G.empty()) std::memcpy(P.img.data() + P.b_frac + P.b_pos + P.b_tr, G.data(), G.size() * 8);
    std::memcpy(P.img.data() + P.b_frac + P.b_pos + P.b_tr + P.b_G, &c.A[0][0], 9 * 8);
    P.alpha = alpha;
    P.rcut = rcut;
    P.ke = ke;
    P.cst = -ke * kPi / (c.vol * alpha * alpha);
    P.self = ke * 2.0 * alpha / std::sqrt(kPi);
    // the key, last
    std::memcpy(P.lat, lat, sizeof(P.lat));
    P.pos.assign(pos, pos + 3 * n);
    P.alpha_in = alpha_in;
    P.rcut_in = rcut_in;
    P.kmax_in = kmax_in;
    P.flags_in = flags_in;
    P.n = n;
    return GOAC_OK;
}

goac_status build_ewald(goac_ctx* ctx, const double* lat, int64_t n, const double* pos, const goac_ewald_params* prm,
                        double* V) {
    EwaldPlan& P = ctx->ewald;
    GOAC_TRY(ewald_plan(ctx, lat, n, pos, prm, P));
    const size_t b_tab = P.img.size();
    // symmetric build: the representatives' rows and the G chunks' partial sums;
    // general build: the reciprocal table T
    constexpr int kChunks = 16;
    const int32_t chunk = (P.K + kChunks - 1) / kChunks;
    const int32_t nz = P.K > 0 ? (P.K + chunk - 1) / chunk : 0;
    const size_t b_rest = P.nb > 0 ? round_up((size_t)P.nb * n * 8, 256) * (size_t)(1 + nz) : (size_t)n * P.ld * 8;
    void* ws = nullptr;
    goac_status st = workspace(ctx, 0, b_tab + b_rest, &ws);
    if (st != GOAC_OK) return st;
    char* p = (char*)ws;
    double* d_frac = (double*)p; p += P.b_frac;
    double* d_pos = (double*)p; p += P.b_pos;
    double* d_tr = (double*)p; p += P.b_tr;
    double* d_G = (double*)p; p += P.b_G;
    double* d_A = (double*)p; p += P.b_A;
    const int32_t* d_sym = (const int32_t*)p; p += P.b_sym;
    GOAC_TRY(upload(ctx, d_frac, P.img.data(), P.img.size()));
    if (P.nb > 0) {
        const int32_t* reps = d_sym;
        const int32_t* site_b = reps + P.nb;
        const int32_t* site_g = site_b + n;
        const int32_t* idx = site_g + n;
        double* Vrep = (double*)p;
        double* part = (double*)(p + round_up((size_t)P.nb * n * 8, 256));
        const unsigned gx = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_ewald_real, dim3(gx, (unsigned)P.nb), dim3(256), (size_t)P.ntrans * 3 * sizeof(double),
                           ctx->stream, n, d_frac, d_A, d_tr, P.ntrans, P.alpha, P.rcut, P.ke, P.cst, P.self, reps,
                           Vrep);
        GOAC_CHECK_LAUNCH(ctx);
        if (nz > 0) {
            hipLaunchKernelGGL(k_ewald_recip_rows, dim3(gx, (unsigned)P.nb, (unsigned)nz), dim3(256), 0, ctx->stream,
                               n, P.K, chunk, reps, d_pos, d_G, part);
            GOAC_CHECK_LAUNCH(ctx);
            const int64_t cnt = (int64_t)P.nb * n;
            hipLaunchKernelGGL(k_ewald_rows_sum, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, ctx->stream, cnt,
                               nz, part, Vrep);
            GOAC_CHECK_LAUNCH(ctx);
        }
        hipLaunchKernelGGL(k_ewald_fill, dim3(gx, (unsigned)n), dim3(256), 0, ctx->stream, n, P.ng, P.m[0], P.m[1],
                           P.m[2], site_b, site_g, idx, Vrep, V);
        GOAC_CHECK_LAUNCH(ctx);
        return GOAC_OK;
    }
    double* d_T = (double*)p;
    {
        dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
        hipLaunchKernelGGL(k_ewald_real, grid, dim3(256), (size_t)P.ntrans * 3 * sizeof(double), ctx->stream, n,
                           d_frac, d_A, d_tr, P.ntrans, P.alpha, P.rcut, P.ke, P.cst, P.self, (const int32_t*)nullptr,
                           V);
        GOAC_CHECK_LAUNCH(ctx);
    }
    if (P.K > 0) {
        const int64_t tot = n * (int64_t)P.ld / 2;
        hipLaunchKernelGGL(k_ewald_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, n, P.K,
                           P.ld, d_pos, d_G, d_T);
        GOAC_CHECK_LAUNCH(ctx);
        st = dgemm_nt(ctx, n, n, P.ld, d_T, P.ld, d_T, P.ld, V, n, 1.0, 1.0, nullptr, true);
        if (st != GOAC_OK) return st;
    }
    // the uploads came from the staging ring, so the host tables may change now
    return GOAC_OK;
}

}  // namespace goac
