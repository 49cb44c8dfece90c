/*
 * goac_oracle.c -- plain, slow FP64 CPU oracle of the pairwise Coulomb
 * cluster-expansion optimiser (Koester, Binninger, Kaghazchi, "Optimization of
 * Coulomb Energies in Gigantic Configurational Spaces of Multi-Element Ionic
 * Crystals", arXiv 2409.08808).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark load this library. It shares no code, header or table
 * with the HIP library; both follow the paper and the written readings of it.
 *
 * Everything is FP64 and written as the definition or the algorithm's steps in
 * order, with no blocking or fusion. Compile with -ffp-contract=off so that every
 * expression rounds exactly as written.
 *
 * Contents
 *   Philox4x32-10 ............ counter-based RNG (Salmon et al., SC'11)
 *   or_ewald_*  .............. periodic point-charge pair matrix and energy
 *                              (Methodology, "Cluster Expansion of Coulomb
 *                              Energy": Ewald summation of point charges)
 *   or_energies .............. E = 1/2 q^T V q (the exact second-order CE)
 *   or_init_occupations ...... random valid start (SI, "Random")
 *   or_mc_run ................ Metropolis / annealed swap Monte Carlo (SI, "Monte
 *                              Carlo" and "Simulated annealing")
 *   or_gd_run ................ best-swap descent to a local minimum (SI,
 *                              "Gradient Descent")
 *   or_remc_exchange ......... replica-exchange step (SI, "Replica Exchange MC")
 *   or_ga_generation ......... genetic algorithm generation (SI, "Genetic
 *                              Algorithm": roulette, swap crossover, mutation,
 *                              elitism)
 *   or_topk .................. the n lowest configurations (Methodology,
 *                              "Implementation and Theoretical Background")
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers:  */
/* as easy as 1, 2, 3"): ten rounds of two 32x32->64 multiplies with the       */
/* Weyl-sequence key schedule.                                                  */
/* ------------------------------------------------------------------------- */
#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

enum { TAG_MC = 1, TAG_INIT = 2, TAG_SEL = 3, TAG_X = 4, TAG_MUT = 5, TAG_REMC = 6 };

void or_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PH_M0 * c0;
        uint64_t p1 = (uint64_t)PH_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PH_W0; k1 += PH_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint64_t seed, uint32_t r[4]) {
    uint32_t ctr[4] = {a, b, c, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, r);
}

/* uniform on (0,1): the top 52 bits of a 64-bit word plus one half, times 2^-52 */
static double unit_open(uint32_t hi, uint32_t lo) {
    uint64_t x = ((uint64_t)hi << 32) | lo;
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

/* splitmix64 finaliser (Steele, Lea, Flood, OOPSLA'14) */
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* one trial's contribution to the order-independent trajectory hash */
uint64_t or_trial_hash(uint64_t t, uint32_t i, uint32_t j, uint32_t acc) {
    uint64_t key = ((uint64_t)i << 33) | ((uint64_t)j << 1) | (uint64_t)(acc & 1u);
    return splitmix64(splitmix64(t) ^ key);
}

/* ------------------------------------------------------------------------- */
/* Ewald pair matrix. V_ij = k_e [psi_real(r_ij) + psi_recip(r_ij) - pi/(W a^2)] */
/* - delta_ij k_e 2a/sqrt(pi), with r_ij = r_j - r_i, W the cell volume, a the  */
/* Ewald splitting parameter. Tin-foil boundary; the uniform neutralising       */
/* background term is kept in every entry. E(q) = 1/2 sum_ij q_i q_j V_ij in eV.*/
/* ------------------------------------------------------------------------- */

/* Coulomb constant e/(4 pi eps0) in eV*Angstrom from CODATA 2018 e and eps0 */
double or_coulomb_constant(void) {
    const double e = 1.602176634e-19;        /* C (exact)      */
    const double eps0 = 8.8541878128e-12;    /* F/m            */
    const double pi = 3.14159265358979323846;
    return e / (4.0 * pi * eps0) * 1e10;
}

typedef struct {
    double A[3][3];      /* rows: lattice vectors                 */
    double B[3][3];      /* rows: reciprocal vectors, a_i.b_j = 2 pi delta_ij */
    double vol;
} cell_t;

static void cell_setup(const double lat[9], cell_t* c) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c->A[i][j] = lat[3 * i + j];
    const double (*a)[3] = (const double (*)[3])c->A;
    /* b1 = 2 pi (a2 x a3)/V etc. */
    double cr[3][3];
    for (int i = 0; i < 3; ++i) {
        const double* u = a[(i + 1) % 3];
        const double* v = a[(i + 2) % 3];
        cr[i][0] = u[1] * v[2] - u[2] * v[1];
        cr[i][1] = u[2] * v[0] - u[0] * v[2];
        cr[i][2] = u[0] * v[1] - u[1] * v[0];
    }
    double det = a[0][0] * cr[0][0] + a[0][1] * cr[0][1] + a[0][2] * cr[0][2];
    c->vol = fabs(det);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c->B[i][j] = 2.0 * pi * cr[i][j] / det;
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* Parameters a value <= 0 leaves to a default: alpha = 5 / W^(1/3), rcut = 6 /
 * alpha (erfc(6) ~ 2e-17), and the reciprocal index sphere |n| <= kmax with kmax =
 * ceil(12 alpha |a|_max / (2 pi)), so every omitted reciprocal term carries a
 * Gaussian factor below e^-36. */
void or_ewald_defaults(const double lat[9], double* alpha, double* rcut, int* kmax) {
    const double pi = 3.14159265358979323846;
    cell_t c;
    cell_setup(lat, &c);
    if (!(*alpha > 0.0)) *alpha = 5.0 / cbrt(c.vol);
    if (!(*rcut > 0.0)) *rcut = 6.0 / *alpha;
    if (*kmax <= 0) {
        double amax = 0.0;
        for (int i = 0; i < 3; ++i) amax = fmax(amax, norm3(c.A[i]));
        *kmax = (int)ceil(12.0 * (*alpha) * amax / (2.0 * pi));
    }
}

/* range of integer image index m along lattice direction d such that some image
 * r + m a_d could lie within rcut: |(r + m A).b_d| <= rcut |b_d|. */
static void image_range(const cell_t* c, const double r[3], double rcut, int lo[3], int hi[3]) {
    const double pi = 3.14159265358979323846;
    for (int d = 0; d < 3; ++d) {
        double rb = r[0] * c->B[d][0] + r[1] * c->B[d][1] + r[2] * c->B[d][2];
        double bn = norm3(c->B[d]);
        lo[d] = (int)floor((-rcut * bn - rb) / (2.0 * pi)) - 1;
        hi[d] = (int)ceil((rcut * bn - rb) / (2.0 * pi)) + 1;
    }
}

/* psi_real(r) = sum over images m with 0 < |r + m A| < rcut of erfc(alpha d)/d */
static double psi_real(const cell_t* c, const double r[3], double alpha, double rcut) {
    int lo[3], hi[3];
    image_range(c, r, rcut, lo, hi);
    double s = 0.0;
    for (int m0 = lo[0]; m0 <= hi[0]; ++m0)
        for (int m1 = lo[1]; m1 <= hi[1]; ++m1)
            for (int m2 = lo[2]; m2 <= hi[2]; ++m2) {
                double x[3];
                for (int k = 0; k < 3; ++k)
                    x[k] = r[k] + m0 * c->A[0][k] + m1 * c->A[1][k] + m2 * c->A[2][k];
                double d = norm3(x);
                if (d > 0.0 && d < rcut) s += erfc(alpha * d) / d;
            }
    return s;
}

/* psi_recip(r) = (4 pi / W) sum over n != 0, |n|^2 <= kmax^2 of
 * exp(-G^2/(4 alpha^2)) / G^2 cos(G.r), G = n1 b1 + n2 b2 + n3 b3 */
static double psi_recip(const cell_t* c, const double r[3], double alpha, int kmax) {
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    for (int n0 = -kmax; n0 <= kmax; ++n0)
        for (int n1 = -kmax; n1 <= kmax; ++n1)
            for (int n2 = -kmax; n2 <= kmax; ++n2) {
                if (n0 == 0 && n1 == 0 && n2 == 0) continue;
                if (n0 * n0 + n1 * n1 + n2 * n2 > kmax * kmax) continue;
                double G[3];
                for (int k = 0; k < 3; ++k) G[k] = n0 * c->B[0][k] + n1 * c->B[1][k] + n2 * c->B[2][k];
                double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                double gr = G[0] * r[0] + G[1] * r[1] + G[2] * r[2];
                s += exp(-g2 / (4.0 * alpha * alpha)) / g2 * cos(gr);
            }
    return 4.0 * pi / c->vol * s;
}

/* One entry V_ij. Returns 0, or -1 on bad parameters. */
int or_ewald_entry(const double lat[9], const double* pos, int64_t i, int64_t j,
                   double alpha, double rcut, int kmax, double* out) {
    const double pi = 3.14159265358979323846;
    or_ewald_defaults(lat, &alpha, &rcut, &kmax);
    if (!(alpha > 0.0) || !(rcut > 0.0) || kmax < 0) return -1;
    cell_t c;
    cell_setup(lat, &c);
    double r[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1], pos[3 * j + 2] - pos[3 * i + 2]};
    double ke = or_coulomb_constant();
    double v = psi_real(&c, r, alpha, rcut) + psi_recip(&c, r, alpha, kmax) - pi / (c.vol * alpha * alpha);
    v = ke * v;
    if (i == j) v -= ke * 2.0 * alpha / sqrt(pi);
    *out = v;
    return 0;
}

/* Full n x n matrix, row-major. OpenMP over rows. */
int or_ewald_matrix(const double lat[9], int64_t n, const double* pos, double alpha, double rcut,
                    int kmax, double* V) {
    or_ewald_defaults(lat, &alpha, &rcut, &kmax);
    if (!(alpha > 0.0) || !(rcut > 0.0) || kmax < 0 || n <= 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) or_ewald_entry(lat, pos, i, j, alpha, rcut, kmax, &V[i * n + j]);
    return 0;
}

/* Ewald energy of a (possibly charged) set of point charges written in the
 * structure-factor form, an independent route to 1/2 q^T V q:
 *   E = k_e [ 1/2 sum_ij sum'_m q_i q_j erfc(a d)/d
 *           + (2 pi / W) sum_{G != 0} exp(-G^2/4a^2)/G^2 |S(G)|^2
 *           - a/sqrt(pi) sum_i q_i^2 - pi Q^2 / (2 W a^2) ],
 * S(G) = sum_i q_i exp(i G.r_i), Q = sum_i q_i. */
double or_ewald_energy(const double lat[9], int64_t n, const double* pos, const double* q,
                       double alpha, double rcut, int kmax) {
    const double pi = 3.14159265358979323846;
    or_ewald_defaults(lat, &alpha, &rcut, &kmax);
    cell_t c;
    cell_setup(lat, &c);
    double ke = or_coulomb_constant();
    double ereal = 0.0;
#pragma omp parallel for reduction(+ : ereal) schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double r[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1], pos[3 * j + 2] - pos[3 * i + 2]};
            acc += q[i] * q[j] * psi_real(&c, r, alpha, rcut);
        }
        ereal += acc;
    }
    ereal *= 0.5;
    double erecip = 0.0;
    for (int n0 = -kmax; n0 <= kmax; ++n0)
        for (int n1 = -kmax; n1 <= kmax; ++n1)
            for (int n2 = -kmax; n2 <= kmax; ++n2) {
                if (n0 == 0 && n1 == 0 && n2 == 0) continue;
                if (n0 * n0 + n1 * n1 + n2 * n2 > kmax * kmax) continue;
                double G[3];
                for (int k = 0; k < 3; ++k) G[k] = n0 * c.B[0][k] + n1 * c.B[1][k] + n2 * c.B[2][k];
                double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                double sre = 0.0, sim = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    double gr = G[0] * pos[3 * i] + G[1] * pos[3 * i + 1] + G[2] * pos[3 * i + 2];
                    sre += q[i] * cos(gr);
                    sim += q[i] * sin(gr);
                }
                erecip += exp(-g2 / (4.0 * alpha * alpha)) / g2 * (sre * sre + sim * sim);
            }
    erecip *= 2.0 * pi / c.vol;
    double q2 = 0.0, qs = 0.0;
    for (int64_t i = 0; i < n; ++i) { q2 += q[i] * q[i]; qs += q[i]; }
    double eself = -alpha / sqrt(pi) * q2;
    double ebg = -pi * qs * qs / (2.0 * c.vol * alpha * alpha);
    return ke * (ereal + erecip + eself + ebg);
}

/* ------------------------------------------------------------------------- */
/* Energies: the exact second-order cluster expansion of point charges,         */
/* E(q) = 1/2 sum_i sum_j q_i q_j V_ij, by a plain double loop.                 */
/* ------------------------------------------------------------------------- */
double or_energy_q(const double* V, int64_t n, const double* q) {
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) e += q[i] * q[j] * V[i * n + j];
    return 0.5 * e;
}

void or_energies(const double* V, int64_t n, int64_t P, const uint8_t* occ, const double* charge,
                 double* E) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < P; ++p) {
        double* q = (double*)malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) q[i] = charge[occ[p * n + i]];
        E[p] = or_energy_q(V, n, q);
        free(q);
    }
}

/* ------------------------------------------------------------------------- */
/* Problem bookkeeping shared by the stochastic routines below.                 */
/* Mobile positions are the sites with sublattice >= 0, in ascending site order. */
/* For sublattice s: P_s positions; n_{s,e} ions of species e (fixed by the     */
/* occupancy constraint); off_{s,e} = sum_{e' < e} n_{s,e'}.                    */
/* ------------------------------------------------------------------------- */
#define OR_MAXS 64
#define OR_MAXE 256

typedef struct {
    int64_t n, M;
    int32_t S, E;            /* sublattices, species */
    int64_t* mob;            /* M: site index of each mobile position */
    int32_t* msub;           /* M: sublattice of each mobile position */
    int64_t subsize[OR_MAXS];
    int64_t suboff[OR_MAXS]; /* offset of sublattice s in the concatenated perm */
    int64_t cnt[OR_MAXS][OR_MAXE];
    int64_t off[OR_MAXS][OR_MAXE];
} prob_t;

static int prob_setup(prob_t* pb, int64_t n, const int32_t* sub, const uint8_t* occ, int32_t n_species) {
    memset(pb, 0, sizeof(*pb));
    pb->n = n;
    pb->E = n_species;
    int32_t S = 0;
    int64_t M = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (sub[i] >= OR_MAXS) return -1;
        if (sub[i] >= 0) { ++M; if (sub[i] + 1 > S) S = sub[i] + 1; }
    }
    pb->S = S;
    pb->M = M;
    pb->mob = (int64_t*)malloc(sizeof(int64_t) * (size_t)(M ? M : 1));
    pb->msub = (int32_t*)malloc(sizeof(int32_t) * (size_t)(M ? M : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (sub[i] >= 0) {
            pb->mob[k] = i;
            pb->msub[k] = sub[i];
            pb->subsize[sub[i]]++;
            pb->cnt[sub[i]][occ[i]]++;
            ++k;
        }
    int64_t acc = 0;
    for (int32_t s = 0; s < S; ++s) {
        pb->suboff[s] = acc;
        acc += pb->subsize[s];
        int64_t o = 0;
        for (int32_t e = 0; e < n_species; ++e) { pb->off[s][e] = o; o += pb->cnt[s][e]; }
    }
    return 0;
}

static void prob_free(prob_t* pb) { free(pb->mob); free(pb->msub); }

/* perm: per sublattice, the mobile positions sorted by (species, position) */
static void perm_sorted(const prob_t* pb, const uint8_t* occ, int32_t* perm) {
    for (int32_t s = 0; s < pb->S; ++s) {
        int64_t w = pb->suboff[s];
        for (int32_t e = 0; e < pb->E; ++e)
            for (int64_t k = 0; k < pb->M; ++k)
                if (pb->msub[k] == s && occ[pb->mob[k]] == e) perm[w++] = (int32_t)k;
    }
}

/* ------------------------------------------------------------------------- */
/* Random valid start (SI, "Random"): per sublattice, the canonical sequence of  */
/* species (ascending id, n_{s,e} copies each) is shuffled by Fisher-Yates,     */
/* k = P_s - 1 .. 1, m = (r (k + 1)) >> 32 with r the first Philox word at       */
/* counter (k, s, chain, instance << 8 | TAG_INIT); entry k of the shuffled      */
/* sequence goes to the k-th position of s in ascending order.                   */
/* ------------------------------------------------------------------------- */
int or_init_occupations(int64_t n, const int32_t* sub, const uint8_t* species, int32_t n_species,
                        int64_t C, uint64_t seed, uint32_t chain_base, uint32_t instance, uint8_t* occ) {
    prob_t pb;
    if (prob_setup(&pb, n, sub, species, n_species)) return -1;
    for (int64_t ch = 0; ch < C; ++ch) {
        uint8_t* o = occ + ch * n;
        memcpy(o, species, (size_t)n);
        for (int32_t s = 0; s < pb.S; ++s) {
            int64_t Ps = pb.subsize[s];
            uint8_t* arr = (uint8_t*)malloc((size_t)(Ps ? Ps : 1));
            int64_t w = 0;
            for (int32_t e = 0; e < n_species; ++e)
                for (int64_t c = 0; c < pb.cnt[s][e]; ++c) arr[w++] = (uint8_t)e;
            for (int64_t k = Ps - 1; k >= 1; --k) {
                uint32_t r[4];
                philox4((uint32_t)k, (uint32_t)s, chain_base + (uint32_t)ch, (instance << 8) | TAG_INIT, seed, r);
                int64_t m = (int64_t)(((uint64_t)r[0] * (uint64_t)(k + 1)) >> 32);
                uint8_t tmp = arr[k]; arr[k] = arr[m]; arr[m] = tmp;
            }
            int64_t kk = 0;
            for (int64_t k = 0; k < pb.M; ++k)
                if (pb.msub[k] == s) o[pb.mob[k]] = arr[kk++];
            free(arr);
        }
    }
    prob_free(&pb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Metropolis swap Monte Carlo with an annealing table (SI, "Monte Carlo",       */
/* "Simulated annealing"). Per chain: occ (n sites), perm (M), counters.         */
/* phi_k = sum_l V_kl q_l over all sites is recomputed from occ at entry.        */
/* Trial t:                                                                      */
/*   (r0..r3) = Philox(ctr = (t_lo, t_hi, chain, instance << 8 | TAG_MC), seed)  */
/*   i = (r0 M) >> 32 (mobile index), s its sublattice, a its species,           */
/*   c = P_s - n_{s,a}; c == 0 is a rejected null trial with j = i               */
/*   k = (r1 c) >> 32, j = perm_s[k < off_{s,a} ? k : k + n_{s,a}], b its species */
/*   d = q_b - q_a, dE = d (phi_i - phi_j) + 1/2 d d (V_ii + V_jj - 2 V_ij)       */
/*   u = ((r2:r3 >> 12) + 1/2) 2^-52, kT = table[row][min(t / B, nb - 1)] with    */
/*   row = kT_row[chain] (0 when no rows are given)                              */
/*   accept iff dE <= 0 or u < exp(-dE / kT)                                     */
/*   on accept: swap occ, swap the two perm entries, phi_k += d (V_ik - V_jk)    */
/*   for all mobile k when d != 0, E += dE, best kept on strict improvement      */
/*   hash += splitmix64(splitmix64(t) ^ (i << 33 | j << 1 | accepted))           */
/* init_perm: 1 starts the chains (counters zero, best = start); 0 resumes them; */
/* 2 reloads them from new occupations (counters and trial index kept, position  */
/* lists rebuilt, best replaced only by a strictly lower start).                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t t;          /* trials done so far                                  */
    uint64_t accepts;    /* accepted trials                                     */
    uint64_t updates;    /* accepted trials with d != 0 (field updates)        */
    uint64_t hash;       /* sum of per-trial hashes mod 2^64                    */
    double E;            /* energy after the last trial                         */
    double best_E;       /* lowest energy seen (strict improvements)            */
    double min_margin;   /* min |dE + kT ln u| over the trials of this call     */
} or_chain_stats;

int or_mc_run(const double* V, int64_t n, const int32_t* sub, const double* charge, int32_t n_species,
              int64_t C, uint8_t* occ, int32_t* perm, uint8_t* best_occ, or_chain_stats* st,
              uint64_t seed, uint32_t chain_base, uint32_t instance, uint64_t n_trials,
              const double* kT, int32_t n_blocks, uint64_t block_len, const int32_t* kT_row,
              int32_t init_perm) {
    if (n_blocks <= 0 || block_len == 0) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t ch = 0; ch < C; ++ch) {
        uint8_t* o = occ + ch * n;
        prob_t pb;
        if (prob_setup(&pb, n, sub, o, n_species)) { err |= 1; continue; }
        const int64_t M = pb.M;
        int32_t* pm = perm + ch * (M ? M : 1);
        or_chain_stats* S = &st[ch];
        if (init_perm == 1) {
            perm_sorted(&pb, o, pm);
            memset(S, 0, sizeof(*S));
        } else if (init_perm == 2) {
            perm_sorted(&pb, o, pm);   /* reload: new occupation, counters kept */
        }
        int32_t* where = (int32_t*)malloc(sizeof(int32_t) * (size_t)(M ? M : 1));
        for (int64_t k = 0; k < M; ++k) where[pm[k]] = (int32_t)k;
        double* q = (double*)malloc(sizeof(double) * (size_t)n);
        double* phi = (double*)malloc(sizeof(double) * (size_t)(M ? M : 1));
        for (int64_t i = 0; i < n; ++i) q[i] = charge[o[i]];
        for (int64_t k = 0; k < M; ++k) {
            double f = 0.0;
            for (int64_t l = 0; l < n; ++l) f += V[pb.mob[k] * n + l] * q[l];
            phi[k] = f;
        }
        double E = or_energy_q(V, n, q);
        if (init_perm == 1 || (init_perm == 2 && E < S->best_E)) {
            S->best_E = E;
            memcpy(best_occ + ch * n, o, (size_t)n);
        }
        S->min_margin = INFINITY;
        for (uint64_t tt = 0; tt < n_trials; ++tt) {
            const uint64_t t = S->t + tt;
            uint32_t r[4];
            philox4((uint32_t)t, (uint32_t)(t >> 32), chain_base + (uint32_t)ch, (instance << 8) | TAG_MC, seed, r);
            int64_t im = M ? (int64_t)(((uint64_t)r[0] * (uint64_t)M) >> 32) : 0;
            if (M == 0) { S->hash += or_trial_hash(t, 0, 0, 0); continue; }
            int32_t s = pb.msub[im];
            int64_t si = pb.mob[im];
            uint8_t a = o[si];
            int64_t c = pb.subsize[s] - pb.cnt[s][a];
            if (c == 0) { S->hash += or_trial_hash(t, (uint32_t)im, (uint32_t)im, 0); continue; }
            int64_t k = (int64_t)(((uint64_t)r[1] * (uint64_t)c) >> 32);
            int64_t idx = k < pb.off[s][a] ? k : k + pb.cnt[s][a];
            int64_t jm = pm[pb.suboff[s] + idx];
            int64_t sj = pb.mob[jm];
            uint8_t b = o[sj];
            double d = charge[b] - charge[a];
            double dE = d * (phi[im] - phi[jm]) + 0.5 * d * d * (V[si * n + si] + V[sj * n + sj] - 2.0 * V[si * n + sj]);
            double u = unit_open(r[2], r[3]);
            uint64_t blk = t / block_len;
            const double* tab = kT + (kT_row ? (int64_t)kT_row[ch] * n_blocks : 0);
            double kt = tab[blk < (uint64_t)n_blocks ? blk : (uint64_t)(n_blocks - 1)];
            int acc = (dE <= 0.0) || (u < exp(-dE / kt));
            double margin = fabs(dE + kt * log(u));
            if (margin < S->min_margin) S->min_margin = margin;
            if (acc) {
                o[si] = b; o[sj] = a;
                int32_t wi = where[im], wj = where[jm];
                pm[wi] = (int32_t)jm; pm[wj] = (int32_t)im;
                where[im] = wj; where[jm] = wi;
                q[si] = charge[b]; q[sj] = charge[a];
                if (d != 0.0) {
                    for (int64_t kk = 0; kk < M; ++kk)
                        phi[kk] += d * (V[si * n + pb.mob[kk]] - V[sj * n + pb.mob[kk]]);
                    S->updates++;
                }
                E += dE;
                S->accepts++;
                if (E < S->best_E) { S->best_E = E; memcpy(best_occ + ch * n, o, (size_t)n); }
            }
            S->hash += or_trial_hash(t, (uint32_t)im, (uint32_t)jm, (uint32_t)acc);
        }
        S->t += n_trials;
        S->E = E;
        free(where); free(q); free(phi);
        prob_free(&pb);
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Gradient descent (SI, "Gradient Descent"): from each start, every neighbour  */
/* reachable by one swap of two ions of different species on the same site      */
/* class is scored by dE (the Monte Carlo trial's expression, with the field     */
/* phi_k = sum_l V_kl q_l over all sites) and the best one is applied, until no  */
/* neighbour lies lower. Reading of "the lowest-energy neighbour": among the     */
/* swaps (i, j), i < j in mobile order, whose dE lies within tol of the lowest   */
/* dE, the lexicographically smallest; symmetry-equivalent neighbours have equal */
/* energies that any implementation only resolves to rounding noise, and the    */
/* window makes the choice independent of it. Descent stops when the lowest dE  */
/* is >= -tol (a local minimum) or after max_steps swaps.                        */
/* ------------------------------------------------------------------------- */
int or_gd_run(const double* V, int64_t n, const int32_t* sub, const double* charge, int32_t n_species,
              int64_t P, uint8_t* occ, int64_t max_steps, double tol, int64_t* steps, double* E_out) {
    if (!(tol >= 0.0) || max_steps < 0) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t p = 0; p < P; ++p) {
        uint8_t* o = occ + p * n;
        prob_t pb;
        if (prob_setup(&pb, n, sub, o, n_species)) { err |= 1; continue; }
        const int64_t M = pb.M;
        double* q = (double*)malloc(sizeof(double) * (size_t)n);
        double* phi = (double*)malloc(sizeof(double) * (size_t)(M ? M : 1));
        for (int64_t i = 0; i < n; ++i) q[i] = charge[o[i]];
        for (int64_t k = 0; k < M; ++k) {
            double f = 0.0;
            for (int64_t l = 0; l < n; ++l) f += V[pb.mob[k] * n + l] * q[l];
            phi[k] = f;
        }
        double E = or_energy_q(V, n, q);
        int64_t st = 0;
        while (st < max_steps) {
            /* lowest dE over all neighbours */
            double lo = INFINITY;
            for (int64_t i = 0; i < M; ++i)
                for (int64_t j = i + 1; j < M; ++j) {
                    const int64_t si = pb.mob[i], sj = pb.mob[j];
                    if (pb.msub[i] != pb.msub[j] || o[si] == o[sj]) continue;
                    const double d = charge[o[sj]] - charge[o[si]];
                    const double dE = d * (phi[i] - phi[j]) +
                                      0.5 * d * d * (V[si * n + si] + V[sj * n + sj] - 2.0 * V[si * n + sj]);
                    if (dE < lo) lo = dE;
                }
            if (!(lo < -tol)) break;
            /* first swap (lexicographic) within tol of the lowest */
            int64_t bi = -1, bj = -1;
            double bdE = 0.0;
            for (int64_t i = 0; i < M && bi < 0; ++i)
                for (int64_t j = i + 1; j < M; ++j) {
                    const int64_t si = pb.mob[i], sj = pb.mob[j];
                    if (pb.msub[i] != pb.msub[j] || o[si] == o[sj]) continue;
                    const double d = charge[o[sj]] - charge[o[si]];
                    const double dE = d * (phi[i] - phi[j]) +
                                      0.5 * d * d * (V[si * n + si] + V[sj * n + sj] - 2.0 * V[si * n + sj]);
                    if (dE <= lo + tol) { bi = i; bj = j; bdE = dE; break; }
                }
            const int64_t si = pb.mob[bi], sj = pb.mob[bj];
            const uint8_t a = o[si], b = o[sj];
            const double d = charge[b] - charge[a];
            o[si] = b; o[sj] = a;
            q[si] = charge[b]; q[sj] = charge[a];
            for (int64_t kk = 0; kk < M; ++kk) phi[kk] += d * (V[si * n + pb.mob[kk]] - V[sj * n + pb.mob[kk]]);
            E += bdE;
            ++st;
        }
        steps[p] = st;
        E_out[p] = E;
        free(q); free(phi);
        prob_free(&pb);
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Replica exchange (SI, "Replica Exchange Monte Carlo"): replicas sit on a      */
/* temperature ladder kT_0 < kT_1 < ...; at exchange step x, neighbour pairs     */
/* (k, k+1) with k = x mod 2, x mod 2 + 2, ... attempt to swap configurations    */
/* and accept with probability min(1, exp((E_k - E_{k+1}) (1/kT_k - 1/kT_{k+1})))*/
/* using u from Philox(ctr = (k, x_lo, x_hi, group << 8 | TAG_REMC), seed).       */
/* slot[k] names the replica currently at temperature k; accepted swaps exchange */
/* slot entries (configurations move, temperatures stay).                        */
/* ------------------------------------------------------------------------- */
int or_remc_exchange(int32_t R, const double* kT, const double* E, int32_t* slot, uint64_t x,
                     uint64_t seed, uint32_t group, uint8_t* accepted) {
    for (int32_t k = (int32_t)(x & 1u); k + 1 < R; k += 2) {
        uint32_t r[4];
        philox4((uint32_t)k, (uint32_t)x, (uint32_t)(x >> 32), (group << 8) | TAG_REMC, seed, r);
        double u = unit_open(r[0], r[1]);
        double Ea = E[slot[k]], Eb = E[slot[k + 1]];
        double arg = (Ea - Eb) * (1.0 / kT[k] - 1.0 / kT[k + 1]);
        int acc = (arg >= 0.0) || (u < exp(arg));
        if (accepted) accepted[k] = (uint8_t)acc;
        if (acc) { int32_t tmp = slot[k]; slot[k] = slot[k + 1]; slot[k + 1] = tmp; }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Genetic algorithm generation (SI, "Genetic Algorithm").                       */
/*  1. elitism: children 0..n_elite-1 are the parents ordered by (E, index)      */
/*  2. roulette weights w_p = E_max - E_p as integers round(w_p 2^30), summed    */
/*     exactly; W = 0 means uniform choice                                       */
/*  3. parents of child c >= n_elite: r = Philox(ctr = (c, g, 0, TAG_SEL));      */
/*     x_A = r0:r1, x_B = r2:r3 (64 bit); target = floor(x W / 2^64); parent =   */
/*     smallest p with cum_p > target (uniform: floor(x P / 2^64))               */
/*  4. swap crossover: the canonical swap path from A to B is walked on a copy   */
/*     ref = A: per sublattice, positions p ascending with ref[p] != B[p] pair   */
/*     with the smallest later q of the sublattice with ref[q] = B[p] and        */
/*     ref[q] != B[q] (one always exists: ref and B share the composition and    */
/*     agree below p); ref swaps p and q. The child (= A) takes that swap iff    */
/*     the top bit of Philox(ctr = (p, c, g, TAG_X)).r0 is set, so each swap of  */
/*     the path from A to B is accepted with probability 1/2                     */
/*  5. mutation: r = Philox(ctr = (c, g, 1, TAG_MUT)); if u(r2:r3) < p_mut, one  */
/*     swap picked as in the MC trial from r0, r1, with the sublattice's         */
/*     positions ordered by (species, position) in the child                     */
/* ------------------------------------------------------------------------- */
int or_ga_generation(int64_t n, const int32_t* sub, int32_t n_species, int64_t P, const uint8_t* pop_in,
                     const double* E_in, uint64_t seed, uint32_t g, int32_t n_elite, double p_mut,
                     uint8_t* pop_out) {
    if (P <= 0) return 0;
    prob_t pb;
    if (prob_setup(&pb, n, sub, pop_in, n_species)) return -1;
    const int64_t M = pb.M;
    /* 1. elitism */
    int64_t ne = n_elite < 0 ? 0 : (n_elite > P ? P : n_elite);
    for (int64_t c = 0; c < ne; ++c) {
        /* the c-th smallest (E, index) pair, by counting */
        for (int64_t p = 0; p < P; ++p) {
            int64_t rank = 0;
            for (int64_t q2 = 0; q2 < P; ++q2)
                if (E_in[q2] < E_in[p] || (E_in[q2] == E_in[p] && q2 < p)) ++rank;
            if (rank == c) { memcpy(pop_out + c * n, pop_in + p * n, (size_t)n); break; }
        }
    }
    /* 2. roulette weights */
    double emax = E_in[0];
    for (int64_t p = 1; p < P; ++p) if (E_in[p] > emax) emax = E_in[p];
    uint64_t* cum = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P);
    uint64_t W = 0;
    const double lim = ldexp(1.0, 62) / (double)P;
    int bad = 0;
    for (int64_t p = 0; p < P; ++p) {
        double w = (emax - E_in[p]) * 0x1p30;
        if (!(w < lim)) bad = 1;
        uint64_t wq = bad ? 0 : (uint64_t)(w + 0.5);
        W += wq;
        cum[p] = W;
    }
    if (bad) { free(cum); prob_free(&pb); return -2; }
    uint8_t* ref = (uint8_t*)malloc((size_t)n);
    for (int64_t c = ne; c < P; ++c) {
        uint32_t r[4];
        philox4((uint32_t)c, g, 0u, TAG_SEL, seed, r);
        uint64_t xs[2] = {((uint64_t)r[0] << 32) | r[1], ((uint64_t)r[2] << 32) | r[3]};
        int64_t par[2];
        for (int h = 0; h < 2; ++h) {
            if (W == 0) {
                par[h] = (int64_t)(((unsigned __int128)xs[h] * (uint64_t)P) >> 64);
            } else {
                uint64_t target = (uint64_t)(((unsigned __int128)xs[h] * W) >> 64);
                int64_t p = 0;
                while (!(cum[p] > target)) ++p;
                par[h] = p;
            }
        }
        const uint8_t* A = pop_in + par[0] * n;
        const uint8_t* B = pop_in + par[1] * n;
        uint8_t* ch = pop_out + c * n;
        memcpy(ch, A, (size_t)n);
        /* 4. swap crossover: walk the canonical swap path from A to B on a copy
         * (ref) and take each of its swaps into the child with probability 1/2 */
        memcpy(ref, A, (size_t)n);
        for (int32_t s = 0; s < pb.S; ++s) {
            for (int64_t p = 0; p < M; ++p) {
                if (pb.msub[p] != s) continue;
                int64_t sp = pb.mob[p];
                if (ref[sp] == B[sp]) continue;
                int64_t qq = -1;
                for (int64_t q2 = p + 1; q2 < M; ++q2) {
                    if (pb.msub[q2] != s) continue;
                    int64_t sq = pb.mob[q2];
                    if (ref[sq] == B[sp] && ref[sq] != B[sq]) { qq = q2; break; }
                }
                if (qq < 0) { free(ref); free(cum); prob_free(&pb); return -3; }  /* cannot happen */
                int64_t sq = pb.mob[qq];
                uint8_t tmp = ref[sp]; ref[sp] = ref[sq]; ref[sq] = tmp;
                uint32_t rx[4];
                philox4((uint32_t)p, (uint32_t)c, g, TAG_X, seed, rx);
                if (rx[0] >> 31) { tmp = ch[sp]; ch[sp] = ch[sq]; ch[sq] = tmp; }
            }
        }
        /* 5. mutation */
        uint32_t rm[4];
        philox4((uint32_t)c, g, 1u, TAG_MUT, seed, rm);
        if (M > 0 && unit_open(rm[2], rm[3]) < p_mut) {
            int64_t im = (int64_t)(((uint64_t)rm[0] * (uint64_t)M) >> 32);
            int32_t s = pb.msub[im];
            uint8_t a = ch[pb.mob[im]];
            int64_t cnum = pb.subsize[s] - pb.cnt[s][a];
            if (cnum > 0) {
                int64_t k = (int64_t)(((uint64_t)rm[1] * (uint64_t)cnum) >> 32);
                int64_t idx = k < pb.off[s][a] ? k : k + pb.cnt[s][a];
                /* idx-th entry of the sublattice ordered by (species, position) */
                int64_t seen = 0, jm = -1;
                for (int32_t e = 0; e < n_species && jm < 0; ++e)
                    for (int64_t q2 = 0; q2 < M; ++q2)
                        if (pb.msub[q2] == s && ch[pb.mob[q2]] == e) {
                            if (seen == idx) { jm = q2; break; }
                            ++seen;
                        }
                int64_t si = pb.mob[im], sj = pb.mob[jm];
                uint8_t tmp = ch[si]; ch[si] = ch[sj]; ch[sj] = tmp;
            }
        }
    }
    free(ref);
    free(cum);
    prob_free(&pb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The k lowest configurations: FP64 energies (double loop), ordered by          */
/* (E, index).                                                                   */
/* ------------------------------------------------------------------------- */
int or_topk(const double* V, int64_t n, int64_t P, const uint8_t* occ, const double* charge, int32_t k,
            int64_t* idx_out, double* E_out) {
    double* E = (double*)malloc(sizeof(double) * (size_t)(P ? P : 1));
    or_energies(V, n, P, occ, charge, E);
    int64_t kk = k < P ? k : P;
    for (int64_t p = 0; p < P; ++p) {
        int64_t rank = 0;
        for (int64_t q = 0; q < P; ++q)
            if (E[q] < E[p] || (E[q] == E[p] && q < p)) ++rank;
        if (rank < kk) { idx_out[rank] = p; E_out[rank] = E[p]; }
    }
    free(E);
    return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
