// Shared declarations of the gfx950 library: device structs, the counter-based
// RNG, the trajectory hash and launch helpers. Host and device code of the
// library include this; the CPU oracle does not.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/goac.h"
#include "lifetime.h"

namespace goac {

constexpr int kMaxSub = 16;       // sublattices per problem
constexpr int kMaxSpecies = 32;   // species ids per problem
constexpr int kPad = 64;          // mobile dimension padded to a multiple of this
constexpr int kBestLog = 256;     // multi-wave chains: swaps logged between best-occupation copies

enum : uint32_t { TAG_MC = 1, TAG_INIT = 2, TAG_SEL = 3, TAG_X = 4, TAG_MUT = 5, TAG_REMC = 6 };

__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products of counter words 0 and 2 with fixed multipliers, the high
// halves xor-ed with the other counter words and the round key, which advances by
// the Weyl constants after every round. Each three-way xor is one gfx950
// three-input bitwise instruction (truth table 0x96, the parity of its inputs).
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ inline u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// uniform on (0, 1): 52 high bits of hi:lo plus one half, times 2^-52 (exact)
__host__ __device__ inline double unit_open(uint32_t hi, uint32_t lo) {
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

// multiply-shift index in [0, n)
__host__ __device__ inline uint32_t mulshift(uint32_t r, uint32_t n) {
    return (uint32_t)(((uint64_t)r * n) >> 32);
}

// splitmix64 output function (Steele, Lea, Flood, OOPSLA'14)
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// per-trial term of the order-independent trajectory hash (sum mod 2^64)
__host__ __device__ inline uint64_t trial_hash(uint64_t t, uint32_t i, uint32_t j, uint32_t acc) {
    return splitmix64(splitmix64(t) ^ (((uint64_t)i << 33) | ((uint64_t)j << 1) | (acc & 1u)));
}

// ------------------------------------------------------------------ address spaces
// Pointers read out of device memory (instance tables) are generic to the
// compiler, which then emits flat loads; flat loads also count against the LDS
// wait counter, so an LDS read after one stalls until the global load returns.
// Casting to the global address space restores global loads.
#define GOAC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GOAC_GLOBAL T* gptr(const T* p) {
    return (const GOAC_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ GOAC_GLOBAL T* gptr_rw(T* p) {
    return (GOAC_GLOBAL T*)p;
}

// ------------------------------------------------------------------ device structs

// Sublattice tables of a problem, laid out as int32 words:
//   [0]            S
//   [1]            E
//   [2 .. 2+S)     P_s  (positions of sublattice s)
//   [.. + S)       start of sublattice s in the concatenated position lists
//   [.. + S*E)     n_{s,e} (ions of species e on sublattice s)
//   [.. + S*E)     off_{s,e} = sum_{e' < e} n_{s,e'}
__host__ __device__ inline int tab_words(int S, int E) { return 2 + 2 * S + 2 * S * E; }

struct ProblemDev {
    int64_t n;
    int32_t M, Mp, S, E;
    int32_t Mq;          // M padded to the population product's 128-wide tiles
    int32_t* mob;        // M: site index of mobile position k (ascending)
    uint8_t* msub;       // Mp: sublattice of position k (0 beyond M)
    uint8_t* ref_occ;    // n: the problem's occupation (fixed-site species)
    int8_t* site_sub;    // n: site class of each site (-1 fixed)
    double* V64;         // M x Mp: mobile block, FP64 (zero beyond M)
    float* V32;          // M x Mp: FP32 rounding of V64
    __hip_bfloat16* Vhi; // Mq x Mq: bf16(W), W = V block-lower-triangular with halved
                         // diagonal 128 x 128 blocks (the population product's weights)
    __hip_bfloat16* Vlo; // Mq x Mq: bf16(W - Vhi)
    double* diag;        // M
    float* rowmax;       // M: max_k |V_ik|, rounded up
    double* rowabs;      // M: sum_k |V_ik|
    double* h;           // Mp: field of the fixed ions
    double* ht;          // Mp: h + V_mm c
    double* phibar;      // S: mean field of each sublattice at the reference occupation
    double* charge;      // E
    double* dq;          // S x E: charge[e] - c_s
    int32_t* tab;        // sublattice tables (tab_words)
    const double* Ed;    // 2: E_ff (energy of the fixed ions), E_t = E_ff + c^T h + 1/2 c^T V_mm c
    double qmax;         // max |charge|
    int mixed_exact;
};

// Per-chain scalars of the Monte Carlo state (device array, one per chain).
struct ChainScalars {
    uint64_t t, accepts, updates, hash, fallbacks, anchors;
    double E, best_E;
    double eps;              // bound on |phi32 - phi| (MIXED)
    float phibound;          // power-of-two bound on |phi| (MIXED)
    uint32_t since_anchor;   // field updates since the last FP64 anchor
    int32_t inst;            // instance index
    uint32_t chain_id;       // chain id in the Philox counters
    int32_t row;             // temperature row
    int32_t status;          // 0, or 1 once the field left its bound
    int64_t off;             // element offset of the chain's arrays
};

// Per-instance view the Monte Carlo kernels read.
struct McInst {
    const double* V64;
    const float* V32;
    const double* diag;
    const float* rowmax;
    const double* h;
    const double* phibar;   // S: offset of the stored FP32 field per sublattice
    const uint8_t* msub;
    const int32_t* tab;
    const double* charge;
    const double* Ed;       // E_ff, E_t of the instance
    int32_t M, Mp, S, E;
    uint32_t instance;      // instance id in the Philox counters
    int32_t pad_;
};

}  // namespace goac

// ------------------------------------------------------------------ host objects
namespace goac {
// Device interface of the context's block cache and lifetime (lifetime.h): HIP
// memory whose users are ordered by the context's stream.
struct HipDev {
    hipStream_t stream = nullptr;
    bool alloc(void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; }
    void release(void* p) { (void)hipFree(p); }
    void drain() { (void)hipStreamSynchronize(stream); }
};
constexpr size_t kPoolMaxBytes = (size_t)8 << 30;  // released blocks a context keeps
}  // namespace goac

constexpr int kWsSlots = 3;   // scratch slots: 0 kernels' operands, 1 GEMM partials, 2 selection
// host-side tables of the last Ewald build and the inputs they were made from
struct EwaldPlan {
    int64_t n = -1;                 // -1: no valid plan
    double lat[9] = {};
    std::vector<double> pos;
    double alpha_in = 0.0, rcut_in = 0.0;
    int32_t kmax_in = 0;
    std::vector<char> img;          // fractional | folded positions | translations | G | lattice
    size_t b_frac = 0, b_pos = 0, b_tr = 0, b_G = 0, b_A = 0;
    int32_t K = 0, ld = 0, ntrans = 0;
    double alpha = 0.0, rcut = 0.0, ke = 0.0, cst = 0.0, self = 0.0;
    int32_t flags_in = 0;
    // translation symmetry of the sites: the grid Z_m0 x Z_m1 x Z_m2 of axis-aligned
    // fractional translations that map the site set onto itself (nb = 0: none found).
    // Site i is translate g_i of representative b_i; idx[b][g] is the site translate
    // g of representative b. Uploaded after the general tables: reps (nb), site_b (n),
    // site_g (n, packed), idx (n), int32 each.
    int32_t nb = 0, ng = 0;
    int32_t m[3] = {1, 1, 1};
    size_t b_sym = 0;
};

struct goac_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    std::string err;
    void* ws[kWsSlots] = {nullptr, nullptr, nullptr};  // scratch, grown on demand
    size_t ws_size[kWsSlots] = {0, 0, 0};
    goac::HipDev dev;                   // the stream-ordered device of the block cache
    goac::BlockCache<goac::HipDev> pool{goac::kPoolMaxBytes};  // released arenas, reused by later ones
    // pinned staging of host-to-device copies: two halves, each with the event
    // recorded after the copies last queued from it
    char* stage = nullptr;
    size_t stage_half = 0, stage_off = 0;
    int stage_cur = 0;
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_pending[2] = {false, false};
    bool capturing = false;  // a stream capture is open on the context's work
    hipStream_t cap = nullptr;  // private stream that graph captures record on (created on first use)
    EwaldPlan ewald;            // reused by a build of the same cell and parameters
    goac::Holders holders;      // the caller's handle and the live problems and chain sets
    // verdict of the last check of caller rows (composition, species ids) or of the
    // chains' drift flags: a device word that kernels queued after the check read,
    // its pinned host copy and the event recorded after that copy
    int32_t* chk_dev = nullptr;
    int32_t* chk_host = nullptr;
    hipEvent_t chk_ev = nullptr;
};

struct goac_problem {
    goac_ctx* ctx = nullptr;
    goac::ProblemDev d{};
    std::vector<int32_t> tab_host;  // tables on the host
    std::vector<int32_t> mob_host;
    std::vector<double> charge_host;
    std::vector<double> shift_host;  // c_s
    int32_t* spos = nullptr;         // M: positions of each sublattice, ascending, concatenated
    int32_t* spos_inv = nullptr;     // M: index of position k in spos
    int32_t* ssite = nullptr;        // M: site of entry x of spos (mob[spos[x]])
    int32_t* fixed_idx = nullptr;    // fixed sites
    int32_t n_fixed = 0;
    mutable bool e_host = false;     // E_ff, E_t read back (on the first request)
    mutable double E_ff = 0.0, E_t = 0.0;
    void* arena = nullptr;           // one allocation holding every device array
    size_t arena_bytes = 0;
    std::map<int64_t, int32_t> pop_kt;  // population size -> n-tiles per K block of the
                                        // mixed energies (set or tuned; else the cost model)
};

struct goac_chains {
    goac_ctx* ctx = nullptr;
    std::vector<goac_problem*> pbs;   // one per instance
    goac_precision prec = GOAC_FP64;
    int64_t C = 0;                    // chains
    int64_t total = 0;                // elements of the per-chain arrays
    int32_t max_Mp = 0;
    int32_t max_S = 1, max_E = 1;
    goac::ChainScalars* sc = nullptr; // C
    goac::McInst* insts = nullptr;    // instances
    void* phi = nullptr;              // float or double, total
    uint8_t* occ = nullptr;           // total
    uint16_t* perm = nullptr;         // total
    uint8_t* best = nullptr;          // total
    int32_t* order = nullptr;         // C, longest chains first
    int32_t* queue = nullptr;         // work counter of the persistent sweep
    void* arena = nullptr;            // one allocation holding every array below
    size_t arena_bytes = 0;
    double* kT = nullptr;             // device kT table
    size_t kT_cap = 0;
    int64_t* d_offs = nullptr;        // C element offsets (device)
    int32_t max_tab = 0;              // int32 words of the largest table
    int32_t max_row = 0;              // largest temperature row in use
    std::vector<int64_t> offs;        // element offsets per chain (host)
    std::vector<int32_t> inst_of;     // instance of each chain (host)
    std::vector<uint32_t> chain_id;   // Philox chain id of each chain
    std::vector<uint32_t> inst_id;    // Philox instance id of each instance
    std::vector<int64_t> count;       // chains per instance
    std::vector<int64_t> first_chain; // first chain of each instance
    std::vector<int64_t> occ_row_off; // byte offset of an instance's first occupation row
    void* scratch = nullptr;          // hybrid rounds: candidate rows, energies, ranks (grown on demand)
    size_t scratch_size = 0;
    int32_t tuned_wg = 0;             // launch configuration chosen by goac_chains_autotune (0: size rule)
    int32_t tuned_per_cu = 0;
    std::vector<double> kT_last;      // the kT table held in kT (uploads are skipped when unchanged)
    double* ladder = nullptr;         // replica-exchange ladder (device) and its host copy
    size_t ladder_cap = 0;
    std::vector<double> ladder_last;
    // GOAC_MC_TIMING: event pairs recorded around each Monte Carlo launch (kind 0)
    // and each batched anchor (kind 1) since the timings were last read
    std::vector<hipEvent_t> tev;
    std::vector<uint8_t> tev_kind;
    size_t tev_used = 0;
};

// ------------------------------------------------------------------ error helpers
namespace goac {

inline goac_status fail(goac_ctx* ctx, goac_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

#define GOAC_HIP(ctx, expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::goac::fail((ctx), e_ == hipErrorOutOfMemory ? GOAC_ENOMEM : GOAC_EHIP, \
                                std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define GOAC_CHECK_LAUNCH(ctx) GOAC_HIP(ctx, hipGetLastError())

// propagate a failed status
#define GOAC_TRY(expr)                \
    do {                              \
        goac_status s_ = (expr);      \
        if (s_ != GOAC_OK) return s_; \
    } while (0)

// Monte Carlo launch arguments
struct McArgs {
    const McInst* insts;
    ChainScalars* sc;
    void* phi;
    uint8_t* occ;
    uint16_t* perm;
    uint8_t* best;
    const int32_t* order;
    int32_t* queue;
    int32_t n_items;
    int32_t n_blocks;
    const double* kT;      // rows x n_blocks
    uint64_t block_len;
    uint64_t n_trials;
    uint64_t seed;
    int32_t reanchor_every;
    int32_t lds_phi_bytes; // bytes reserved for phi (Mp_max * sizeof)
    int32_t Mp_max;
    int32_t tab_max;       // int32 words reserved for tables
    int32_t inline_anchor; // MIXED: re-anchor inside the kernel (small cells) or leave it to
                           // the batched FP64 product between chunks (large cells)
    int32_t msub_lds;      // some instance has several site classes: their ids live in LDS
};

goac_status mc_launch(goac_ctx* ctx, const McArgs& a, bool mixed, bool trace, int wg, size_t lds, int grid);
goac_status build_q64(goac_ctx* ctx, int64_t P, int64_t n, int32_t M, int32_t Mp, int32_t E, const uint8_t* occ,
                      const int32_t* mob, const double* charge, double* Q, const int32_t* gate = nullptr);

// scratch memory of a context (grown, never shrunk)
goac_status workspace(goac_ctx* ctx, int slot, size_t bytes, void** out);

// Where a call takes its scratch: the context's workspace slots (base null), or a
// block the caller provides, carved in request order at 256-byte alignment.
struct WsSource {
    goac_ctx* ctx = nullptr;
    char* base = nullptr;
    size_t cap = 0, off = 0;
    goac_status get(int slot, size_t bytes, void** out) {
        if (!base) return workspace(ctx, slot, bytes, out);
        const size_t o = (off + 255) / 256 * 256;
        if (o + bytes > cap) return fail(ctx, GOAC_EINVAL, "scratch block too small");
        *out = base + o;
        off = o + bytes;
        return GOAC_OK;
    }
};

// arenas of problems and chain sets: a block released to the context is handed to
// the next arena that fits in it (at most twice its size); *bytes is rounded up
goac_status pool_get(goac_ctx* ctx, size_t* bytes, void** out);
// stream-ordered copy of host memory to the device through the pinned staging ring
goac_status upload(goac_ctx* ctx, void* dst, const void* src, size_t bytes);
void pool_put(goac_ctx* ctx, void* p, size_t bytes);

// Occupancy constraints of Eq. 2 on P caller rows (P x n): every mobile species id
// below the problem's species count and the species counts of every sublattice
// equal to the problem's. rows_check_enqueue queues the check and leaves its verdict
// in ctx->chk_dev (non-zero: a row breaks them), which kernels queued afterwards
// may read; rows_check_wait waits for that check alone and returns EINVAL on a
// broken row.
goac_status rows_check_enqueue(goac_problem* pb, int64_t P, const uint8_t* occ);
goac_status rows_check_wait(goac_ctx* ctx, const char* who);
inline goac_status rows_check(goac_problem* pb, int64_t P, const uint8_t* occ, const char* who) {
    GOAC_TRY(rows_check_enqueue(pb, P, occ));
    return rows_check_wait(pb->ctx, who);
}

// population energies (mixed bf16 hi+lo or FP64) and the k lowest of P energies
// by (E, index); cnt_scratch holds P int32. With a gate, the kernels that read the
// rows and write E do nothing while *gate is non-zero (rows a check rejected).
// The mixed path takes chk (an int32, zero on entry) instead: its row kernel checks
// the rows on the way and ors a broken row into *chk; the verdict is copied to *host
// (pinned) when host is set and ev (when set) recorded right after that kernel; E is
// left as it was when *chk is set.
goac_status energies_mixed(goac_problem* pb, int64_t P, const uint8_t* occ, double* E, int32_t kt = 0,
                           int32_t* chk = nullptr, WsSource* ws = nullptr, int32_t* host = nullptr,
                           hipEvent_t ev = nullptr);
goac_status energies_fp64(goac_problem* pb, int64_t P, const uint8_t* occ, double* E,
                          const int32_t* gate = nullptr, WsSource* ws = nullptr);
// scratch bytes (with the 256-byte alignment of WsSource) that energies of P rows take
size_t energies_scratch_bytes(const goac_problem* pb, int64_t P, goac_precision prec);
// launch of the composition check of P rows, or-ing a broken row into *flag
// (cleared first by the launch)
goac_status rows_check_launch(goac_problem* pb, int64_t P, const uint8_t* occ, int32_t* flag);
// copies of the chains' occupations, best occupations and counters (any may be
// null), queued on the stream without a wait
goac_status chains_export_enqueue(goac_chains* ch, uint8_t* occ, uint8_t* best, goac_chain_stats* stats);
// energies in either precision, without a check of the rows (rows the library made)
goac_status energies_enqueue(goac_problem* pb, int64_t P, const uint8_t* occ, goac_precision prec, double* E);
goac_status ga_generation_enqueue(goac_problem* pb, int64_t P, const uint8_t* pop_in, const double* E_in,
                                  const goac_ga_params* prm, uint8_t* pop_out, bool zero_err, int32_t** err_out,
                                  const uint32_t* g_dev = nullptr, bool check_first = false);
goac_status ga_check_err(goac_ctx* ctx, const int32_t* err);
goac_status rank_select(goac_ctx* ctx, int64_t P, const double* E, int32_t k, int32_t* cnt_scratch,
                        int64_t* idx64, int32_t* idx32, double* Eout);

// kernels shared across translation units
// C = alpha A B^T + beta C (FP64); sym: A = B and M = N, upper tiles computed and mirrored
goac_status dgemm_nt(goac_ctx* ctx, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                     const int32_t* M_dev, bool sym = false, WsSource* ws = nullptr);
// Looks up, once per device and with that device current, the device address of
// the allocation-free entry point's scratch array (noalloc.hip).
hipError_t noalloc_setup(int device);
// K splits of that product (its partials take splits x M x N doubles when > 1)
int dgemm_splits(const goac_ctx* ctx, int64_t M, int64_t N, int64_t K, const int32_t* M_dev, bool sym);

}  // namespace goac
