// Host side of the C ABI (include/fhe.h): parameter checks, constant tables,
// workspace layout and the launch sequences of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "fhe.h"
#include "kernels.hpp"
#include "modarith.hpp"
#include "ntt_core.hpp"
#include "tables.hpp"

// Workspace of fhe_mul_relin_static: one array per device, held by the
// loaded code object until the process ends.  In host code `scratch` only
// names the symbol; its device address (one per device) comes from
// hipGetSymbolAddress with that device current and is kept in scratch_dev.
static __device__ __align__(256) uint8_t scratch[FHE_STATIC_WS_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
fhe_status scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return FHE_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FHE_EDEVICE;
        scratch_dev[device] = ptr;
    }
    *out = scratch_dev[device];
    return FHE_OK;
}

// ------------------------------------------------------------ host math ----

uint64_t hmul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t hpow(uint64_t b, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = hmul(r, b, m);
        b = hmul(b, b, m);
        e >>= 1;
    }
    return r;
}

uint64_t hgcd(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Inverse of a modulo m (gcd(a, m) = 1), extended Euclid in signed 128-bit.
uint64_t hinv(uint64_t a, uint64_t m) {
    __int128 t = 0, nt = 1, r = m, nr = a % m;
    while (nr != 0) {
        __int128 qq = r / nr, tmp;
        tmp = t - qq * nt; t = nt; nt = tmp;
        tmp = r - qq * nr; r = nr; nr = tmp;
    }
    if (t < 0) t += m;
    return (uint64_t)t;
}

bool is_prime_u64(uint64_t n) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (uint64_t a : bases) {
        uint64_t x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; r++) {
            x = hmul(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }
uint64_t mont(uint64_t x, uint64_t q) { return (uint64_t)(((u128)(x % q) << 64) % q); }

uint64_t neg_inv64(uint64_t q) {  // -q^-1 mod 2^64 (q odd), Newton iteration
    uint64_t x = q;  // q * q = 1 mod 8
    for (int i = 0; i < 6; i++) x *= 2 - q * x;
    return (uint64_t)0 - x;
}

// psi = x^((q-1)/2n) for the smallest x >= 2 with psi^n = -1 mod q.
uint64_t find_psi(uint64_t q, uint32_t n) {
    for (uint64_t x = 2;; x++) {
        uint64_t psi = hpow(x, (q - 1) / (2 * (uint64_t)n), q);
        if (hpow(psi, n, q) == q - 1) return psi;
    }
}

uint32_t bitrev(uint32_t x, int L) {
    uint32_t r = 0;
    for (int i = 0; i < L; i++) r |= ((x >> i) & 1u) << (L - 1 - i);
    return r;
}

// Smallest primitive root of the prime t (trial-division factorisation of t-1).
bool primitive_root(uint64_t t, uint64_t *g) {
    std::vector<uint64_t> f;
    uint64_t m = t - 1;
    for (uint64_t p = 2; p * p <= m && p < (1ull << 22); p++) {
        if (m % p == 0) {
            f.push_back(p);
            while (m % p == 0) m /= p;
        }
    }
    if (m > 1) {
        if (!is_prime_u64(m)) return false;
        f.push_back(m);
    }
    for (uint64_t x = 2; x < t; x++) {
        bool ok = true;
        for (uint64_t p : f)
            if (hpow(x, (t - 1) / p, t) == 1) { ok = false; break; }
        if (ok) { *g = x; return true; }
    }
    return false;
}

// (M - 1) / 2 modulo m for M the product of `basis`, M odd: ((M mod 2m) - 1) / 2.
uint64_t half_mod(const std::vector<uint64_t> &basis, uint64_t m) {
    uint64_t m2 = 2 * m;
    uint64_t r = 1 % m2;
    for (uint64_t b : basis) r = hmul(r, b % m2, m2);
    return ((r + m2 - 1) % m2) / 2;
}

uint64_t prod_mod(const std::vector<uint64_t> &basis, uint64_t m, int skip = -1) {
    uint64_t r = 1 % m;
    for (size_t i = 0; i < basis.size(); i++)
        if ((int)i != skip) r = hmul(r, basis[i] % m, m);
    return r;
}

void build_mrc(MrcConst &M, const std::vector<uint64_t> &basis, const std::vector<uint64_t> &targets) {
    std::memset(&M, 0, sizeof(M));
    const int K = (int)basis.size();
    M.K = (uint32_t)K;
    M.ntarget = (uint32_t)targets.size();
    for (int b = 0; b < K; b++) {
        M.m[b] = basis[b];
        M.one_p[b] = shoup(1, basis[b]);
        for (int a = 0; a < b; a++) {
            M.inv[a][b] = hinv(basis[a] % basis[b], basis[b]);
            M.inv_p[a][b] = shoup(M.inv[a][b], basis[b]);
        }
    }
    // mixed-radix digits of (M - 1)/2 from its residues (m_b - 1)/2
    uint64_t d[FHE_MAXB];
    for (int b = 0; b < K; b++) {
        const uint64_t mb = basis[b];
        uint64_t v = (mb - 1) / 2;
        for (int a = 0; a < b; a++) {
            v = (v + mb - d[a] % mb) % mb;
            v = hmul(v, M.inv[a][b], mb);
        }
        d[b] = v;
        M.half_digit[b] = v;
    }
    for (size_t j = 0; j < targets.size(); j++) {
        const uint64_t p = targets[j];
        M.target[j] = p;
        M.tgt_one_p[j] = shoup(1, p);
        for (int b = 0; b < K; b++) {
            M.m_mod_t[b][j] = basis[b] % p;
            M.m_mod_t_p[b][j] = shoup(M.m_mod_t[b][j], p);
        }
        M.M_mod_t[j] = prod_mod(basis, p);
    }
}

// ------------------------------------------------------------------ events --

struct EvPair {
    hipEvent_t a, b;
};

}  // namespace

struct fhe_ctx {
    int device = 0;
    uint32_t n = 0, L = 0, k = 0, kp = 0, K = 0, encoding = 0;
    uint64_t t = 0;
    std::vector<uint64_t> primes;  // Q then P
    // slot encoding (host)
    std::vector<uint64_t> enc_tw, enc_itw;
    uint64_t t_ninv = 0;
    // device allocations
    void *d_pc = nullptr, *d_tw = nullptr, *d_itw = nullptr, *d_cc = nullptr;
    void *d_mrc_q = nullptr, *d_mrc_p = nullptr, *d_counters = nullptr;
    DevCtx dev{};
    size_t batch_limit = 0, default_limit = 0;
    // fused product kernel (k_mul_tensor / k_square_tensor) from this many
    // (item, limb) workgroups per launch on; fewer take the unfused kernels
    // (index 0: products of two ciphertexts, 1: squarings)
    size_t fused_min_rows[2] = {128, 0};
    bool validate = false;
    bool timing = false;
    std::vector<EvPair> pending[KK_COUNT];
    std::vector<hipEvent_t> free_events;
    double total_ms[KK_COUNT] = {};
    uint64_t launches[KK_COUNT] = {};
    // own stream (default priority) and fork/join events for fhe_mul_relin_multi,
    // and the graphs of fhe_square_chain; created on first use
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // A graph holds the addresses, the chunking and the fused/unfused choice
    // of the launches it recorded: its key is all of them, and the setters of
    // the launch shape drop every graph.  `done` is recorded after each replay
    // so a graph is destroyed only once its last replay has finished.
    struct ChainGraph {
        const void *rlk, *x, *ws;
        size_t count, ws_bytes, batch_limit, fused_min_rows;
        uint32_t depth;
        hipGraph_t g;
        hipGraphExec_t ge;
        hipEvent_t done;
    };
    std::vector<ChainGraph> graphs;
    // operand tables of the base conversions on the matrix cores (bases of at
    // most 8 primes each side, every prime at least 2^20), or null
    void *d_mx = nullptr;
    // operand tables of the matrix-core first transform pass (fhe_ntt_pass0),
    // built on first use
    void *d_p0w = nullptr;
    // persistent key switching of fhe_mul_relin_multi when this context leads
    // the call: mode (1 on where it applies, 0 off) and the queue counter
    int multi_persistent = 0;
    void *d_persist = nullptr;
    // device address of the static workspace of fhe_mul_relin_static on this
    // context's device (shared by every context on the device)
    void *scratch = nullptr;
    // pinned staging of fhe_weighted_sum's weights; the event marks the end of
    // the last copy out of it
    int32_t *wpin = nullptr;
    size_t wpin_cap = 0;
    hipEvent_t wpin_ev = nullptr;
};

namespace {

// Most squaring-chain graphs a context keeps (each holds its buffers' addresses).
constexpr size_t kMaxGraphs = 16;
// Most parts of one persistent key-switching launch.
constexpr size_t kMaxPersistParts = kRelinQueueParts;

const char *kKernelNames[KK_COUNT] = {"lift_q2p",   "square_tensor", "scale_round", "relin_fused",
                                      "ntt_rows",   "elementwise",   "bridge",      "misc",
                                      "mul_tensor", "fwd_ext",       "tensor_intt", "pass0_valu",
                                      "pass0_mfma"};

hipEvent_t take_event(fhe_ctx *c) {
    if (!c->free_events.empty()) {
        hipEvent_t e = c->free_events.back();
        c->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through f(), bracketed by events when timing is enabled.
template <typename F>
fhe_status run(fhe_ctx *c, int kind, hipStream_t s, F &&f) {
    EvPair ev{nullptr, nullptr};
    if (c->timing) {
        ev.a = take_event(c);
        ev.b = take_event(c);
        if (ev.a) hipEventRecord(ev.a, s);
    }
    hipError_t e = f();
    if (c->timing) {
        if (ev.b) hipEventRecord(ev.b, s);
        if (ev.a && ev.b) c->pending[kind].push_back(ev);
        c->launches[kind] += 1;
    }
    return e == hipSuccess ? FHE_OK : FHE_EDEVICE;
}

#define FHE_TRY(expr)                         \
    do {                                      \
        fhe_status _st = (expr);              \
        if (_st != FHE_OK) return _st;        \
    } while (0)

#define FHE_HIP(expr)                                      \
    do {                                                   \
        if ((expr) != hipSuccess) return FHE_EDEVICE;      \
    } while (0)

size_t ct_words(const fhe_ctx *c) { return 2 * (size_t)c->k * c->n; }

// Workspace words per product: E (extended inputs), Dt (tensor), C2.
size_t item_words_mul(const fhe_ctx *c, bool square) {
    const size_t npoly = square ? 2 : 4;
    return ((npoly + 3) * c->K + c->k) * c->n;
}

size_t bridge_group(const fhe_ctx *c) {
    size_t g = c->batch_limit / c->t;
    return g ? g : 1;
}

// Inputs per group of the power-basis bridge: its largest product level has
// hmax products per input (hmax the largest power of two below t - 1).
size_t powers_group(const fhe_ctx *c) {
    size_t hmax = 1;
    while (hmax * 2 < c->t - 1) hmax *= 2;
    size_t g = c->batch_limit / hmax;
    return g ? g : 1;
}

bool overlaps(const void *a, const void *b, size_t bytes) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

bool overlaps2(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bbytes && y < x + abytes;
}

fhe_status check_canonical(fhe_ctx *c, const uint64_t *a, size_t nrows, int kmod, int off,
                           hipStream_t s) {
    if (!c->validate || nrows == 0) return FHE_OK;
    unsigned int *flag = (unsigned int *)c->d_counters + 2;
    FHE_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned int), s));
    FHE_HIP(launch_validate(c->dev, a, nrows, kmod, off, flag, s));
    unsigned int h = 0;
    FHE_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
    FHE_HIP(hipStreamSynchronize(s));
    return h ? FHE_ENONCANON : FHE_OK;
}

// The fused product kernel runs one workgroup per (item, limb) doing seven
// transforms in a row; with few such workgroups the unfused kernels (one
// workgroup per transform, seven times as many) finish sooner (measured at
// n = 16384: one item faster unfused, sixteen faster fused): the default
// threshold is 128 workgroups for products, and fhe_autotune_mul_relin moves
// it (and the chunk size) per context from timings.

// The product pipeline on `count` items with workspace for min(count, limit).

fhe_status mul_relin_impl(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                          uint64_t *out, size_t count, void *ws, hipStream_t s, bool relin = true) {
    const bool square = (a == b);
    const int npoly = square ? 2 : 4;
    const size_t n = c->n, K = c->K, k = c->k, ctw = ct_words(c);
    const size_t chunk = c->batch_limit;
    for (size_t off = 0; off < count; off += chunk) {
        const size_t items = count - off < chunk ? count - off : chunk;
        const uint64_t *ai = a + off * ctw;
        const uint64_t *bi = b + off * ctw;
        uint64_t *oi = out + off * ctw;
        uint64_t *E = (uint64_t *)ws;
        uint64_t *Dt = E + items * npoly * K * n;
        uint64_t *C2 = Dt + items * 3 * K * n;
        const DevCtx &d = c->dev;
        FHE_TRY(run(c, KK_LIFT, s, [&] { return launch_lift(d, ai, bi, E, npoly, items, s); }));
        if (items * K >= c->fused_min_rows[square ? 1 : 0]) {
            if (square)
                FHE_TRY(run(c, KK_SQUARE_TENSOR, s, [&] { return launch_square_tensor(d, ai, E, Dt, items, s); }));
            else
                FHE_TRY(run(c, KK_MUL_TENSOR, s, [&] { return launch_mul_tensor(d, ai, bi, E, Dt, items, s); }));
        } else {  // few items: one workgroup per transform keeps more of the chip busy
            FHE_TRY(run(c, KK_FWD_EXT, s, [&] { return launch_fwd_ext(d, ai, bi, E, npoly, items, s); }));
            FHE_TRY(run(c, KK_TENSOR_INTT, s, [&] { return launch_tensor_intt(d, E, Dt, square, items, s); }));
        }
        FHE_TRY(run(c, KK_SCALE, s, [&] { return launch_scale(d, Dt, oi, C2, items, s); }));
        if (relin)
            FHE_TRY(run(c, KK_RELIN_FUSED, s, [&] { return launch_relin_fused(d, C2, rlk, oi, items, s); }));
    }
    return FHE_OK;
}

// Where mul_relin_impl leaves C2 of a batch that fits one chunk.
uint64_t *c2_of_single_chunk(const fhe_ctx *c, void *ws, size_t count, bool square) {
    const size_t n = c->n, K = c->K, npoly = square ? 2 : 4;
    return (uint64_t *)ws + count * npoly * K * n + count * 3 * K * n;
}

// Products of `count` items from transformed operands (k_lift + k_fwd_ext
// layout [.][2][K][n]): item z multiplies input z mod na of Ahat by entry z of
// Bhat; chunks of the batch cap, workspace as for products.
fhe_status mul_relin_pre2_impl(fhe_ctx *c, const uint64_t *rlk, const uint64_t *Ahat, size_t na,
                               const uint64_t *Bhat, uint64_t *out, size_t count, void *ws, hipStream_t s) {
    const size_t n = c->n, K = c->K, ctw = ct_words(c);
    const size_t chunk = c->batch_limit;
    const DevCtx &d = c->dev;
    for (size_t off = 0; off < count; off += chunk) {
        const size_t items = count - off < chunk ? count - off : chunk;
        uint64_t *oi = out + off * ctw;
        uint64_t *Dt = (uint64_t *)ws;
        uint64_t *C2 = Dt + items * 3 * K * n;
        FHE_TRY(run(c, KK_MUL_TENSOR, s,
                    [&] { return launch_mul_tensor_pre2(d, Ahat, (int)na, off, Bhat, Dt, items, s); }));
        FHE_TRY(run(c, KK_SCALE, s, [&] { return launch_scale(d, Dt, oi, C2, items, s); }));
        FHE_TRY(run(c, KK_RELIN_FUSED, s, [&] { return launch_relin_fused(d, C2, rlk, oi, items, s); }));
    }
    return FHE_OK;
}

fhe_status alloc_copy(void **dst, const void *src, size_t bytes) {
    if (hipMalloc(dst, bytes) != hipSuccess) {
        *dst = nullptr;
        return FHE_ENOMEM;
    }
    if (hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return FHE_EDEVICE;
    return FHE_OK;
}

// Destroys graph i of the squaring-chain cache after its last replay ended.
void drop_graph(fhe_ctx *c, size_t i) {
    fhe_ctx::ChainGraph &cg = c->graphs[i];
    if (cg.done) {
        (void)hipEventSynchronize(cg.done);
        (void)hipEventDestroy(cg.done);
    }
    (void)hipGraphExecDestroy(cg.ge);
    (void)hipGraphDestroy(cg.g);
    c->graphs.erase(c->graphs.begin() + (long)i);
}

void drop_graphs(fhe_ctx *c) {
    while (!c->graphs.empty()) drop_graph(c, c->graphs.size() - 1);
}

void release(fhe_ctx *c) {
    drop_graphs(c);
    if (c->wpin_ev) {
        (void)hipEventSynchronize(c->wpin_ev);
        (void)hipEventDestroy(c->wpin_ev);
    }
    if (c->wpin) hipHostFree(c->wpin);
    if (c->fork_ev) hipEventDestroy(c->fork_ev);
    if (c->join_ev) hipEventDestroy(c->join_ev);
    if (c->aux) hipStreamDestroy(c->aux);
    void *ptrs[] = {c->d_pc,       c->d_tw,  c->d_itw, c->d_cc,      c->d_mrc_q, c->d_mrc_p,
                    c->d_counters, c->d_p0w, c->d_mx,  c->d_persist};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (int i = 0; i < KK_COUNT; i++)
        for (auto &e : c->pending[i]) {
            hipEventDestroy(e.a);
            hipEventDestroy(e.b);
        }
    for (auto e : c->free_events) hipEventDestroy(e);
}

// Host slot transforms modulo t (merged-psi Cooley-Tukey / Gentleman-Sande).
void host_fwd_mod_t(std::vector<uint64_t> &a, const std::vector<uint64_t> &tw, uint64_t t) {
    const size_t n = a.size();
    size_t len = n;
    for (size_t m = 1; m < n; m <<= 1) {
        len >>= 1;
        for (size_t i = 0; i < m; i++) {
            const size_t j1 = 2 * i * len;
            const uint64_t S = tw[m + i];
            for (size_t j = j1; j < j1 + len; j++) {
                const uint64_t U = a[j], V = hmul(a[j + len], S, t);
                a[j] = (U + V) % t;
                a[j + len] = (U + t - V) % t;
            }
        }
    }
}

void host_inv_mod_t(std::vector<uint64_t> &a, const std::vector<uint64_t> &itw, uint64_t t,
                    uint64_t ninv) {
    const size_t n = a.size();
    size_t len = 1;
    for (size_t m = n; m > 1; m >>= 1) {
        size_t j1 = 0;
        const size_t h = m >> 1;
        for (size_t i = 0; i < h; i++) {
            const uint64_t S = itw[h + i];
            for (size_t j = j1; j < j1 + len; j++) {
                const uint64_t U = a[j], V = a[j + len];
                a[j] = (U + V) % t;
                a[j + len] = hmul((U + t - V) % t, S, t);
            }
            j1 += 2 * len;
        }
        len <<= 1;
    }
    for (auto &v : a) v = hmul(v, ninv, t);
}

}  // namespace

// =================================================================== ABI ====

extern "C" {

const char *fhe_status_str(fhe_status s) {
    switch (s) {
        case FHE_OK: return "ok";
        case FHE_EINVAL: return "invalid argument";
        case FHE_EPARAM: return "parameter set rejected";
        case FHE_ENOMEM: return "device allocation failed";
        case FHE_EDEVICE: return "HIP error";
        case FHE_ESHAPE: return "shape mismatch";
        case FHE_ENONCANON: return "non-canonical input word";
        case FHE_EUNSUPPORTED: return "operation not supported for these parameters";
        case FHE_EWORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

// Balanced base-256 digits (each in [-128, 127]) of x < 2^62 (any x with
// x + 0x8080808080808080 < 2^64).
void balanced_digits(uint64_t x, int8_t d[8]) {
    const uint64_t B = 0x8080808080808080ull;
    const uint64_t y = (x + B) ^ B;
    for (int u = 0; u < 8; u++) d[u] = (int8_t)(uint8_t)(y >> (8 * u));
}

// Operand table of one matrix-core conversion (layout of ConvMx): weights
// W[t][s] modulo m[t] for targets t < nt and sources s < ns (zero elsewhere).
void mx_table(int32_t (*tab)[64][4], const uint64_t (*W)[FHE_MX_MAXB], const uint64_t *m, int nt, int ns) {
    for (int mm = 0; mm < 4; mm++)
        for (int lane = 0; lane < 64; lane++) {
            const int row = lane % 16, t = 4 * (mm / 2) + row / 4, v = 4 * (mm % 2) + row % 4, g = lane / 16;
            uint8_t bytes[16];
            for (int b = 0; b < 16; b++) {
                const int src = g + 4 * (b / 8), u = b % 8;
                int8_t val = 0;
                if (t < nt && src < ns) {
                    int8_t d[8];
                    balanced_digits(hmul(W[t][src], (1ull << (8 * u)) % m[t], m[t]), d);
                    val = d[v];
                }
                bytes[b] = (uint8_t)val;
            }
            std::memcpy(tab[mm][lane], bytes, 16);
        }
}

// The tables of the matrix-core conversions from those of the vector ALU ones.
void build_conv_mx(const ConvConst &cc, ConvMx &mx) {
    const int k = (int)cc.k, kp = (int)cc.kp;
    const u128 bias = (u128)FHE_MX_BIAS * 0x0101010101010101ull;  // FHE_MX_BIAS sum_v 256^v
    auto neg_bias = [&](uint64_t m) { return (m - (uint64_t)(bias % m)) % m; };
    uint64_t W[FHE_MX_MAXB][FHE_MX_MAXB] = {};
    for (int j = 0; j < kp; j++)
        for (int i = 0; i < k; i++) W[j][i] = cc.lift_m[j][i];
    mx_table(mx.a_lift, W, cc.p, kp, k);
    for (int j = 0; j < kp; j++)
        for (int i = 0; i < k; i++) W[j][i] = hmul(cc.scale_m[j][i], cc.phinv[j], cc.p[j]);
    mx_table(mx.a_scale, W, cc.p, kp, k);
    std::memset(W, 0, sizeof(W));
    for (int j = 0; j < kp; j++) W[j][j] = hmul(cc.scale_m[j][k], cc.phinv[j], cc.p[j]);
    mx_table(mx.a_sdp, W, cc.p, kp, kp);
    for (int i = 0; i < k; i++)
        for (int j = 0; j < kp; j++) W[i][j] = cc.p2q_m[i][j];
    mx_table(mx.a_p2q, W, cc.q, k, kp);
    for (int j = 0; j < kp; j++) {
        const uint64_t pj = cc.p[j];
        mx.e_lift[j] = neg_bias(pj);
        mx.e_scale[j] = (hmul(cc.scale_m[j][k + 2], cc.phinv[j], pj) + neg_bias(pj)) % pj;
        mx.s_v[j] = hmul(cc.scale_m[j][k + 1], cc.phinv[j], pj);
        mx.l_beta[j] = cc.lift_m[j][k];
    }
    for (int i = 0; i < k; i++) {
        mx.e_p2q[i] = neg_bias(cc.q[i]);
        mx.p_beta[i] = cc.p2q_m[i][kp];
    }
}

fhe_status fhe_ctx_create(const fhe_params *p, int hip_device, fhe_ctx **out) {
    if (!p || !out || !p->q) return FHE_EINVAL;
    const uint32_t n = p->n, k = p->k;
    if (n < 16 || n > 16384 || (n & (n - 1))) return FHE_EPARAM;
    if (k < 1 || k > (uint32_t)FHE_MAXK) return FHE_EPARAM;
    if (p->t < 2 || p->t >= (1ull << 62)) return FHE_EPARAM;
    if (p->encoding != FHE_ENC_SLOTS && p->encoding != FHE_ENC_COEFF) return FHE_EPARAM;
    std::vector<uint64_t> qs(p->q, p->q + k);
    double log2q = 0;
    for (uint32_t i = 0; i < k; i++) {
        const uint64_t qi = qs[i];
        if (qi < 3 || qi >= (1ull << 61) || qi % (2ull * n) != 1 || !is_prime_u64(qi)) return FHE_EPARAM;
        for (uint32_t j = 0; j < i; j++)
            if (qs[j] == qi) return FHE_EPARAM;
        if (hgcd(p->t, qi) != 1) return FHE_EPARAM;
        log2q += std::log2((double)qi);
    }
    if (p->encoding == FHE_ENC_SLOTS && (!is_prime_u64(p->t) || p->t % (2ull * n) != 1)) return FHE_EPARAM;

    // Auxiliary primes: the largest primes below a cap that are 1 mod 2n and
    // not in Q, until P > 4 t n q (the scaled tensor is then unique modulo P).
    // The cap is 2^58 when that takes no more primes than the cap 2^61: primes
    // below 2^64 / (4 (L + 1)) let the transforms skip conditional subtractions.
    const double need = std::log2((double)p->t) + std::log2((double)n) + log2q + 2.0;
    const uint64_t step = 2ull * n;
    auto aux_primes = [&](uint64_t cap, std::vector<uint64_t> &ps) {
        double have = 0;
        uint64_t cand = (cap - 2) / step * step + 1;
        while (have < need) {
            if (ps.size() >= (size_t)FHE_MAXKP || cand < (cap >> 2)) return false;
            bool inq = false;
            for (uint64_t qi : qs) inq |= (qi == cand);
            if (!inq && is_prime_u64(cand) && hgcd(p->t, cand) == 1) {
                ps.push_back(cand);
                have += std::log2((double)cand);
            }
            cand -= step;
        }
        return true;
    };
    std::vector<uint64_t> ps, ps_small;
    if (!aux_primes(1ull << 61, ps)) return FHE_EPARAM;
    if (aux_primes(1ull << 58, ps_small) && ps_small.size() <= ps.size()) ps.swap(ps_small);

    fhe_ctx *c = new fhe_ctx();
    c->n = n;
    c->k = k;
    c->kp = (uint32_t)ps.size();
    c->K = c->k + c->kp;
    c->t = p->t;
    c->encoding = p->encoding;
    c->device = hip_device;
    for (int L = 0; L < 32; L++)
        if ((1u << L) == n) c->L = L;
    c->primes = qs;
    c->primes.insert(c->primes.end(), ps.begin(), ps.end());
    const char *v = std::getenv("FHE_VALIDATE");
    c->validate = v && v[0] == '1';

    // slot transform tables (host)
    if (c->encoding == FHE_ENC_SLOTS) {
        uint64_t g = 0;
        if (!primitive_root(c->t, &g)) {
            delete c;
            return FHE_EPARAM;
        }
        const uint64_t psi = hpow(g, (c->t - 1) / (2 * (uint64_t)n), c->t);
        const uint64_t ipsi = hinv(psi, c->t);
        c->enc_tw.resize(n);
        c->enc_itw.resize(n);
        for (uint32_t i = 0; i < n; i++) {
            c->enc_tw[i] = hpow(psi, bitrev(i, c->L), c->t);
            c->enc_itw[i] = hpow(ipsi, bitrev(i, c->L), c->t);
        }
        c->t_ninv = hinv(n % c->t, c->t);
    }

    // ---- device tables ----
    std::vector<PrimeConst> pc(c->K);
    std::vector<Tw> tw((size_t)c->K * n), itw((size_t)c->K * n);
    for (uint32_t l = 0; l < c->K; l++) {
        const uint64_t q = c->primes[l];
        PrimeConst &P = pc[l];
        std::memset(&P, 0, sizeof(P));
        P.q = q;
        P.qinv_neg = neg_inv64(q);
        P.one_p = shoup(1, q);
        P.ninv = hinv(n % q, q);
        P.ninv_p = shoup(P.ninv, q);
        P.ninvm = mont(P.ninv, q);
        P.ninvm_p = shoup(P.ninvm, q);
        P.r32 = (uint64_t)(((u128)1 << 32) % q);
        P.r32_p = shoup(P.r32, q);
        P.mx_neg_bias = (q - (uint64_t)(((u128)FHE_MX_BIAS * 0x0101010101010101ull) % q)) % q;
        P.off59 = ((1ull << 59) + q - 1) / q * q;
        P.off62 = ((1ull << 62) + q - 1) / q * q;
        const uint64_t psi = find_psi(q, n), ipsi = hinv(psi, q);
        std::vector<uint64_t> pw(n), ipw(n);
        pw[0] = 1;
        ipw[0] = 1;
        for (uint32_t i = 1; i < n; i++) {
            pw[i] = hmul(pw[i - 1], psi, q);
            ipw[i] = hmul(ipw[i - 1], ipsi, q);
        }
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t r = bitrev(i, c->L);
            tw[(size_t)l * n + i] = Tw{pw[r], shoup(pw[r], q)};
            itw[(size_t)l * n + i] = Tw{ipw[r], shoup(ipw[r], q)};
        }
    }

    ConvConst *cc = new ConvConst();
    std::memset(cc, 0, sizeof(ConvConst));
    cc->k = k;
    cc->kp = c->kp;
    cc->t = c->t;
    const uint64_t t = c->t;
    for (uint32_t i = 0; i < k; i++) {
        cc->q[i] = qs[i];
        cc->q_qinv[i] = neg_inv64(qs[i]);
        cc->q_one[i] = shoup(1, qs[i]);
    }
    for (uint32_t j = 0; j < c->kp; j++) {
        cc->p[j] = ps[j];
        cc->p_qinv[j] = neg_inv64(ps[j]);
        cc->p_one[j] = shoup(1, ps[j]);
    }
    const uint64_t q_mod_t = prod_mod(qs, t);
    for (uint32_t i = 0; i < k; i++) {
        const uint64_t qi = qs[i];
        const uint64_t qhinv = hinv(prod_mod(qs, qi, (int)i), qi);
        cc->qhinv[i] = qhinv;
        cc->qhinv_p[i] = shoup(qhinv, qi);
        cc->inv_q[i] = 1.0 / (double)qi;
        const uint64_t tq = t % qi;
        cc->tqhinv[i] = hmul(tq, qhinv, qi);
        cc->tqhinv_p[i] = shoup(cc->tqhinv[i], qi);
        const uint64_t hq = (qi - 1) / 2;  // (q - 1)/2 = -1/2 modulo q_i
        cc->hqhinv[i] = hmul(hq, qhinv, qi);
        cc->h_q[i] = hq;
        cc->t_q[i] = tq;
        cc->t_qs[i] = shoup(tq, qi);
        // Delta = floor(q/t) = (q - [q]_t)/t = -[q]_t t^-1 modulo q_i
        const uint64_t dq = hmul((qi - q_mod_t % qi) % qi, hinv(tq, qi), qi);
        cc->delta_q[i] = dq;
        cc->delta_qs[i] = shoup(dq, qi);
    }
    for (uint32_t j = 0; j < c->kp; j++) {
        const uint64_t pj = ps[j];
        const uint64_t qmod = prod_mod(qs, pj);
        const uint64_t qinv = hinv(qmod, pj);
        const uint64_t hp = half_mod(qs, pj);
        for (uint32_t i = 0; i < k; i++) {
            cc->lift_m[j][i] = mont(prod_mod(qs, pj, (int)i), pj);
            const uint64_t qiinv = hinv(qs[i] % pj, pj);
            cc->scale_m[j][i] = mont((pj - qiinv) % pj, pj);
        }
        cc->lift_m[j][k] = mont((pj - qmod) % pj, pj);
        cc->scale_m[j][k] = mont(hmul(t % pj, qinv, pj), pj);
        cc->scale_m[j][k + 1] = mont(1, pj);
        cc->scale_m[j][k + 2] = mont(hmul(hp, qinv, pj), pj);
        cc->h_p[j] = hp;
        cc->t_p[j] = t % pj;
        cc->t_ps[j] = shoup(t % pj, pj);
        cc->qinv_p[j] = qinv;
        cc->qinv_ps[j] = shoup(qinv, pj);
        const uint64_t phat = prod_mod(ps, pj, (int)j);
        cc->phinv[j] = hinv(phat, pj);
        cc->phinv_p[j] = shoup(cc->phinv[j], pj);
        cc->inv_p[j] = 1.0 / (double)pj;
    }
    for (uint32_t i = 0; i < k; i++) {
        for (uint32_t j = 0; j < c->kp; j++) cc->p2q_m[i][j] = mont(prod_mod(ps, qs[i], (int)j), qs[i]);
        const uint64_t pmod = prod_mod(ps, qs[i]);
        cc->p2q_m[i][c->kp] = mont((qs[i] - pmod) % qs[i], qs[i]);
    }
    // bounds of the multiply-accumulates (every operand canonical; overflow
    // counts at most the basis size)
    auto fits = [](u128 T, uint64_t m) { return (uint64_t)(T >> 64) <= 2 * m - 2; };
    cc->fast_lift = cc->fast_scale_p = cc->fast_p2q = 1;
    for (uint32_t j = 0; j < c->kp; j++) {
        const uint64_t pm = ps[j] - 1;
        u128 T = 0;
        for (uint32_t i = 0; i < k; i++) T += (u128)(qs[i] - 1) * pm;
        const u128 Tl = T + (u128)k * pm;
        const u128 Ts = T + (u128)pm * pm + (u128)k * pm + pm;
        if (!fits(Tl, ps[j])) cc->fast_lift = 0;
        if (!fits(Ts, ps[j])) cc->fast_scale_p = 0;
    }
    for (uint32_t i = 0; i < k; i++) {
        const uint64_t qm = qs[i] - 1;
        u128 T = 0;
        for (uint32_t j = 0; j < c->kp; j++) T += (u128)(ps[j] - 1) * qm;
        T += (u128)c->kp * qm;
        if (!fits(T, qs[i])) cc->fast_p2q = 0;
    }
    cc->h_t = half_mod(qs, t);
    cc->qinv_t = hinv(q_mod_t, t);
    cc->qinv_ts = shoup(cc->qinv_t, t);
    cc->t_one_p = shoup(1, t);

    MrcConst *mq = new MrcConst(), *mp = new MrcConst();
    std::vector<uint64_t> tq_targets(ps);
    tq_targets.push_back(t);
    build_mrc(*mq, qs, tq_targets);
    build_mrc(*mp, ps, qs);

    fhe_status st = FHE_OK;
    if (hipSetDevice(hip_device) != hipSuccess) st = FHE_EDEVICE;
    if (st == FHE_OK) st = scratch_address(hip_device, &c->scratch);
    if (st == FHE_OK) st = alloc_copy(&c->d_pc, pc.data(), pc.size() * sizeof(PrimeConst));
    if (st == FHE_OK) st = alloc_copy(&c->d_tw, tw.data(), tw.size() * sizeof(Tw));
    if (st == FHE_OK) st = alloc_copy(&c->d_itw, itw.data(), itw.size() * sizeof(Tw));
    if (st == FHE_OK) st = alloc_copy(&c->d_cc, cc, sizeof(ConvConst));
    if (st == FHE_OK) st = alloc_copy(&c->d_mrc_q, mq, sizeof(MrcConst));
    if (st == FHE_OK) st = alloc_copy(&c->d_mrc_p, mp, sizeof(MrcConst));
    // matrix-core conversions: at most 8 primes each side; primes of at least
    // 2^20 keep the high word of every reduced sum below 2m - 1
    bool mx_ok = k <= (uint32_t)FHE_MX_MAXB && c->kp <= (uint32_t)FHE_MX_MAXB;
    for (uint64_t m : c->primes) mx_ok = mx_ok && m >= (1ull << 20);
    if (st == FHE_OK && mx_ok) {
        ConvMx *mx = new ConvMx();
        std::memset(mx, 0, sizeof(ConvMx));
        build_conv_mx(*cc, *mx);
        st = alloc_copy(&c->d_mx, mx, sizeof(ConvMx));
        delete mx;
    }
    if (st == FHE_OK) {
        uint64_t zeros[4] = {0, 0, 0, 0};
        st = alloc_copy(&c->d_counters, zeros, sizeof(zeros));
    }
    delete cc;
    delete mq;
    delete mp;
    if (st != FHE_OK) {
        release(c);
        delete c;
        return st;
    }
    DevCtx &d = c->dev;
    d.n = (int)n;
    d.L = (int)c->L;
    d.k = (int)k;
    d.kp = (int)c->kp;
    d.K = (int)c->K;
    d.t = c->t;
    d.pc = (const PrimeConst *)c->d_pc;
    d.tw = (const Tw *)c->d_tw;
    d.itw = (const Tw *)c->d_itw;
    d.cc = (const ConvConst *)c->d_cc;
    d.mrc_q = (const MrcConst *)c->d_mrc_q;
    d.mrc_p = (const MrcConst *)c->d_mrc_p;
    d.fallback = (unsigned long long *)c->d_counters;
    d.mx = (const ConvMx *)c->d_mx;
    uint64_t qmin = c->primes[0], qmax = c->primes[0];
    for (uint32_t i = 1; i < k; i++) {
        qmin = c->primes[i] < qmin ? c->primes[i] : qmin;
        qmax = c->primes[i] > qmax ? c->primes[i] : qmax;
    }
    d.digit_raw = (u128)qmax < (u128)qmin * 4;
    d.lazy_q = d.lazy_all = 1;
    d.lazy_limbs = 0;
    for (uint32_t i = 0; i < c->K; i++) {
        if (c->primes[i] < UINT64_MAX / (4ull * (c->L + 1))) {
            d.lazy_limbs |= 1ull << i;
        } else {
            d.lazy_all = 0;
            if (i < k) d.lazy_q = 0;
        }
    }
    // lazy key switching also sums up to 16 products below 2q unreduced
    for (uint32_t i = 0; i < k; i++)
        if (c->primes[i] >= (1ull << 59)) d.lazy_q = 0;
    // default chunk: about 8 GiB of product workspace
    size_t per = item_words_mul(c, false) * 8;
    c->default_limit = ((size_t)8 << 30) / per;
    if (c->default_limit < 1) c->default_limit = 1;
    if (c->default_limit > 65535) c->default_limit = 65535;
    c->batch_limit = c->default_limit;
    *out = c;
    return FHE_OK;
}

void fhe_ctx_destroy(fhe_ctx *c) {
    if (!c) return;
    hipDeviceSynchronize();
    release(c);
    delete c;
}

size_t fhe_ct_words(const fhe_ctx *c) { return c ? ct_words(c) : 0; }
size_t fhe_pk_words(const fhe_ctx *c) { return c ? ct_words(c) : 0; }
size_t fhe_rlk_words(const fhe_ctx *c) { return c ? 2 * (size_t)c->k * c->k * c->n : 0; }
uint32_t fhe_aux_primes(const fhe_ctx *c) { return c ? c->kp : 0; }

size_t fhe_workspace_bytes(const fhe_ctx *c, int op, size_t count) {
    if (!c) return 0;
    const size_t n = c->n, k = c->k;
    const size_t lim = c->batch_limit;
    switch (op) {
        case FHE_OP_MUL_RELIN:
        case FHE_OP_SQUARE_RELIN: {
            const size_t items = count < lim ? count : lim;
            return items * item_words_mul(c, op == FHE_OP_SQUARE_RELIN) * 8;
        }
        case FHE_OP_BRIDGE: {
            size_t g = bridge_group(c);
            if (count < g) g = count;
            const size_t chains = g * c->t;
            return (chains * ct_words(c) + chains * item_words_mul(c, true)) * 8;
        }
        case FHE_OP_KEYGEN:
            return (6 * k * n) * 8 + n + 4 * n + k * n * 8 + 4 * n + 64;
        case FHE_OP_ENCRYPT:
            return (2 * k * n + count * k * n + count * 2 * k * n + count * n) * 8 + count * n +
                   count * 2 * n * 4 + 256;
        case FHE_OP_DECRYPT:
            return (k * n + 2 * count * k * n + count * n) * 8 + n + 256;
        case FHE_OP_RLK_IMPORT:
            return 0;
        case FHE_OP_WEIGHTED_SUM:
            // padded int32 rows (at most 8 slots per weight), or the int8 operand
            // table of the matrix cores: ceil(nout/16) ceil(nin/64) KiB
            // <= 81 count + 1024 bytes for nout, nin <= count
            return 81 * count + 1024;
        case FHE_OP_GATE:
            return 2 * count * ct_words(c) * 8 + fhe_workspace_bytes(c, FHE_OP_MUL_RELIN, count);
        case FHE_OP_COMPARE:
            return 6 * count * ct_words(c) * 8 + fhe_workspace_bytes(c, FHE_OP_MUL_RELIN, count);
        case FHE_OP_ARGMAX:
            return 2 * count * ct_words(c) * 8 + fhe_workspace_bytes(c, FHE_OP_COMPARE, count);
        case FHE_OP_BRIDGE_POWERS: {
            if (c->t < 3 || c->t > 257) return 0;
            const size_t e = c->t - 1;
            size_t hmax = 1;
            while (hmax * 2 < e) hmax *= 2;
            size_t g = powers_group(c);
            if (count < g) g = count;
            const size_t wbytes = ((20 * weighted_sum_row_stride(c->t) * 4 + 255) / 256) * 256;
            return (e * ct_words(c) + hmax * 2 * (size_t)c->K * c->n) * g * 8 + wbytes +
                   fhe_workspace_bytes(c, FHE_OP_MUL_RELIN, hmax * g);
        }
        case FHE_OP_MOD_TO_INT: {
            const size_t a = fhe_workspace_bytes(c, FHE_OP_BRIDGE, count);
            const size_t b = 7 * count * ct_words(c) * 8 + fhe_workspace_bytes(c, FHE_OP_MUL_RELIN, count);
            return a > b ? a : b;
        }
    }
    return 0;
}

fhe_status fhe_set_fused_threshold(fhe_ctx *c, int square, size_t min_rows) {
    if (!c) return FHE_EINVAL;
    c->fused_min_rows[square ? 1 : 0] = min_rows;
    drop_graphs(c);
    return FHE_OK;
}

fhe_status fhe_set_conv_method(fhe_ctx *c, int method) {
    if (!c || (method != 0 && method != 1)) return FHE_EINVAL;
    if (method == 1 && !c->d_mx) return FHE_EUNSUPPORTED;
    c->dev.mx = method ? (const ConvMx *)c->d_mx : nullptr;
    drop_graphs(c);
    return FHE_OK;
}

int fhe_conv_method(const fhe_ctx *c) { return c && c->dev.mx ? 1 : 0; }

fhe_status fhe_set_batch_limit(fhe_ctx *c, size_t max_items) {
    if (!c) return FHE_EINVAL;
    c->batch_limit = max_items ? (max_items > 65535 ? 65535 : max_items) : c->default_limit;
    drop_graphs(c);
    return FHE_OK;
}

// ------------------------------------------------------------------ keys ----

fhe_status fhe_keygen(fhe_ctx *c, const int8_t *s, const uint64_t *pk_a, const int32_t *pk_e,
                      const uint64_t *rlk_a, const int32_t *rlk_e, uint64_t *pk_dev, uint64_t *rlk_dev,
                      void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c || !s || !pk_a || !pk_e || !rlk_a || !rlk_e || !pk_dev || !rlk_dev || !ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_KEYGEN, 1)) return FHE_EWORKSPACE;
    const size_t n = c->n, k = c->k, kn = k * n;
    uint64_t *S = (uint64_t *)ws, *A = S + kn, *prod = A + kn, *Er = prod + kn, *S2 = Er + kn,
             *tmp = S2 + kn;
    int8_t *s_dev = (int8_t *)(tmp + kn);
    int32_t *e_dev = (int32_t *)(s_dev + ((n + 63) & ~(size_t)63));
    const DevCtx &d = c->dev;
    FHE_HIP(hipMemcpyAsync(s_dev, s, n, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_small_to_rns(d, s_dev, 1, S, 1, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, S, k, k, 0, NTT_FWD, st); }));
    // pk0 = -(a s + e), pk1 = a
    FHE_HIP(hipMemcpyAsync(A, pk_a, kn * 8, hipMemcpyHostToDevice, st));
    FHE_HIP(hipMemcpyAsync(pk_dev + kn, pk_a, kn * 8, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, A, k, k, 0, NTT_FWD, st); }));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_pointwise_mont(d, A, S, prod, k, 0, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, prod, k, k, 0, NTT_INV_MONT, st); }));
    FHE_HIP(hipMemcpyAsync(e_dev, pk_e, n * 4, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_small_to_rns(d, e_dev, 0, Er, 1, st); }));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_key_b(d, prod, Er, nullptr, -1, pk_dev, st); }));
    // s^2 (coefficient form)
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_pointwise_mont(d, S, S, S2, k, 0, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, S2, k, k, 0, NTT_INV_MONT, st); }));
    // rlk_i = (-(a_i s + e_i) + eps_i s^2, a_i), built in coefficient form in rlk_dev
    for (size_t i = 0; i < k; i++) {
        uint64_t *b_i = rlk_dev + (i * 2 + 0) * kn;
        uint64_t *a_i = rlk_dev + (i * 2 + 1) * kn;
        FHE_HIP(hipMemcpyAsync(A, rlk_a + i * kn, kn * 8, hipMemcpyHostToDevice, st));
        FHE_HIP(hipMemcpyAsync(a_i, rlk_a + i * kn, kn * 8, hipMemcpyHostToDevice, st));
        FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, A, k, k, 0, NTT_FWD, st); }));
        FHE_TRY(run(c, KK_MISC, st, [&] { return launch_pointwise_mont(d, A, S, prod, k, 0, st); }));
        FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, prod, k, k, 0, NTT_INV_MONT, st); }));
        FHE_HIP(hipMemcpyAsync(e_dev, rlk_e + i * n, n * 4, hipMemcpyHostToDevice, st));
        FHE_TRY(run(c, KK_MISC, st, [&] { return launch_small_to_rns(d, e_dev, 0, Er, 1, st); }));
        FHE_TRY(run(c, KK_MISC, st, [&] { return launch_key_b(d, prod, Er, S2, (int)i, b_i, st); }));
        // the staging buffers are reused next iteration: wait for this one
        FHE_HIP(hipStreamSynchronize(st));
    }
    FHE_TRY(run(c, KK_NTT_ROWS, st,
                [&] { return launch_ntt_rows(d, rlk_dev, 2 * k * k, k, 0, NTT_FWD_NINVM, st); }));
    FHE_HIP(hipStreamSynchronize(st));
    return FHE_OK;
}

fhe_status fhe_rlk_import(fhe_ctx *c, const uint64_t *rlk_coeff, uint64_t *rlk_dev, void *ws,
                          size_t ws_bytes, hipStream_t st) {
    (void)ws;
    (void)ws_bytes;
    if (!c || !rlk_coeff || !rlk_dev) return FHE_EINVAL;
    const size_t words = fhe_rlk_words(c);
    if (rlk_coeff != rlk_dev) {
        if (overlaps(rlk_coeff, rlk_dev, words * 8)) return FHE_EINVAL;
        FHE_HIP(hipMemcpyAsync(rlk_dev, rlk_coeff, words * 8, hipMemcpyDeviceToDevice, st));
    }
    FHE_TRY(check_canonical(c, rlk_dev, 2 * (size_t)c->k * c->k, c->k, 0, st));
    return run(c, KK_NTT_ROWS, st, [&] {
        return launch_ntt_rows(c->dev, rlk_dev, 2 * (size_t)c->k * c->k, c->k, 0, NTT_FWD_NINVM, st);
    });
}

// -------------------------------------------------------------- encoding ----

fhe_status fhe_encode(const fhe_ctx *c, const uint64_t *vals, uint64_t *pt) {
    if (!c || !vals || !pt) return FHE_EINVAL;
    const size_t n = c->n;
    if (c->encoding == FHE_ENC_COEFF) {
        for (size_t i = 0; i < n; i++) pt[i] = vals[i] % c->t;
        return FHE_OK;
    }
    std::vector<uint64_t> a(n);
    for (size_t j = 0; j < n; j++) a[bitrev((uint32_t)j, c->L)] = vals[j] % c->t;
    host_inv_mod_t(a, c->enc_itw, c->t, c->t_ninv);
    std::memcpy(pt, a.data(), n * 8);
    return FHE_OK;
}

fhe_status fhe_decode(const fhe_ctx *c, const uint64_t *pt, uint64_t *vals) {
    if (!c || !vals || !pt) return FHE_EINVAL;
    const size_t n = c->n;
    if (c->encoding == FHE_ENC_COEFF) {
        for (size_t i = 0; i < n; i++) vals[i] = pt[i] % c->t;
        return FHE_OK;
    }
    std::vector<uint64_t> a(pt, pt + n);
    for (auto &v : a) v %= c->t;
    host_fwd_mod_t(a, c->enc_tw, c->t);
    for (size_t j = 0; j < n; j++) vals[j] = a[bitrev((uint32_t)j, c->L)];
    return FHE_OK;
}

// ------------------------------------------------------------- enc / dec ----

fhe_status fhe_encrypt(fhe_ctx *c, const uint64_t *pk_dev, const uint64_t *pt, const int8_t *u,
                       const int32_t *e, uint64_t *ct_dev, size_t count, void *ws, size_t ws_bytes,
                       hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!pk_dev || !pt || !u || !e || !ct_dev || !ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_ENCRYPT, count)) return FHE_EWORKSPACE;
    for (size_t i = 0; i < count * c->n; i++)
        if (pt[i] >= c->t) return FHE_EINVAL;
    const size_t n = c->n, k = c->k, kn = k * n;
    uint64_t *PK = (uint64_t *)ws, *U = PK + 2 * kn, *prod = U + count * kn, *pt_dev = prod + 2 * count * kn;
    int8_t *u_dev = (int8_t *)(pt_dev + count * n);
    int32_t *e_dev = (int32_t *)(u_dev + ((count * n + 63) & ~(size_t)63));
    const DevCtx &d = c->dev;
    FHE_HIP(hipMemcpyAsync(PK, pk_dev, 2 * kn * 8, hipMemcpyDeviceToDevice, st));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, PK, 2 * k, k, 0, NTT_FWD, st); }));
    FHE_HIP(hipMemcpyAsync(u_dev, u, count * n, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_small_to_rns(d, u_dev, 1, U, count, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, U, count * k, k, 0, NTT_FWD, st); }));
    for (int p = 0; p < 2; p++) {
        uint64_t *dst = prod + p * count * kn;
        FHE_TRY(run(c, KK_MISC, st,
                    [&] { return launch_pointwise_mont(d, U, PK + p * kn, dst, count * k, 1, st); }));
    }
    FHE_TRY(run(c, KK_NTT_ROWS, st,
                [&] { return launch_ntt_rows(d, prod, 2 * count * k, k, 0, NTT_INV_MONT, st); }));
    FHE_HIP(hipMemcpyAsync(e_dev, e, count * 2 * n * 4, hipMemcpyHostToDevice, st));
    FHE_HIP(hipMemcpyAsync(pt_dev, pt, count * n * 8, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_encrypt_finish(d, prod, e_dev, pt_dev, ct_dev, count, st); }));
    FHE_HIP(hipStreamSynchronize(st));
    return FHE_OK;
}

fhe_status fhe_decrypt(fhe_ctx *c, const int8_t *s, const uint64_t *ct_dev, uint64_t *pt, size_t count,
                       void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!s || !ct_dev || !pt || !ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_DECRYPT, count)) return FHE_EWORKSPACE;
    const size_t n = c->n, k = c->k, kn = k * n;
    uint64_t *S = (uint64_t *)ws, *C1 = S + kn, *X = C1 + count * kn, *pt_dev = X + count * kn;
    int8_t *s_dev = (int8_t *)(pt_dev + count * n);
    const DevCtx &d = c->dev;
    FHE_HIP(hipMemcpyAsync(s_dev, s, n, hipMemcpyHostToDevice, st));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_small_to_rns(d, s_dev, 1, S, 1, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, S, k, k, 0, NTT_FWD, st); }));
    // C1 <- c1 of every ciphertext, X <- c1 s
    FHE_HIP(hipMemcpy2DAsync(C1, kn * 8, ct_dev + kn, 2 * kn * 8, kn * 8, count, hipMemcpyDeviceToDevice, st));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, C1, count * k, k, 0, NTT_FWD, st); }));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_pointwise_mont(d, C1, S, X, count * k, 1, st); }));
    FHE_TRY(run(c, KK_NTT_ROWS, st, [&] { return launch_ntt_rows(d, X, count * k, k, 0, NTT_INV_MONT, st); }));
    // X <- X + c0
    FHE_HIP(hipMemcpy2DAsync(C1, kn * 8, ct_dev, 2 * kn * 8, kn * 8, count, hipMemcpyDeviceToDevice, st));
    FHE_TRY(run(c, KK_ELEMENTWISE, st, [&] { return launch_addsub(d, X, C1, X, count * k, 0, st); }));
    FHE_TRY(run(c, KK_MISC, st, [&] { return launch_decrypt_scale(d, X, pt_dev, count, st); }));
    FHE_HIP(hipMemcpyAsync(pt, pt_dev, count * n * 8, hipMemcpyDeviceToHost, st));
    FHE_HIP(hipStreamSynchronize(st));
    return FHE_OK;
}

// ----------------------------------------------------------- elementwise ----

static fhe_status addsub_common(fhe_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out,
                                size_t count, int op, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!a || !out || (op != 2 && !b)) return FHE_EINVAL;
    const size_t bytes = count * ct_words(c) * 8;
    if (out != a && overlaps(out, a, bytes)) return FHE_EINVAL;
    if (op != 2 && out != b && overlaps(out, b, bytes)) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, a, count * 2 * c->k, c->k, 0, st));
    if (op != 2) FHE_TRY(check_canonical(c, b, count * 2 * c->k, c->k, 0, st));
    return run(c, KK_ELEMENTWISE, st,
               [&] { return launch_addsub(c->dev, a, b, out, count * 2 * c->k, op, st); });
}

fhe_status fhe_add(fhe_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count,
                   hipStream_t st) {
    return addsub_common(c, a, b, out, count, 0, st);
}

fhe_status fhe_sub(fhe_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count,
                   hipStream_t st) {
    return addsub_common(c, a, b, out, count, 1, st);
}

fhe_status fhe_neg(fhe_ctx *c, const uint64_t *a, uint64_t *out, size_t count, hipStream_t st) {
    return addsub_common(c, a, nullptr, out, count, 2, st);
}

static fhe_status plain_common(fhe_ctx *c, const uint64_t *a, uint64_t cval, uint64_t *out,
                               size_t count, int sign, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!a || !out) return FHE_EINVAL;
    if (cval >= c->t) return FHE_EINVAL;
    const size_t bytes = count * ct_words(c) * 8;
    if (out != a && overlaps(out, a, bytes)) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, a, count * 2 * c->k, c->k, 0, st));
    return run(c, KK_ELEMENTWISE, st,
               [&] { return launch_plain_const(c->dev, a, out, count, cval, sign, st); });
}

fhe_status fhe_add_plain_const(fhe_ctx *c, const uint64_t *a, uint64_t cval, uint64_t *out,
                               size_t count, hipStream_t st) {
    return plain_common(c, a, cval, out, count, +1, st);
}

fhe_status fhe_sub_plain_const(fhe_ctx *c, const uint64_t *a, uint64_t cval, uint64_t *out,
                               size_t count, hipStream_t st) {
    return plain_common(c, a, cval, out, count, -1, st);
}

// -------------------------------------------------------------- hot path ----

static fhe_status mul_args_ok(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                              uint64_t *out, size_t count, void *ws, size_t ws_bytes);

fhe_status fhe_mul_relin_static(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                                uint64_t *out, size_t count, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!c->scratch) return FHE_EDEVICE;
    const bool square = (a == b);
    const size_t need = fhe_workspace_bytes(c, square ? FHE_OP_SQUARE_RELIN : FHE_OP_MUL_RELIN, count);
    if (need > (size_t)FHE_STATIC_WS_BYTES) return FHE_EWORKSPACE;
    // the static array is the library's own memory: only the operands'
    // mutual aliasing needs checking (mul_args_ok with the array as workspace)
    FHE_TRY(mul_args_ok(c, rlk, a, b, out, count, c->scratch, FHE_STATIC_WS_BYTES));
    FHE_TRY(check_canonical(c, a, count * 2 * c->k, c->k, 0, st));
    if (!square) FHE_TRY(check_canonical(c, b, count * 2 * c->k, c->k, 0, st));
    // per-launch timing would create events on demand: off for this call
    const bool timing = c->timing;
    c->timing = false;
    const fhe_status res = mul_relin_impl(c, rlk, a, b, out, count, c->scratch, st);
    c->timing = timing;
    return res;
}

fhe_status fhe_mul_relin(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                         uint64_t *out, size_t count, void *ws, size_t ws_bytes, hipStream_t st) {
    FHE_TRY(mul_args_ok(c, rlk, a, b, out, count, ws, ws_bytes));
    if (count == 0) return FHE_OK;
    const bool square = (a == b);
    FHE_TRY(check_canonical(c, a, count * 2 * c->k, c->k, 0, st));
    if (!square) FHE_TRY(check_canonical(c, b, count * 2 * c->k, c->k, 0, st));
    return mul_relin_impl(c, rlk, a, b, out, count, ws, st);
}

fhe_status fhe_autotune_mul_relin(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                                  uint64_t *out, size_t count, void *ws, size_t ws_bytes, hipStream_t st,
                                  size_t *chunk_out, int *fused_out) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_EINVAL;
    if (!rlk || !a || !b || !out || !ws) return FHE_EINVAL;
    const bool square = (a == b);
    const size_t bytes = count * ct_words(c) * 8;
    if (overlaps(out, a, bytes) || overlaps(out, b, bytes)) return FHE_EINVAL;
    const size_t saved_limit = c->batch_limit, saved_thr = c->fused_min_rows[square ? 1 : 0];
    drop_graphs(c);  // recorded graphs hold the launch shape this call changes
    // candidates: chunk caps (whole batch, halves, quarters) x fused or not
    size_t caps[3];
    int ncaps = 0;
    for (size_t div = 1; div <= 4 && ncaps < 3; div *= 2) {
        size_t cap = (count + div - 1) / div;
        if (cap > saved_limit) cap = saved_limit;
        if (ncaps == 0 || caps[ncaps - 1] != cap) caps[ncaps++] = cap;
    }
    if (ws_bytes < fhe_workspace_bytes(c, square ? FHE_OP_SQUARE_RELIN : FHE_OP_MUL_RELIN, count)) return FHE_EWORKSPACE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FHE_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FHE_EDEVICE;
    }
    const bool timing = c->timing;
    c->timing = false;
    float best = -1.0f;
    size_t best_cap = saved_limit;
    int best_fused = 1;
    fhe_status st_all = FHE_OK;
    for (int ci = 0; ci < ncaps && st_all == FHE_OK; ci++)
        for (int fused = 0; fused < 2 && st_all == FHE_OK; fused++) {
            c->batch_limit = caps[ci];
            c->fused_min_rows[square ? 1 : 0] = fused ? 0 : (size_t)-1;
            st_all = mul_relin_impl(c, rlk, a, b, out, count, ws, st);  // warm
            if (st_all != FHE_OK) break;
            float total = 0.0f;
            for (int rep = 0; rep < 3 && st_all == FHE_OK; rep++) {
                if (hipEventRecord(e0, st) != hipSuccess) st_all = FHE_EDEVICE;
                if (st_all == FHE_OK) st_all = mul_relin_impl(c, rlk, a, b, out, count, ws, st);
                if (st_all == FHE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                    st_all = FHE_EDEVICE;
                float ms = 0.0f;
                if (st_all == FHE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st_all = FHE_EDEVICE;
                total += ms;
            }
            if (st_all == FHE_OK && (best < 0.0f || total < best)) {
                best = total;
                best_cap = caps[ci];
                best_fused = fused;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = timing;
    if (st_all != FHE_OK) {
        c->batch_limit = saved_limit;
        c->fused_min_rows[square ? 1 : 0] = saved_thr;
        return st_all;
    }
    // keep the winner: the chunk cap, and a threshold that sends this batch's
    // chunks to the faster product path
    c->batch_limit = best_cap;
    const size_t rows = best_cap * c->K;
    c->fused_min_rows[square ? 1 : 0] = best_fused ? (saved_thr < rows ? saved_thr : rows) : rows + 1;
    if (chunk_out) *chunk_out = best_cap;
    if (fused_out) *fused_out = best_fused;
    return FHE_OK;
}

static fhe_status ensure_aux(fhe_ctx *c) {
    if (c->aux) return FHE_OK;
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
        c->aux = nullptr;
        return FHE_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess)
        return FHE_EDEVICE;
    return FHE_OK;
}

// The persistent key switching of fhe_mul_relin_multi takes parts of ring
// sizes 4096, 8192 and 16384 whose batch fits one chunk (its C2 stays in the
// part's workspace until the shared launch), at most kMaxPersistParts of
// them, when the leading context allows it and at least two ring sizes meet.
static bool persistent_applies(const fhe_mul_part *parts, size_t nparts) {
    if (!parts[0].ctx->multi_persistent || nparts > kMaxPersistParts) return false;
    uint32_t sizes = 0;
    int lazy = -1, raw = -1;
    for (size_t i = 0; i < nparts; i++) {
        const fhe_mul_part &p = parts[i];
        if (p.count == 0) continue;
        const uint32_t n = p.ctx->n;
        if ((n != 4096 && n != 8192 && n != 16384) || p.count > p.ctx->batch_limit ||
            p.count * p.ctx->k >= (1ull << 31))
            return false;
        // one key-switching variant per launch
        const int l = p.ctx->dev.lazy_q ? 1 : 0, r = (p.ctx->dev.lazy_q && p.ctx->dev.digit_raw) ? 1 : 0;
        if ((lazy >= 0 && l != lazy) || (raw >= 0 && r != raw)) return false;
        lazy = l;
        raw = r;
        sizes |= n;
    }
    return (sizes & (sizes - 1)) != 0;
}

static fhe_status ensure_persist(fhe_ctx *c) {
    if (c->d_persist) return FHE_OK;
    if (hipMalloc(&c->d_persist, 256) != hipSuccess) {
        c->d_persist = nullptr;
        return FHE_ENOMEM;
    }
    return FHE_OK;
}

static fhe_status mul_args_ok(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                              uint64_t *out, size_t count, void *ws, size_t ws_bytes) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!rlk || !a || !b || !out || !ws) return FHE_EINVAL;
    const size_t bytes = count * ct_words(c) * 8;
    if (out != a && overlaps(out, a, bytes)) return FHE_EINVAL;
    if (out != b && overlaps(out, b, bytes)) return FHE_EINVAL;
    const size_t need = fhe_workspace_bytes(c, a == b ? FHE_OP_SQUARE_RELIN : FHE_OP_MUL_RELIN, count);
    if (ws_bytes < need) return FHE_EWORKSPACE;
    // the pipeline writes all of its workspace: it must not overlap any operand
    if (overlaps2(ws, need, a, bytes) || overlaps2(ws, need, b, bytes) || overlaps2(ws, need, out, bytes))
        return FHE_EINVAL;
    return FHE_OK;
}

fhe_status fhe_mul_relin_multi(const fhe_mul_part *parts, size_t nparts, hipStream_t st) {
    if (nparts == 0) return FHE_OK;
    if (!parts) return FHE_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FHE_EDEVICE;
    for (size_t i = 0; i < nparts; i++) {
        const fhe_mul_part &p = parts[i];
        if (!p.ctx) return FHE_EINVAL;
        FHE_TRY(mul_args_ok(p.ctx, p.rlk_dev, p.a, p.b, p.out, p.count, p.ws, p.ws_bytes));
        if (p.ctx->device != dev) return FHE_EINVAL;
        if (p.count == 0) continue;
        const size_t pb = p.count * ct_words(p.ctx) * 8;
        const size_t pw = fhe_workspace_bytes(p.ctx, p.a == p.b ? FHE_OP_SQUARE_RELIN : FHE_OP_MUL_RELIN, p.count);
        for (size_t j = 0; j < nparts; j++) {
            const fhe_mul_part &o = parts[j];
            if (j == i || o.count == 0) continue;
            const size_t ob = o.count * ct_words(o.ctx) * 8;
            const size_t ow = fhe_workspace_bytes(o.ctx, o.a == o.b ? FHE_OP_SQUARE_RELIN : FHE_OP_MUL_RELIN, o.count);
            // parts may run concurrently: an output or a workspace of one part
            // must not overlap anything another part reads or writes
            if (overlaps2(p.out, pb, o.out, ob) || overlaps2(p.out, pb, o.a, ob) || overlaps2(p.out, pb, o.b, ob) ||
                overlaps2(p.ws, pw, o.ws, ow) || overlaps2(p.ws, pw, o.a, ob) || overlaps2(p.ws, pw, o.b, ob) ||
                overlaps2(p.ws, pw, o.out, ob))
                return FHE_EINVAL;
        }
        FHE_TRY(ensure_aux(p.ctx));
    }
    fhe_ctx *lead = parts[0].ctx;
    const bool persist = persistent_applies(parts, nparts);
    if (persist) FHE_TRY(ensure_persist(lead));
    hipEvent_t fork = lead->fork_ev;
    FHE_HIP(hipEventRecord(fork, st));
    // on an error after some parts were enqueued, `st` still waits for them,
    // so the caller's stream never runs ahead of work on its buffers
    fhe_status res = FHE_OK;
    size_t enq = 0;
    for (; enq < nparts && res == FHE_OK; enq++) {
        const fhe_mul_part &p = parts[enq];
        if (p.count == 0) continue;
        fhe_ctx *c = p.ctx;
        if (hipStreamWaitEvent(c->aux, fork, 0) != hipSuccess) {
            res = FHE_EDEVICE;
            break;
        }
        res = check_canonical(c, p.a, p.count * 2 * c->k, c->k, 0, c->aux);
        if (res == FHE_OK && p.a != p.b) res = check_canonical(c, p.b, p.count * 2 * c->k, c->k, 0, c->aux);
        if (res == FHE_OK) res = mul_relin_impl(c, p.rlk_dev, p.a, p.b, p.out, p.count, p.ws, c->aux, !persist);
        if (hipEventRecord(c->join_ev, c->aux) != hipSuccess && res == FHE_OK) res = FHE_EDEVICE;
    }
    for (size_t i = 0; i < enq && i < nparts; i++)
        if (parts[i].count && hipStreamWaitEvent(st, parts[i].ctx->join_ev, 0) != hipSuccess && res == FHE_OK)
            res = FHE_EDEVICE;
    if (res != FHE_OK || !persist) return res;
    // every part's C2 is ready: one persistent key-switching launch over all
    // of them, largest ring first
    std::vector<size_t> order;
    for (size_t i = 0; i < nparts; i++)
        if (parts[i].count) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return parts[x].ctx->n > parts[y].ctx->n; });
    RelinQueue Q{};
    size_t tasks = 0;
    for (size_t o = 0; o < order.size(); o++) {
        const fhe_mul_part &p = parts[order[o]];
        const fhe_ctx *c = p.ctx;
        const size_t per = 16384 / c->n, rows = p.count * c->k;
        RelinPart &r = Q.part[o];
        r.c = c->dev;
        r.C2 = c2_of_single_chunk(c, p.ws, p.count, p.a == p.b);
        r.rlk = p.rlk_dev;
        r.out = p.out;
        r.items = (uint32_t)p.count;
        r.wg_tasks = (uint32_t)((rows + per - 1) / per);
        r.kmagic = (uint32_t)(((1ull << 32) + c->k - 1) / c->k);
        tasks += r.wg_tasks;
    }
    Q.nparts = (int)order.size();
    unsigned int *queue = (unsigned int *)lead->d_persist;
    const DevCtx &d0 = parts[order[0]].ctx->dev;
    const int lazy = d0.lazy_q ? 1 : 0, raw = (d0.lazy_q && d0.digit_raw) ? 1 : 0;
    return run(lead, KK_RELIN_FUSED, st, [&] { return launch_relin_persist(Q, lazy, raw, queue, tasks, st); });
}

fhe_status fhe_set_multi_persistent(fhe_ctx *c, int enable) {
    if (!c) return FHE_EINVAL;
    c->multi_persistent = enable ? 1 : 0;
    return FHE_OK;
}

fhe_status fhe_autotune_mul_relin_multi(const fhe_mul_part *parts, size_t nparts, hipStream_t st,
                                        int *persistent) {
    if (nparts == 0 || !parts || !parts[0].ctx) return FHE_EINVAL;
    fhe_ctx *lead = parts[0].ctx;
    const int saved = lead->multi_persistent;
    // time both modes only where the persistent launch applies
    lead->multi_persistent = 1;
    const bool applies = persistent_applies(parts, nparts);
    lead->multi_persistent = saved;
    if (!applies) {
        if (persistent) *persistent = 0;
        lead->multi_persistent = 0;
        return FHE_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FHE_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FHE_EDEVICE;
    }
    float best = -1.0f;
    int best_mode = 0;
    fhe_status res = FHE_OK;
    for (int mode = 0; mode < 2 && res == FHE_OK; mode++) {
        lead->multi_persistent = mode;
        res = fhe_mul_relin_multi(parts, nparts, st);  // warm
        float total = 0.0f;
        for (int rep = 0; rep < 3 && res == FHE_OK; rep++) {
            if (hipEventRecord(e0, st) != hipSuccess) res = FHE_EDEVICE;
            if (res == FHE_OK) res = fhe_mul_relin_multi(parts, nparts, st);
            if (res == FHE_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                res = FHE_EDEVICE;
            float ms = 0.0f;
            if (res == FHE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) res = FHE_EDEVICE;
            total += ms;
        }
        if (res == FHE_OK && (best < 0.0f || total < best)) {
            best = total;
            best_mode = mode;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    lead->multi_persistent = res == FHE_OK ? best_mode : saved;
    if (res == FHE_OK && persistent) *persistent = best_mode;
    return res;
}

fhe_status fhe_square_chain(fhe_ctx *c, const uint64_t *rlk, uint64_t *x, uint32_t depth, size_t count,
                            void *ws, size_t ws_bytes, int graph, hipStream_t st) {
    FHE_TRY(mul_args_ok(c, rlk, x, x, x, count, ws, ws_bytes));
    if (count == 0 || depth == 0) return FHE_OK;
    FHE_TRY(check_canonical(c, x, count * 2 * c->k, c->k, 0, st));
    // eager when not asked for a graph, and when validation (memsets) or
    // per-launch timing (events) is on
    if (!graph || c->validate || c->timing) {
        for (uint32_t d = 0; d < depth; d++) FHE_TRY(mul_relin_impl(c, rlk, x, x, x, count, ws, st));
        return FHE_OK;
    }
    const size_t thr = c->fused_min_rows[1];
    for (auto &cg : c->graphs)
        if (cg.rlk == rlk && cg.x == x && cg.ws == ws && cg.count == count && cg.depth == depth &&
            cg.ws_bytes == ws_bytes && cg.batch_limit == c->batch_limit && cg.fused_min_rows == thr) {
            FHE_HIP(hipGraphLaunch(cg.ge, st));
            FHE_HIP(hipEventRecord(cg.done, st));
            return FHE_OK;
        }
    // bounded cache: the oldest graph goes first
    while (c->graphs.size() >= kMaxGraphs) drop_graph(c, 0);
    // record the launches on the context's own stream (capture executes
    // nothing), then run the graph on the caller's stream
    FHE_TRY(ensure_aux(c));
    FHE_HIP(hipStreamBeginCapture(c->aux, hipStreamCaptureModeRelaxed));
    fhe_status rec = FHE_OK;
    for (uint32_t d = 0; d < depth && rec == FHE_OK; d++) rec = mul_relin_impl(c, rlk, x, x, x, count, ws, c->aux);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->aux, &g);
    if (rec != FHE_OK || ec != hipSuccess || !g) {
        if (g) hipGraphDestroy(g);
        return rec != FHE_OK ? rec : FHE_EDEVICE;
    }
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(g);
        return FHE_EDEVICE;
    }
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
        hipGraphExecDestroy(ge);
        hipGraphDestroy(g);
        return FHE_EDEVICE;
    }
    c->graphs.push_back({rlk, x, ws, count, ws_bytes, c->batch_limit, thr, depth, g, ge, done});
    FHE_HIP(hipGraphLaunch(ge, st));
    FHE_HIP(hipEventRecord(done, st));
    return FHE_OK;
}

fhe_status fhe_bridge_to_bits(fhe_ctx *c, const uint64_t *rlk, const uint64_t *x, uint32_t nbits,
                              uint64_t *bits, uint64_t *eq, size_t count, void *ws, size_t ws_bytes,
                              hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (c->encoding != FHE_ENC_COEFF || !is_prime_u64(c->t) || c->t < 3 ||
        ((c->t - 1) & (c->t - 2)) != 0 || c->t > 65537)
        return FHE_EUNSUPPORTED;
    if (nbits == 0 || nbits > 20 || (1ull << nbits) < c->t) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!rlk || !x || !bits || !ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_BRIDGE, count)) return FHE_EWORKSPACE;
    const size_t ctw = ct_words(c);
    if (overlaps2(bits, count * nbits * ctw * 8, x, count * ctw * 8)) return FHE_EINVAL;
    if (eq && (overlaps2(eq, count * c->t * ctw * 8, x, count * ctw * 8) ||
               overlaps2(eq, count * c->t * ctw * 8, bits, count * nbits * ctw * 8)))
        return FHE_EINVAL;
    FHE_TRY(check_canonical(c, x, count * 2 * c->k, c->k, 0, st));
    const int T = (int)c->t;
    // without eq outputs the test c = 0 contributes to no bit and is skipped
    const int c0 = eq ? 0 : 1, Tc = T - c0;
    int squarings = 0;
    while ((1ull << squarings) < c->t - 1) squarings++;
    const size_t G = bridge_group(c);
    const size_t gmax = count < G ? count : G;
    uint64_t *y = (uint64_t *)ws;
    void *ws2 = y + gmax * T * ctw;
    const DevCtx &d = c->dev;
    for (size_t g0 = 0; g0 < count; g0 += G) {
        const size_t gc = count - g0 < G ? count - g0 : G;
        const size_t chains = gc * Tc;
        // First squaring, shared by the chains of an input (kernels_conv.hip):
        // the input's own square up to the key switching, then per chain the
        // corrected components 0 and 1 plus the shared key-switching output.
        const uint64_t *xg = x + g0 * ctw;
        const size_t n = c->n, K = c->K, k = c->k;
        uint64_t *E1 = (uint64_t *)ws2;
        uint64_t *D1 = E1 + gc * 2 * K * n;
        uint64_t *C21 = D1 + gc * 3 * K * n;
        uint64_t *R1 = C21 + gc * k * n;
        uint64_t *gam = R1 + gc * 2 * k * n;
        FHE_TRY(run(c, KK_LIFT, st, [&] { return launch_lift(d, xg, xg, E1, 2, gc, st); }));
        FHE_TRY(run(c, KK_SQUARE_TENSOR, st, [&] { return launch_square_tensor(d, xg, E1, D1, gc, st); }));
        FHE_TRY(run(c, KK_SCALE, st, [&] { return launch_scale(d, D1, nullptr, C21, gc, st, 2, 1); }));
        FHE_HIP(hipMemsetAsync(R1, 0, gc * 2 * k * n * sizeof(uint64_t), st));
        FHE_TRY(run(c, KK_RELIN_FUSED, st, [&] { return launch_relin_fused(d, C21, rlk, R1, gc, st); }));
        FHE_TRY(run(c, KK_BRIDGE, st, [&] { return launch_bridge_gamma(d, xg, E1, gam, chains, Tc, c0, st); }));
        FHE_TRY(run(c, KK_SCALE, st,
                    [&] { return launch_scale_chain(d, D1, xg, E1, gam, R1, y, chains, Tc, st); }));
        for (int sq = 1; sq < squarings; sq++) FHE_TRY(mul_relin_impl(c, rlk, y, y, y, chains, ws2, st));
        uint64_t *eqp = eq ? eq + g0 * T * ctw : nullptr;
        FHE_TRY(run(c, KK_BRIDGE, st, [&] {
            return launch_bridge_combine(d, y, bits + g0 * nbits * ctw, eqp, gc, Tc, (int)nbits, c0, st);
        }));
    }
    return FHE_OK;
}

fhe_status fhe_bits_to_mod(fhe_ctx *c, const uint64_t *bits, uint32_t nbits, uint64_t *out,
                           size_t count, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (nbits == 0) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!bits || !out) return FHE_EINVAL;
    if (overlaps2(out, count * ct_words(c) * 8, bits, count * nbits * ct_words(c) * 8)) return FHE_EINVAL;
    return run(c, KK_ELEMENTWISE, st,
               [&] { return launch_horner(c->dev, bits, (int)nbits, out, count, 0, st); });
}




// ------------------------------------------------- modular linear stage ----

// Weight rows [nout][nin] padded to the kernel's row stride, staged in pinned
// memory (the previous copy out of it must have finished), then copied
// asynchronously to dst on st.
// Pinned staging buffer of at least `words` 32-bit words (the previous copy
// out of it must have finished first).
static fhe_status pinned_stage(fhe_ctx *c, size_t words) {
    if (!c->wpin_ev && hipEventCreateWithFlags(&c->wpin_ev, hipEventDisableTiming) != hipSuccess) {
        c->wpin_ev = nullptr;
        return FHE_EDEVICE;
    }
    FHE_HIP(hipEventSynchronize(c->wpin_ev));
    if (words > c->wpin_cap) {
        if (c->wpin) (void)hipHostFree(c->wpin);
        c->wpin = nullptr;
        c->wpin_cap = 0;
        if (hipHostMalloc((void **)&c->wpin, words * 4, hipHostMallocDefault) != hipSuccess) {
            c->wpin = nullptr;
            return FHE_ENOMEM;
        }
        c->wpin_cap = words;
    }
    return FHE_OK;
}

static fhe_status stage_weights(fhe_ctx *c, const int32_t *w, size_t nout, size_t nin, int32_t *dst,
                                hipStream_t st) {
    const size_t stride = weighted_sum_row_stride(nin);
    const size_t words = nout * stride;
    FHE_TRY(pinned_stage(c, words));
    std::memset(c->wpin, 0, words * 4);
    for (size_t m = 0; m < nout; m++) std::memcpy(c->wpin + m * stride, w + m * nin, nin * 4);
    FHE_HIP(hipMemcpyAsync(dst, c->wpin, words * 4, hipMemcpyHostToDevice, st));
    FHE_HIP(hipEventRecord(c->wpin_ev, st));
    return FHE_OK;
}

// The int8 operand table of the matrix-core weighted sum, staged like the weights.
static fhe_status stage_weights_mx(fhe_ctx *c, const int32_t *w, size_t nout, size_t nin, void *dst,
                                   hipStream_t st) {
    const size_t bytes = weighted_sum_mx_bytes(nout, nin);
    FHE_TRY(pinned_stage(c, (bytes + 3) / 4));
    weighted_sum_mx_table(w, nout, nin, (int8_t *)c->wpin);
    FHE_HIP(hipMemcpyAsync(dst, c->wpin, bytes, hipMemcpyHostToDevice, st));
    FHE_HIP(hipEventRecord(c->wpin_ev, st));
    return FHE_OK;
}

fhe_status fhe_weighted_sum(fhe_ctx *c, const uint64_t *in, size_t nin, const int32_t *w, size_t nout,
                            uint64_t *out, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (nout == 0) return FHE_OK;
    if (!out || (nin && (!in || !w || !ws))) return FHE_EINVAL;
    const size_t ctb = ct_words(c) * 8;
    if (nin && overlaps2(out, nout * ctb, in, nin * ctb)) return FHE_EINVAL;
    if (nin == 0) {
        FHE_HIP(hipMemsetAsync(out, 0, nout * ctb, st));
        return FHE_OK;
    }
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_WEIGHTED_SUM, nout * nin)) return FHE_EWORKSPACE;
    const size_t stride = weighted_sum_row_stride(nin);
    for (size_t m = 0; m < nout; m++) {
        uint64_t abs_sum = 0;
        for (size_t j = 0; j < nin; j++) {
            const int64_t v = w[m * nin + j];
            abs_sum += (uint64_t)(v < 0 ? -v : v);
        }
        if (abs_sum >= (1ull << 30)) return FHE_EINVAL;
    }
    (void)stride;
    FHE_TRY(check_canonical(c, in, nin * 2 * c->k, c->k, 0, st));
    // the matrix cores (with the context's matrix-core conversions) for weights in [-127, 127]
    bool mx = c->dev.mx != nullptr;
    for (size_t i = 0; mx && i < nout * nin; i++) mx = w[i] >= -127 && w[i] <= 127;
    if (mx) {
        FHE_TRY(stage_weights_mx(c, w, nout, nin, ws, st));
        return run(c, KK_ELEMENTWISE, st,
                   [&] { return launch_weighted_sum_mx(c->dev, in, nin, ws, nout, out, st); });
    }
    int32_t *wd = (int32_t *)ws;
    FHE_TRY(stage_weights(c, w, nout, nin, wd, st));
    return run(c, KK_ELEMENTWISE, st, [&] { return launch_weighted_sum(c->dev, in, nin, wd, nout, out, st); });
}

// ------------------------------------------------------ bit-level side ----
// Compositions of the product and the elementwise kernels, in the order the
// header documents (the oracle evaluates the same sequence).

static fhe_status ew(fhe_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t count, int op,
                     hipStream_t st) {  // op 0: a + b, 1: a - b, 2: -a
    return run(c, KK_ELEMENTWISE, st,
               [&] { return launch_addsub(c->dev, a, b, out, count * 2 * c->k, op, st); });
}

static fhe_status one_minus(fhe_ctx *c, const uint64_t *a, uint64_t *out, size_t count, hipStream_t st) {
    FHE_TRY(ew(c, a, nullptr, out, count, 2, st));
    return run(c, KK_ELEMENTWISE, st, [&] { return launch_plain_const(c->dev, out, out, count, 1, +1, st); });
}

static fhe_status gate_impl(fhe_ctx *c, const uint64_t *rlk, int gate, const uint64_t *a, const uint64_t *b,
                            const uint64_t *cc, uint64_t *out, size_t count, void *ws, hipStream_t st) {
    const size_t ctw = ct_words(c);
    uint64_t *t0 = (uint64_t *)ws, *t1 = t0 + count * ctw;
    void *mws = t1 + count * ctw;
    switch (gate) {
        case FHE_GATE_NOT:
            return one_minus(c, a, out, count, st);
        case FHE_GATE_MUX:
            FHE_TRY(ew(c, b, cc, t0, count, 1, st));
            FHE_TRY(mul_relin_impl(c, rlk, a, t0, t1, count, mws, st));
            return ew(c, t1, cc, out, count, 0, st);
        case FHE_GATE_AND:
            return mul_relin_impl(c, rlk, a, b, out, count, mws, st);
        default:
            break;
    }
    FHE_TRY(mul_relin_impl(c, rlk, a, b, t0, count, mws, st));  // p = a b
    if (gate == FHE_GATE_NAND) return one_minus(c, t0, out, count, st);
    FHE_TRY(ew(c, a, b, out, count, 0, st));
    FHE_TRY(ew(c, out, t0, out, count, 1, st));  // OR
    if (gate == FHE_GATE_XOR || gate == FHE_GATE_XNOR) FHE_TRY(ew(c, out, t0, out, count, 1, st));
    if (gate == FHE_GATE_NOR || gate == FHE_GATE_XNOR) return one_minus(c, out, out, count, st);
    return FHE_OK;
}

fhe_status fhe_gate(fhe_ctx *c, const uint64_t *rlk, int gate, const uint64_t *a, const uint64_t *b,
                    const uint64_t *cc, uint64_t *out, size_t count, void *ws, size_t ws_bytes,
                    hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (gate < FHE_GATE_AND || gate > FHE_GATE_MUX) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    const bool needs_b = gate != FHE_GATE_NOT, needs_c = gate == FHE_GATE_MUX, needs_mul = gate != FHE_GATE_NOT;
    if (!a || !out || (needs_b && !b) || (needs_c && !cc) || (needs_mul && (!rlk || !ws))) return FHE_EINVAL;
    const size_t bytes = count * ct_words(c) * 8;
    if (out != a && overlaps(out, a, bytes)) return FHE_EINVAL;
    if (needs_b && out != b && overlaps(out, b, bytes)) return FHE_EINVAL;
    if (needs_c && out != cc && overlaps(out, cc, bytes)) return FHE_EINVAL;
    if (needs_mul && ws_bytes < fhe_workspace_bytes(c, FHE_OP_GATE, count)) return FHE_EWORKSPACE;
    FHE_TRY(check_canonical(c, a, count * 2 * c->k, c->k, 0, st));
    if (needs_b) FHE_TRY(check_canonical(c, b, count * 2 * c->k, c->k, 0, st));
    if (needs_c) FHE_TRY(check_canonical(c, cc, count * 2 * c->k, c->k, 0, st));
    return gate_impl(c, rlk, gate, a, b, cc, out, count, ws, st);
}

// Bit i of every item of a [count][nbits][2][k][n] into a contiguous [count] block.
static fhe_status gather_bit(fhe_ctx *c, const uint64_t *v, uint32_t nbits, uint32_t i, uint64_t *dst,
                             size_t count, hipStream_t st) {
    const size_t ctb = ct_words(c) * 8;
    FHE_HIP(hipMemcpy2DAsync(dst, ctb, v + (size_t)i * ct_words(c), nbits * ctb, ctb, count,
                             hipMemcpyDeviceToDevice, st));
    return FHE_OK;
}

static fhe_status less_than_impl(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b,
                                 uint32_t nbits, uint64_t *out, size_t count, void *ws, hipStream_t st) {
    const size_t cw = count * ct_words(c);
    uint64_t *A = (uint64_t *)ws, *B = A + cw, *Pr = B + cw, *D = Pr + cw, *E = D + cw, *T = E + cw;
    void *mws = T + cw;
    for (uint32_t i = 0; i < nbits; i++) {
        FHE_TRY(gather_bit(c, a, nbits, i, A, count, st));
        FHE_TRY(gather_bit(c, b, nbits, i, B, count, st));
        FHE_TRY(mul_relin_impl(c, rlk, A, B, Pr, count, mws, st));  // p = a_i b_i
        if (i == 0) {
            FHE_TRY(ew(c, B, Pr, out, count, 1, st));  // lt = d_0
            continue;
        }
        FHE_TRY(ew(c, B, Pr, D, count, 1, st));   // d = b_i - p
        FHE_TRY(ew(c, A, B, E, count, 0, st));    // e = 1 - ((a + b) - p - p)
        FHE_TRY(ew(c, E, Pr, E, count, 1, st));
        FHE_TRY(ew(c, E, Pr, E, count, 1, st));
        FHE_TRY(one_minus(c, E, E, count, st));
        FHE_TRY(ew(c, out, D, T, count, 1, st));  // lt = e (lt - d) + d
        FHE_TRY(mul_relin_impl(c, rlk, E, T, T, count, mws, st));
        FHE_TRY(ew(c, T, D, out, count, 0, st));
    }
    return FHE_OK;
}

fhe_status fhe_less_than(fhe_ctx *c, const uint64_t *rlk, const uint64_t *a, const uint64_t *b, uint32_t nbits,
                         uint64_t *out, size_t count, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (nbits == 0) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!rlk || !a || !b || !out || !ws) return FHE_EINVAL;
    const size_t ctb = ct_words(c) * 8;
    if (overlaps2(out, count * ctb, a, count * nbits * ctb) || overlaps2(out, count * ctb, b, count * nbits * ctb))
        return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_COMPARE, count)) return FHE_EWORKSPACE;
    FHE_TRY(check_canonical(c, a, count * nbits * 2 * c->k, c->k, 0, st));
    FHE_TRY(check_canonical(c, b, count * nbits * 2 * c->k, c->k, 0, st));
    return less_than_impl(c, rlk, a, b, nbits, out, count, ws, st);
}

fhe_status fhe_argmax(fhe_ctx *c, const uint64_t *rlk, const uint64_t *scores, uint32_t ncls, uint32_t nbits,
                      uint64_t *out, size_t count, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (nbits == 0 || ncls < 2 || ncls > 16) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!rlk || !scores || !out || !ws) return FHE_EINVAL;
    const size_t ctw = ct_words(c), cw = count * ctw, sw = count * nbits * ctw;
    if (overlaps2(out, ncls * cw * 8, scores, ncls * sw * 8)) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_ARGMAX, count)) return FHE_EWORKSPACE;
    FHE_TRY(check_canonical(c, scores, ncls * count * nbits * 2 * c->k, c->k, 0, st));
    uint64_t *Lt = (uint64_t *)ws, *Na = Lt + cw;
    void *cws = Na + cw;
    void *mws = (uint8_t *)cws + 6 * cw * 8;  // the comparison's product workspace
    bool first[16];
    for (uint32_t a = 0; a < ncls; a++) first[a] = true;
    for (uint32_t a = 0; a < ncls; a++)
        for (uint32_t b = a + 1; b < ncls; b++) {
            FHE_TRY(less_than_impl(c, rlk, scores + a * sw, scores + b * sw, nbits, Lt, count, cws, st));
            FHE_TRY(one_minus(c, Lt, Na, count, st));
            uint64_t *oa = out + a * cw, *ob = out + b * cw;
            if (first[a]) FHE_HIP(hipMemcpyAsync(oa, Na, cw * 8, hipMemcpyDeviceToDevice, st));
            else FHE_TRY(mul_relin_impl(c, rlk, oa, Na, oa, count, mws, st));
            if (first[b]) FHE_HIP(hipMemcpyAsync(ob, Lt, cw * 8, hipMemcpyDeviceToDevice, st));
            else FHE_TRY(mul_relin_impl(c, rlk, ob, Lt, ob, count, mws, st));
            first[a] = first[b] = false;
        }
    return FHE_OK;
}

// ------------------------------------------------ bridge from the powers ----
// The bits of the bridge as weighted sums of x^0..x^(t-1): bit_j = sum over
// c in [1, t) with bit j of c set of 1 - (x - c)^(t-1), expanded binomially
// (centred weights modulo t); x^0 is the noiseless encryption of 1.

static void bridge_weights(uint64_t t, uint32_t nbits, std::vector<int32_t> &W) {
    W.assign((size_t)nbits * t, 0);
    std::vector<uint64_t> binom(t, 1);  // C(t-1, k) mod t
    for (uint64_t k = 1; k < t; k++) binom[k] = (uint64_t)((u128)binom[k - 1] * ((t - k) % t) % t * hinv(k % t, t) % t);
    for (uint32_t j = 0; j < nbits; j++) {
        std::vector<uint64_t> row(t, 0);
        for (uint64_t cc = 1; cc < t; cc++) {
            if (!((cc >> j) & 1)) continue;
            row[0] = (row[0] + 1) % t;
            const uint64_t mc = t - cc;  // -c mod t
            for (uint64_t k = 0; k < t; k++) {
                const uint64_t term = (uint64_t)((u128)binom[k] * hpow(mc, t - 1 - k, t) % t);
                row[k] = (row[k] + t - term) % t;
            }
        }
        for (uint64_t k = 0; k < t; k++)
            W[(size_t)j * t + k] = (int32_t)(row[k] > t / 2 ? (int64_t)row[k] - (int64_t)t : (int64_t)row[k]);
    }
}

fhe_status fhe_bridge_to_bits_powers(fhe_ctx *c, const uint64_t *rlk, const uint64_t *x, uint32_t nbits,
                                     uint64_t *bits, size_t count, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (c->encoding != FHE_ENC_COEFF || !is_prime_u64(c->t) || c->t < 3 || c->t > 257) return FHE_EUNSUPPORTED;
    if (nbits == 0 || nbits > 20 || (1ull << nbits) < c->t) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!rlk || !x || !bits || !ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_BRIDGE_POWERS, count)) return FHE_EWORKSPACE;
    const size_t ctw = ct_words(c), ctb = ctw * 8;
    if (overlaps2(bits, count * nbits * ctb, x, count * ctb)) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, x, count * 2 * c->k, c->k, 0, st));
    const size_t e = c->t - 1;
    size_t hmax = 1;
    while (hmax * 2 < e) hmax *= 2;
    const size_t G = powers_group(c);
    const size_t gmax = count < G ? count : G;
    // workspace: powers [e][gmax] (coefficient form), the transforms of the
    // extended powers x^1..x^hmax [hmax][gmax][2][K][n] (the operands of every
    // product), the weights, then the product workspace
    const size_t tw_words = 2 * (size_t)c->K * c->n;
    uint64_t *Pw = (uint64_t *)ws;
    uint64_t *T = Pw + e * gmax * ctw;
    int32_t *wd = (int32_t *)(T + hmax * gmax * tw_words);
    void *mws = (uint8_t *)wd + ((20 * weighted_sum_row_stride(c->t) * 4 + 255) / 256) * 256;
    std::vector<int32_t> W;
    bridge_weights(c->t, nbits, W);
    FHE_TRY(stage_weights(c, W.data(), nbits, c->t, wd, st));
    const DevCtx &d = c->dev;
    for (size_t g0 = 0; g0 < count; g0 += G) {
        const size_t gc = count - g0 < G ? count - g0 : G;
        const size_t bw = gc * ctw;      // one power of every input of the group
        const size_t tb = gc * tw_words; // its transform
        FHE_HIP(hipMemcpyAsync(Pw, x + g0 * ctw, bw * 8, hipMemcpyDeviceToDevice, st));
        FHE_TRY(run(c, KK_LIFT, st, [&] { return launch_lift(d, Pw, Pw, T, 2, gc, st); }));
        FHE_TRY(run(c, KK_FWD_EXT, st, [&] { return launch_fwd_ext(d, Pw, Pw, T, 2, gc, st); }));
        // level of x^(h+1) .. x^(2h): x^(h+r) = x^h x^r, r = 1..min(h, e - h),
        // from the cached transforms; the new powers up to hmax are then
        // lifted and transformed once for the later levels
        for (size_t h = 1; h < e; h *= 2) {
            const size_t nk = (2 * h <= e ? 2 * h : e) - h;
            FHE_TRY(mul_relin_pre2_impl(c, rlk, T + (h - 1) * tb, gc, T, Pw + h * bw, nk * gc, mws, st));
            const size_t keep = h + nk <= hmax ? nk : (h < hmax ? hmax - h : 0);
            if (keep) {
                const uint64_t *np = Pw + h * bw;
                uint64_t *nt = T + h * tb;
                FHE_TRY(run(c, KK_LIFT, st, [&] { return launch_lift(d, np, np, nt, 2, keep * gc, st); }));
                FHE_TRY(run(c, KK_FWD_EXT, st, [&] { return launch_fwd_ext(d, np, np, nt, 2, keep * gc, st); }));
            }
        }
        FHE_TRY(run(c, KK_ELEMENTWISE, st, [&] {
            return launch_weighted_sum_items(c->dev, Pw, bw, ctw, c->t, 1, wd, nbits, bits + g0 * nbits * ctw, ctw,
                                             nbits * ctw, gc, st);
        }));
    }
    return FHE_OK;
}

// ---------------------------------------------------------- signed casts ----

fhe_status fhe_int_to_mod(fhe_ctx *c, const uint64_t *bits, uint32_t nbits, uint64_t *out, size_t count,
                          hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (nbits == 0) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!bits || !out) return FHE_EINVAL;
    if (overlaps2(out, count * ct_words(c) * 8, bits, count * nbits * ct_words(c) * 8)) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, bits, count * nbits * 2 * c->k, c->k, 0, st));
    return run(c, KK_ELEMENTWISE, st,
               [&] { return launch_horner(c->dev, bits, (int)nbits, out, count, 1, st); });
}

// In place on bits [count][nbits] (least significant first): the unsigned
// value X becomes the signed bits Y of the paper's SecureMod -> SecureInt
// equation (constant 2^nbits - t added by a ripple-carry adder of the gates,
// then a MUX on the leading bit).  Bit i is read (gathered) before it is
// overwritten, and the leading bit is gathered first.
static fhe_status signed_bits_impl(fhe_ctx *c, const uint64_t *rlk, uint64_t *bits, uint32_t nbits,
                                   size_t count, void *ws, hipStream_t st) {
    const size_t ctw = ct_words(c), cw = count * ctw, ctb = ctw * 8;
    uint64_t *Msb = (uint64_t *)ws, *Xi = Msb + cw, *Ca = Xi + cw, *Pp = Ca + cw, *O = Pp + cw, *Ai = O + cw,
             *T = Ai + cw;
    void *mws = T + cw;
    const uint64_t cst = (1ull << nbits) - c->t;
    FHE_TRY(gather_bit(c, bits, nbits, nbits - 1, Msb, count, st));
    bool have_carry = false;
    for (uint32_t i = 0; i < nbits; i++) {
        FHE_TRY(gather_bit(c, bits, nbits, i, Xi, count, st));
        const bool ci = (cst >> i) & 1;
        if (!have_carry) {
            if (ci) {
                FHE_TRY(one_minus(c, Xi, Ai, count, st));
                FHE_HIP(hipMemcpyAsync(Ca, Xi, cw * 8, hipMemcpyDeviceToDevice, st));
                have_carry = true;
            } else {
                FHE_HIP(hipMemcpyAsync(Ai, Xi, cw * 8, hipMemcpyDeviceToDevice, st));
            }
        } else {
            FHE_TRY(mul_relin_impl(c, rlk, Xi, Ca, Pp, count, mws, st));  // p = X_i carry
            FHE_TRY(ew(c, Xi, Ca, O, count, 0, st));                       // OR
            FHE_TRY(ew(c, O, Pp, O, count, 1, st));
            FHE_TRY(ew(c, O, Pp, Ai, count, 1, st));                       // XOR
            if (ci) {
                FHE_TRY(one_minus(c, Ai, Ai, count, st));  // XNOR, carry = OR
                uint64_t *t = Ca;
                Ca = O;
                O = t;
            } else {  // carry = AND
                uint64_t *t = Ca;
                Ca = Pp;
                Pp = t;
            }
        }
        // Y_i = MSB (A_i - X_i) + X_i
        FHE_TRY(ew(c, Ai, Xi, T, count, 1, st));
        FHE_TRY(mul_relin_impl(c, rlk, Msb, T, T, count, mws, st));
        FHE_TRY(ew(c, T, Xi, T, count, 0, st));
        FHE_HIP(hipMemcpy2DAsync(bits + (size_t)i * ctw, nbits * ctb, T, ctb, ctb, count, hipMemcpyDeviceToDevice,
                                 st));
    }
    return FHE_OK;
}

fhe_status fhe_mod_to_int(fhe_ctx *c, const uint64_t *rlk, const uint64_t *x, uint32_t nbits, uint64_t *bits,
                          size_t count, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!ws) return FHE_EINVAL;
    if (ws_bytes < fhe_workspace_bytes(c, FHE_OP_MOD_TO_INT, count)) return FHE_EWORKSPACE;
    FHE_TRY(fhe_bridge_to_bits(c, rlk, x, nbits, bits, nullptr, count, ws, ws_bytes, st));
    return signed_bits_impl(c, rlk, bits, nbits, count, ws, st);
}

fhe_status fhe_ntt(fhe_ctx *c, int inverse, uint64_t *polys, size_t count, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (count == 0) return FHE_OK;
    if (!polys) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, polys, count * c->k, c->k, 0, st));
    return run(c, KK_NTT_ROWS, st, [&] {
        return launch_ntt_rows(c->dev, polys, count * c->k, c->k, 0, inverse ? NTT_INV : NTT_FWD, st);
    });
}

// ---------------------------------------------------------------- timing ----

// Operand table of the matrix-core first pass, per Q limb l: the pass's
// 16 x 16 matrix M (the four butterfly levels applied to unit vectors, with
// the transform's twiddles psi^bitrev(2^u + v)), then the A operands
// W[h][v][lane][16 bytes] = 7-bit limb v of M[j][e] 2^(7u) 2^64 mod q for
// j = lane % 16 and byte r: e = 4 (lane / 16) + 2h + r / 8, u = r % 8.
static fhe_status ensure_pass0_tables(fhe_ctx *c) {
    if (c->d_p0w) return FHE_OK;
    const uint32_t k = c->k, n = c->n, L = c->L;
    std::vector<uint8_t> W((size_t)k * 16 * 64 * 16);
    for (uint32_t l = 0; l < k; l++) {
        const uint64_t q = c->primes[l], psi = find_psi(q, n);
        uint64_t M[16][16];
        for (int col = 0; col < 16; col++) {
            uint64_t vec[16] = {};
            vec[col] = 1;
            for (int u = 0; u < 4; u++) {
                const int half = 16 >> (u + 1);
                for (int v = 0; v < (1 << u); v++) {
                    const uint64_t w = hpow(psi, bitrev((1u << u) + v, (int)L), q);
                    for (int wi = 0; wi < half; wi++) {
                        const int e0 = (v << (4 - u)) | wi;
                        const uint64_t X = vec[e0], t = hmul(w, vec[e0 + half], q);
                        vec[e0] = (X + t) % q;
                        vec[e0 + half] = (X + q - t) % q;
                    }
                }
            }
            for (int j = 0; j < 16; j++) M[j][col] = vec[j];
        }
        const uint64_t r64 = (uint64_t)(((u128)1 << 64) % q);
        for (int h = 0; h < 2; h++)
            for (int v = 0; v < 8; v++)
                for (int lane = 0; lane < 64; lane++)
                    for (int r = 0; r < 16; r++) {
                        const int j = lane % 16, e = 4 * (lane / 16) + 2 * h + r / 8, u = r % 8;
                        const uint64_t val = hmul(hmul(M[j][e], hpow(2, 7 * u, q), q), r64, q);
                        W[(((size_t)l * 16 + h * 8 + v) * 64 + lane) * 16 + r] = (uint8_t)((val >> (7 * v)) & 127);
                    }
    }
    FHE_HIP(hipSetDevice(c->device));
    fhe_status st = alloc_copy(&c->d_p0w, W.data(), W.size());
    if (st != FHE_OK) c->d_p0w = nullptr;
    return st;
}

fhe_status fhe_ntt_pass0(fhe_ctx *c, int method, uint32_t reps, uint64_t *polys, size_t count, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (method != 0 && method != 1) return FHE_EINVAL;
    if (reps == 0 || reps > 1024) return FHE_EINVAL;
    if (c->n < 1024) return FHE_EUNSUPPORTED;
    // 8 limbs of 7 bits hold residues below 2^56; primes below 2^55 keep the
    // recombined sum below 33 * 2^64 < q 2^64 (one Montgomery reduction)
    if (method == 1)
        for (uint32_t i = 0; i < c->k; i++)
            if (c->primes[i] >= (1ull << 55)) return FHE_EUNSUPPORTED;
    if (count == 0) return FHE_OK;
    if (!polys) return FHE_EINVAL;
    FHE_TRY(check_canonical(c, polys, count * c->k, c->k, 0, st));
    if (method == 1) FHE_TRY(ensure_pass0_tables(c));
    return run(c, method ? KK_PASS0_MFMA : KK_PASS0_VALU, st, [&] {
        return launch_pass0(c->dev, method, c->d_p0w, polys, count * c->k, c->k, 0, (int)reps, st);
    });
}

fhe_status fhe_set_timing(fhe_ctx *c, int enable) {
    if (!c) return FHE_EINVAL;
    c->timing = enable != 0;
    return FHE_OK;
}

int fhe_kernel_kinds(void) { return KK_COUNT; }

const char *fhe_kernel_name(int kind) {
    return (kind >= 0 && kind < KK_COUNT) ? kKernelNames[kind] : "unknown";
}

fhe_status fhe_kernel_stats(fhe_ctx *c, int kind, double *total_ms, uint64_t *launches) {
    if (!c || kind < 0 || kind >= KK_COUNT || !total_ms || !launches) return FHE_EINVAL;
    for (auto &ev : c->pending[kind]) {
        if (hipEventSynchronize(ev.b) != hipSuccess) return FHE_EDEVICE;
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return FHE_EDEVICE;
        c->total_ms[kind] += ms;
        c->free_events.push_back(ev.a);
        c->free_events.push_back(ev.b);
    }
    c->pending[kind].clear();
    *total_ms = c->total_ms[kind];
    *launches = c->launches[kind];
    return FHE_OK;
}

fhe_status fhe_reset_kernel_stats(fhe_ctx *c) {
    if (!c) return FHE_EINVAL;
    for (int i = 0; i < KK_COUNT; i++) {
        double ms;
        uint64_t l;
        fhe_status s = fhe_kernel_stats(c, i, &ms, &l);
        if (s != FHE_OK) return s;
        c->total_ms[i] = 0;
        c->launches[i] = 0;
    }
    return FHE_OK;
}

fhe_status fhe_sync(fhe_ctx *c, hipStream_t st) {
    if (!c) return FHE_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return FHE_EDEVICE;
    const hipError_t e = hipStreamSynchronize(st);
    const hipError_t l = hipGetLastError();
    return (e == hipSuccess && l == hipSuccess) ? FHE_OK : FHE_EDEVICE;
}

fhe_status fhe_fallback_count(fhe_ctx *c, uint64_t *count) {
    if (!c || !count) return FHE_EINVAL;
    FHE_HIP(hipDeviceSynchronize());
    FHE_HIP(hipMemcpy(count, c->d_counters, 8, hipMemcpyDeviceToHost));
    return FHE_OK;
}

}  // extern "C"
