// C ABI of the e-ph collision-integral library (declared in include/ephbte.h).
//
// A plan owns the device copy of the channel layout and every workspace the
// drivers need.  Entry points validate their arguments before enqueuing any
// work, run on the caller's stream and report failures through a status code
// plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ephbte.h"
#include "kernels.hpp"
#include "layout.hpp"

namespace ephbte {

static thread_local std::string g_last_error;

static ephbte_status fail(ephbte_status s, const std::string &m) {
    g_last_error = m;
    return s;
}

struct HipError {
    hipError_t e;
    const char *where;
};

static void hip_check(hipError_t e, const char *where) {
    if (e != hipSuccess) throw HipError{e, where};
}
#define HIPC(x) hip_check((x), #x)

// Scratch of the allocation-free forward pass (ephbte_collision_integral_noalloc):
// the call's {hw, N} table, the per-chunk partial sums of the rows.  One copy
// per GPU, held until the process ends and shared by every such call on that
// GPU.  Host code never uses the array's name as an address: its device
// address is looked up once per device (scratch_base) and kept.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_base[kMaxDevices] = {};

static constexpr double kHbar = 0.6582119569;     // eV fs
static constexpr double kKb = 8.617333262e-5;     // eV / K
static constexpr double kPi = 3.14159265358979323846;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct GraphEntry {
    const void *f, *nph;
    int64_t ldf;
    int B, steps;
    double dt;
    hipStream_t stream;
    int64_t ws_gen;
    hipGraphExec_t exec;
};

}  // namespace ephbte

using namespace ephbte;

struct ephbte_plan_s {
    int device = 0;
    int dtype = EPHBTE_F64;
    int S = 0, nm = 0;
    int64_t nch = 0, E = 0;          // channels passed at build; entries of the kept channels
    int64_t nch_kept = 0;
    int32_t *drop_idx = nullptr;     // [n_drop] caller indices removed by the channel selection
    int64_t n_drop = 0;
    // field term of Eq. 1: neighbour table (device, [S][3][2]) and rates (1/fs)
    int32_t *nbr = nullptr;
    bool nbr_ok = false;
    double drift_rate[3] = {0.0, 0.0, 0.0};
    bool drift_on = false;
    // phonon side: elastic-mode mask, full k-grid count, and the channels
    // grouped by phonon pair {q, -q} (pair records, buckets, chunks)
    uint32_t elastic = 0;
    double nk = 1.0;
    // Bose statistics (ephbte_build_opts.statistics = 1): the entry points
    // map n to f = -n for the kernels (see boson_neg); max |f| of each pass's
    // input sets the fixed-point scale
    bool boson = false;
    unsigned long long *fmax_bits = nullptr;
    uint32_t *ph_pa = nullptr, *ph_pb = nullptr;
    void *ph_g2 = nullptr;            // [n_modes][ph_ld]
    int32_t *ph_chan = nullptr;       // [n_modes][ph_ld] caller channel of each slot, -1: none
    int64_t ph_np = 0, ph_ld = 0, ph_nchunks = 0, ph_nbuckets = 0;
    int64_t *ph_chunk_beg = nullptr;
    int32_t *ph_chunk_bucket = nullptr, *ph_bucket_chunk = nullptr, *ph_bucket_q = nullptr,
            *ph_bucket_qm = nullptr, *ph_q_bucket = nullptr;
    uint32_t *ph_bucket_modes = nullptr;
    int nq[3] = {0, 0, 0};
    double sigma = 0, nqnorm = 0;
    std::vector<int64_t> row_ptr;   // host copy for re-chunking
    std::vector<int32_t> pmin, pmax; // host: partner range of each destination
    int n_cu = 256;
    // layout (device)
    uint32_t *pnu = nullptr;
    void *g2 = nullptr;
    void *st = nullptr;
    void *hw = nullptr;
    int32_t *ent_chan = nullptr;
    double *e2tab = nullptr;        // 2^(j/256), j = 0 .. 255
    // chunks (device)
    int64_t *chunk_beg = nullptr;
    int32_t *chunk_dest = nullptr;
    int32_t *dest_chunk = nullptr;
    int64_t n_chunks = 0;
    TileRec *tiles = nullptr;
    int64_t n_tiles = 0;
    TileRec *small_tiles = nullptr;   // half-size tiles over the same chunks (reverse pass, transport)
    int64_t n_small_tiles = 0;
    // single-copy pass: chunks over the upper part (p > d) of each row
    int64_t *sym_chunk_beg = nullptr, *sym_chunk_end = nullptr;
    int32_t *sym_chunk_dest = nullptr, *sym_dest_chunk = nullptr;
    TileRec *sym_tiles = nullptr;
    int64_t n_sym_chunks = 0, n_sym_tiles = 0;
    std::vector<int64_t> upper_beg;        // host: first entry of row d with p > d
    std::vector<int32_t> pmin_up, pmax_up;  // host: partner range of that part
    unsigned long long *jacc = nullptr;     // [S] partner-side fixed-point sums (zero between calls)
    unsigned long long *nmax_bits = nullptr, *gmax_bits = nullptr;
    double *pack_bmax = nullptr;            // per-block max |N| of the last pack
    int sym_lds_states = 0;
    int pr_lds_states = 0;      // partner window of the pair-record passes
    int pr_threads = 1024;      // threads per workgroup of the pair forward pass
    int pair_order = 1;         // records of the LDS tiles: 1 q order, 2 destination order
    int pair_shift = 0;         // q order by table row >> pair_shift
    bool sym_ok = false;                    // the single-copy window fits the LDS of a workgroup
    int layout = 2;                         // B = 1 forward: 1 duplicated rows, 2 single copy,
                                            // 3 single copy over pair records
    // pair records of the single-copy pass (built when most of their mode
    // slots hold a channel): partners, |g|^2 slots [n_modes][pr_ld], the
    // caller channel of each slot, and their chunks and tiles
    uint32_t *pr_partner = nullptr;
    void *pr_g2 = nullptr;
    int32_t *pr_chan = nullptr;
    int32_t *pr_ch0 = nullptr;             // first channel of a record whose slots are consecutive, else -1
    int64_t pr_np = 0, pr_ld = 0;
    std::vector<int64_t> pr_rowptr;        // host: pair rows, for re-chunking
    std::vector<uint32_t> pr_partner_host; // host: partner of each record, destination order
    std::vector<uint32_t> pr_perm;         // host: device position -> record in destination
                                           // order (empty: the same order)
    std::vector<uint32_t> st_key;          // host: packed box (padded table) or grid coordinates
    std::array<int64_t, 6> pr_key{};       // settings the pair tiles were built with
    bool pr_key_set = false;
    bool pr_all_q = false;                 // every pair tile is q-ordered
    int64_t *pr_chunk_beg = nullptr, *pr_chunk_end = nullptr;
    int32_t *pr_chunk_dest = nullptr, *pr_dest_chunk = nullptr;
    TileRec *pr_tiles = nullptr;
    int64_t n_pr_chunks = 0, n_pr_tiles = 0;
    bool pr_ok = false;
    bool exp_table = true;                 // FP64 Gaussians of the pair pass from the LDS table
    unsigned long long *lmax_bits = nullptr;  // max |lam| of the pair reverse pass (double bits)
    unsigned long long *mmax_bits = nullptr;  // max |mu| and max |N| of the phonon side's dL/df over
                                              // pair records (its own slots: other passes keep theirs)
    // batched pass: tiles of destinations and per-destination sub-tile offsets
    BTileRec *btiles = nullptr;
    int64_t *sub_off = nullptr;
    int64_t n_btiles = 0;
    int pt = 0;                 // partners per sub-tile
    // batched reverse pass: its own tiles (twice the LDS per partner), built on first use
    BTileRec *vbtiles = nullptr;
    int64_t *vsub_off = nullptr;
    int64_t n_vbtiles = 0;
    int vpt = 0;
    int batch_min = 8;          // smallest B that uses the batched kernels
    int lds_states = 0;
    size_t lds_max = 65536;      // device limit of LDS per workgroup
    bool fused = true;
    // phonon table indexed by padded k differences (one subtraction per entry)
    bool padq = false;
    int qoff = 0;
    int64_t qpad_n = 0;         // rows of the box table (QBox)
    QBox qbox{};
    uint32_t qorg[3] = {0, 0, 0};   // per-axis origin of the shifted k coordinates
    // box rows some entry references (ascending); the packs write only these,
    // the others stay zero from the table's allocation
    int32_t *used_rows = nullptr;
    int64_t n_used_rows = 0;
    bool tab_mm = false;        // box table stored one block per mode
    int chunk_entries = 0;
    int64_t tile_entries = 0;   // 0: default target per tile
    int block_threads = 256;
    bool xcd_map = true;
    // workspaces, grown on demand
    DevBuf part, sym_part, rk_ua, rk_ub, rk_acc, hwN;
    DevBuf tr_W, tr_tau_inv, tr_tau, tr_rhs, tr_xa, tr_xb, tr_part, tr_red, tr_red2;
    DevBuf adj_ck, adj_U, adj_la, adj_lb, adj_acc, adj_g, adj_f;
    DevBuf cp_Ma, cp_Mb, cp_acc, cp_rate;   // coupled step: phonon stages, sum, rate
    DevBuf ph_part;                          // phonon pass: chunk partials
    DevBuf ph_tab4;                          // {hw, N, mu} table of the phonon-side reverse pass
    // reverse of the coupled step: checkpoints and stage inputs of (f, N),
    // adjoint vectors of both
    DevBuf ca_ckf, ca_ckN, ca_U, ca_M, ca_gf, ca_gN, ca_a, ca_b, ca_uf, ca_uN, ca_sf, ca_sN, ca_mu;
    DevBuf bs_x, bs_y;                       // Bose plans: negated inputs
    DevBuf nvec;                             // per-vector baths of the batched pass
    double *host_red = nullptr;   // pinned
    hipStream_t own_stream = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    // work of consecutive calls is ordered even across streams: the plan's
    // workspaces are shared by every call
    hipEvent_t ev_last = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    std::vector<GraphEntry> graphs;
    // launch timing of the forward pass's main kernel (ephbte_kernel_timing):
    // a pair of events per eager launch, recorded on its stream, reused
    bool ktime_on = false;
    std::vector<hipEvent_t> ktime_ev;
    size_t ktime_used = 0;
    int64_t ws_gen = 0;   // bumped whenever a workspace moves
    size_t layout_bytes = 0;

    size_t bytes() const {
        size_t b = layout_bytes;
        const DevBuf *w[] = {&part,  &sym_part, &rk_ua, &rk_ub, &rk_acc, &hwN, &tr_W,  &tr_tau_inv, &tr_tau,
                             &tr_rhs, &tr_xa, &tr_xb, &tr_part, &tr_red, &tr_red2, &adj_ck,
                             &adj_U, &adj_la, &adj_lb, &adj_acc, &adj_g, &adj_f, &cp_Ma, &cp_Mb,
                             &cp_acc, &cp_rate, &ph_part, &ph_tab4, &ca_ckf, &ca_ckN, &ca_U, &ca_M,
                             &ca_gf, &ca_gN, &ca_a, &ca_b, &ca_uf, &ca_uN, &ca_sf, &ca_sN, &ca_mu,
                             &bs_x, &bs_y, &nvec};
        for (auto *x : w) b += x->bytes;
        return b;
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) HIPC(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void dfree(void *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename P> void dalloc(P *&p, size_t bytes, size_t *acc) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    p = static_cast<P *>(q);
    if (acc) *acc += bytes;
}

// Grows a workspace; every reallocation bumps *gen so that HIP graphs that
// captured the old address are re-captured.
void ensure(DevBuf &b, size_t bytes, int64_t *gen) {
    if (b.bytes >= bytes && b.p) return;
    ++*gen;
    dfree(b.p);
    b.bytes = 0;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    b.p = q;
    b.bytes = bytes;
}

// ensure() for tables whose packs write only the referenced rows: a new
// allocation is cleared once (finite zeros where masked lanes may read)
void ensure_zeroed(ephbte_plan P, DevBuf &b, size_t bytes) {
    const int64_t gen = P->ws_gen;
    ensure(b, bytes, &P->ws_gen);
    if (P->ws_gen != gen) {
        HIPC(hipMemset(b.p, 0, b.bytes));
        HIPC(hipDeviceSynchronize());
    }
}

// Device address of `scratch` on device dev (which must be current), looked
// up on the first call for that device and kept.
void *scratch_base(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw HipError{hipErrorInvalidDevice, "scratch_base"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_base[dev]) {
        void *ptr = nullptr;
        HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
        g_scratch_base[dev] = ptr;
    }
    return g_scratch_base[dev];
}

void free_graphs(ephbte_plan P) {
    for (auto &g : P->graphs) (void)hipGraphExecDestroy(g.exec);
    P->graphs.clear();
}

void free_plan(ephbte_plan P) {
    if (!P) return;
    (void)hipSetDevice(P->device);
    free_graphs(P);
    void **ptrs[] = {(void **)&P->pnu,       (void **)&P->g2,         (void **)&P->st,
                     (void **)&P->hw,        (void **)&P->ent_chan,   (void **)&P->chunk_beg,
                     (void **)&P->chunk_dest, (void **)&P->dest_chunk, (void **)&P->tiles,
                     (void **)&P->btiles,    (void **)&P->sub_off,    (void **)&P->e2tab,
                     (void **)&P->sym_chunk_beg, (void **)&P->sym_chunk_end, (void **)&P->sym_chunk_dest,
                     (void **)&P->sym_dest_chunk, (void **)&P->sym_tiles, (void **)&P->jacc,
                     (void **)&P->nmax_bits, (void **)&P->gmax_bits, (void **)&P->pack_bmax,
                     (void **)&P->drop_idx, (void **)&P->vbtiles, (void **)&P->vsub_off,
                     (void **)&P->nbr, (void **)&P->small_tiles, (void **)&P->ph_pa,
                     (void **)&P->ph_pb, (void **)&P->ph_g2, (void **)&P->ph_chan,
                     (void **)&P->ph_chunk_beg, (void **)&P->ph_chunk_bucket, (void **)&P->ph_bucket_chunk,
                     (void **)&P->ph_bucket_q, (void **)&P->ph_bucket_qm, (void **)&P->ph_q_bucket,
                     (void **)&P->ph_bucket_modes, (void **)&P->pr_partner, (void **)&P->pr_g2,
                     (void **)&P->pr_chan, (void **)&P->pr_chunk_beg, (void **)&P->pr_chunk_end,
                     (void **)&P->pr_chunk_dest, (void **)&P->pr_dest_chunk, (void **)&P->pr_tiles,
                     (void **)&P->lmax_bits, (void **)&P->mmax_bits, (void **)&P->pr_ch0, (void **)&P->fmax_bits,
                     (void **)&P->used_rows};
    for (auto pp : ptrs) dfree(*pp);
    DevBuf *w[] = {&P->part,   &P->sym_part, &P->rk_ua,  &P->rk_ub,   &P->rk_acc, &P->hwN, &P->tr_W,   &P->tr_tau_inv,
                   &P->tr_tau, &P->tr_rhs, &P->tr_xa,   &P->tr_xb,  &P->tr_part, &P->tr_red,
                   &P->tr_red2, &P->adj_ck, &P->adj_U,  &P->adj_la, &P->adj_lb, &P->adj_acc,
                   &P->adj_g,  &P->adj_f, &P->cp_Ma, &P->cp_Mb, &P->cp_acc, &P->cp_rate, &P->ph_part,
                   &P->ph_tab4, &P->ca_ckf, &P->ca_ckN, &P->ca_U, &P->ca_M, &P->ca_gf, &P->ca_gN, &P->ca_a,
                   &P->ca_b, &P->ca_uf, &P->ca_uN, &P->ca_sf, &P->ca_sN, &P->ca_mu, &P->bs_x, &P->bs_y, &P->nvec};
    for (auto *b : w) dfree(b->p);
    if (P->host_red) (void)hipHostFree(P->host_red);
    if (P->ev_a) (void)hipEventDestroy(P->ev_a);
    if (P->ev_b) (void)hipEventDestroy(P->ev_b);
    if (P->ev_last) (void)hipEventDestroy(P->ev_last);
    for (hipEvent_t e : P->ktime_ev) (void)hipEventDestroy(e);
    if (P->own_stream) (void)hipStreamDestroy(P->own_stream);
    delete P;
}

int64_t grid_x(ephbte_plan P) { return P->xcd_map ? 8 * ((P->n_chunks + 7) / 8) : P->n_chunks; }

// workgroups for n tiles (tile_of_block pads to a multiple of the 8 XCDs)
unsigned tile_grid(ephbte_plan P, int64_t n) {
    return static_cast<unsigned>(P->xcd_map ? 8 * ((n + 7) / 8) : n);
}

unsigned grid_of(int64_t n) {
    return static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((n + 255) / 256, 4096), 1));
}

// Puts the device's pair records in the order of order_pair_tiles (q order
// inside the LDS tiles when qord, else destination order) and replaces the
// chunk table and tiles by the renumbered ones.  The stream words are
// uploaded; the mode slots (|g|^2, channel) and first channels are gathered
// on the device from their current order.
void order_pair_records(ephbte_plan P, ChunkTable &pc, std::vector<Tile> &tp, bool qord) {
    const int64_t np = P->pr_np;
    RowKey rk;
    rk.key = P->st_key.data();
    rk.padq = P->padq;
    rk.qoff = P->qoff;
    rk.shift = P->pair_shift;
    for (int a = 0; a < 3; ++a) rk.n[a] = P->nq[a];
    PairOrder o;
    if (qord) {
        o = order_pair_tiles(pc, tp, P->pr_partner_host, rk, kPairChunksPerTile, 65536);
    } else {
        // destination order: the tiles and chunks as built
        o.chunks = pc;
        o.tiles = tp;
        o.perm.resize(static_cast<size_t>(np));
        for (int64_t x = 0; x < np; ++x) o.perm[x] = static_cast<uint32_t>(x);
        o.word = P->pr_partner_host;
    }
    // device gather indices: idx[i] = current device position of the record
    // that goes to position i
    std::vector<uint32_t> idx(static_cast<size_t>(np));
    bool same = true;
    if (P->pr_perm.empty()) {
        idx = o.perm;
    } else {
        std::vector<uint32_t> inv(static_cast<size_t>(np));
        for (int64_t x = 0; x < np; ++x) inv[P->pr_perm[x]] = static_cast<uint32_t>(x);
        for (int64_t x = 0; x < np; ++x) idx[x] = inv[o.perm[x]];
    }
    for (int64_t x = 0; x < np && same; ++x) same = idx[x] == static_cast<uint32_t>(x);
    if (!same) {
        const size_t ld = static_cast<size_t>(P->pr_ld), nm = static_cast<size_t>(P->nm);
        const size_t es = P->dtype == EPHBTE_F64 ? 8 : 4;
        uint32_t *d_idx = nullptr;
        void *g_new = nullptr;
        int32_t *c_new = nullptr, *c0_new = nullptr;
        size_t dummy = 0;
        dalloc(d_idx, sizeof(uint32_t) * static_cast<size_t>(np), &dummy);
        dalloc(g_new, es * ld * nm, &dummy);
        dalloc(c_new, sizeof(int32_t) * ld * nm, &dummy);
        dalloc(c0_new, sizeof(int32_t) * ld, &dummy);
        HIPC(hipMemcpy(d_idx, idx.data(), sizeof(uint32_t) * static_cast<size_t>(np), hipMemcpyHostToDevice));
        const dim3 grid(grid_of(static_cast<int64_t>(ld))), block(256);
        if (es == 8)
            hipLaunchKernelGGL((k_permute_pairs<double>), grid, block, 0, nullptr, (const uint32_t *)d_idx, np,
                               static_cast<int64_t>(ld), P->nm, (const double *)P->pr_g2, (double *)g_new,
                               (const int32_t *)P->pr_chan, c_new, (const int32_t *)P->pr_ch0, c0_new);
        else
            hipLaunchKernelGGL((k_permute_pairs<float>), grid, block, 0, nullptr, (const uint32_t *)d_idx, np,
                               static_cast<int64_t>(ld), P->nm, (const float *)P->pr_g2, (float *)g_new,
                               (const int32_t *)P->pr_chan, c_new, (const int32_t *)P->pr_ch0, c0_new);
        HIPC(hipGetLastError());
        HIPC(hipDeviceSynchronize());
        dfree(reinterpret_cast<void *&>(d_idx));
        dfree(P->pr_g2);
        dfree(reinterpret_cast<void *&>(P->pr_chan));
        dfree(reinterpret_cast<void *&>(P->pr_ch0));
        P->pr_g2 = g_new;
        P->pr_chan = c_new;
        P->pr_ch0 = c0_new;
    }
    {
        std::vector<uint32_t> w(static_cast<size_t>(P->pr_ld), 0u);
        std::copy(o.word.begin(), o.word.end(), w.begin());
        HIPC(hipMemcpy(P->pr_partner, w.data(), sizeof(uint32_t) * w.size(), hipMemcpyHostToDevice));
    }
    bool ident = true;
    for (int64_t x = 0; x < np && ident; ++x) ident = o.perm[x] == static_cast<uint32_t>(x);
    if (ident) P->pr_perm.clear();
    else P->pr_perm = std::move(o.perm);
    pc = std::move(o.chunks);
    tp = std::move(o.tiles);
}

void upload_chunks(ephbte_plan P, int64_t chunk_entries) {
    ChunkTable t = make_chunks(P->row_ptr, chunk_entries);
    free_graphs(P);
    dfree(reinterpret_cast<void *&>(P->chunk_beg));
    dfree(reinterpret_cast<void *&>(P->chunk_dest));
    dfree(reinterpret_cast<void *&>(P->dest_chunk));
    size_t dummy = 0;
    dalloc(P->chunk_beg, t.chunk_beg.size() * sizeof(int64_t), &dummy);
    dalloc(P->chunk_dest, t.chunk_dest.size() * sizeof(int32_t), &dummy);
    dalloc(P->dest_chunk, t.dest_chunk.size() * sizeof(int32_t), &dummy);
    HIPC(hipMemcpy(P->chunk_beg, t.chunk_beg.data(), t.chunk_beg.size() * sizeof(int64_t),
                   hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->chunk_dest, t.chunk_dest.data(), t.chunk_dest.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->dest_chunk, t.dest_chunk.data(), t.dest_chunk.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
    P->n_chunks = t.n_chunks;
    P->fused = t.one_per_dest;
    P->chunk_entries = static_cast<int>(std::min<int64_t>(chunk_entries, INT32_MAX));
    // tiles: by default about 6 per compute unit (3 per resident workgroup slot
    // at two workgroups per CU), measured best on the 100^3 system
    const int64_t target = P->tile_entries > 0
                               ? P->tile_entries
                               : P->E / (6 * static_cast<int64_t>(P->n_cu)) + 1;
    std::vector<Tile> tl = make_tiles(t, P->row_ptr, P->pmin, P->pmax, P->lds_states, target);
    static_assert(sizeof(Tile) == sizeof(TileRec), "tile record layout");
    dfree(reinterpret_cast<void *&>(P->tiles));
    dalloc(P->tiles, tl.size() * sizeof(TileRec), &dummy);
    HIPC(hipMemcpy(P->tiles, tl.data(), tl.size() * sizeof(TileRec), hipMemcpyHostToDevice));
    P->n_tiles = static_cast<int64_t>(tl.size());
    // the reverse pass does more work per entry; half-size tiles (about 12 per
    // CU) measured 4-5 % faster than the forward's on the 100^3 system
    const int64_t target_v = P->tile_entries > 0
                                 ? P->tile_entries
                                 : P->E / (12 * static_cast<int64_t>(P->n_cu)) + 1;
    std::vector<Tile> tv = make_tiles(t, P->row_ptr, P->pmin, P->pmax, P->lds_states, target_v);
    dfree(reinterpret_cast<void *&>(P->small_tiles));
    dalloc(P->small_tiles, std::max<size_t>(tv.size(), 1) * sizeof(TileRec), &dummy);
    if (!tv.empty())
        HIPC(hipMemcpy(P->small_tiles, tv.data(), tv.size() * sizeof(TileRec), hipMemcpyHostToDevice));
    P->n_small_tiles = static_cast<int64_t>(tv.size());
    if (P->upper_beg.empty()) return;
    // single-copy tables over the upper parts of the rows; one workgroup per CU
    // (1024 threads), about 4 tiles each (measured; smaller tiles pay more
    // window staging and partner-side flushes)
    std::vector<int64_t> row_end(P->row_ptr.begin() + 1, P->row_ptr.end());
    ChunkTable u = make_chunks_seg(P->upper_beg, row_end, chunk_entries);
    const int64_t nch = P->E / 2;
    const int64_t target_u = P->tile_entries > 0 ? P->tile_entries / 2 + 1
                                                 : nch / (4 * static_cast<int64_t>(P->n_cu)) + 1;
    std::vector<Tile> tu = make_tiles(u, P->row_ptr, P->pmin_up, P->pmax_up, P->sym_lds_states, target_u);
    dfree(reinterpret_cast<void *&>(P->sym_chunk_beg));
    dfree(reinterpret_cast<void *&>(P->sym_chunk_end));
    dfree(reinterpret_cast<void *&>(P->sym_chunk_dest));
    dfree(reinterpret_cast<void *&>(P->sym_dest_chunk));
    dfree(reinterpret_cast<void *&>(P->sym_tiles));
    dalloc(P->sym_chunk_beg, u.chunk_beg.size() * sizeof(int64_t), &dummy);
    dalloc(P->sym_chunk_end, std::max<size_t>(u.chunk_end.size(), 1) * sizeof(int64_t), &dummy);
    dalloc(P->sym_chunk_dest, std::max<size_t>(u.chunk_dest.size(), 1) * sizeof(int32_t), &dummy);
    dalloc(P->sym_dest_chunk, u.dest_chunk.size() * sizeof(int32_t), &dummy);
    dalloc(P->sym_tiles, std::max<size_t>(tu.size(), 1) * sizeof(TileRec), &dummy);
    HIPC(hipMemcpy(P->sym_chunk_beg, u.chunk_beg.data(), u.chunk_beg.size() * sizeof(int64_t),
                   hipMemcpyHostToDevice));
    if (!u.chunk_end.empty()) {
        HIPC(hipMemcpy(P->sym_chunk_end, u.chunk_end.data(), u.chunk_end.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->sym_chunk_dest, u.chunk_dest.data(), u.chunk_dest.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
    }
    HIPC(hipMemcpy(P->sym_dest_chunk, u.dest_chunk.data(), u.dest_chunk.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
    if (!tu.empty())
        HIPC(hipMemcpy(P->sym_tiles, tu.data(), tu.size() * sizeof(TileRec), hipMemcpyHostToDevice));
    P->n_sym_chunks = u.n_chunks;
    P->n_sym_tiles = static_cast<int64_t>(tu.size());
    if (!P->pr_ok) return;
    // pair records: the same split, counted in pairs (a pair carries all modes).
    // Their tiling (and order) depends only on these settings: a tuning change
    // that leaves them as they are keeps the records where they are.
    const std::array<int64_t, 6> pr_key = {chunk_entries, P->tile_entries, P->pr_lds_states, P->pair_order,
                                           P->pair_shift, P->n_cu};
    if (P->pr_key_set && P->pr_key == pr_key) return;
    std::vector<int64_t> pbeg(P->pr_rowptr.begin(), P->pr_rowptr.end() - 1);
    std::vector<int64_t> pend(P->pr_rowptr.begin() + 1, P->pr_rowptr.end());
    ChunkTable pc = make_chunks_seg(pbeg, pend, chunk_entries);
    const int64_t target_p = P->tile_entries > 0 ? P->tile_entries / (2 * static_cast<int64_t>(P->nm)) + 1
                                                 : P->pr_np / (4 * static_cast<int64_t>(P->n_cu)) + 1;
    // in q order, a tile's window stages its destinations too
    const bool qord = P->pair_order == 1 && P->pr_np < (int64_t(1) << 32);
    std::vector<int32_t> wmin;
    if (qord) {
        wmin = P->pmin_up;
        for (int64_t d = 0; d < P->S; ++d)
            if (P->pmax_up[d] >= P->pmin_up[d]) wmin[d] = static_cast<int32_t>(d);
    }
    std::vector<Tile> tp = make_tiles(pc, P->row_ptr, qord ? wmin : P->pmin_up, P->pmax_up, P->pr_lds_states,
                                      target_p);
    order_pair_records(P, pc, tp, qord);
    dfree(reinterpret_cast<void *&>(P->pr_chunk_beg));
    dfree(reinterpret_cast<void *&>(P->pr_chunk_end));
    dfree(reinterpret_cast<void *&>(P->pr_chunk_dest));
    dfree(reinterpret_cast<void *&>(P->pr_dest_chunk));
    dfree(reinterpret_cast<void *&>(P->pr_tiles));
    dalloc(P->pr_chunk_beg, pc.chunk_beg.size() * sizeof(int64_t), &dummy);
    dalloc(P->pr_chunk_end, std::max<size_t>(pc.chunk_end.size(), 1) * sizeof(int64_t), &dummy);
    dalloc(P->pr_chunk_dest, std::max<size_t>(pc.chunk_dest.size(), 1) * sizeof(int32_t), &dummy);
    dalloc(P->pr_dest_chunk, pc.dest_chunk.size() * sizeof(int32_t), &dummy);
    dalloc(P->pr_tiles, std::max<size_t>(tp.size(), 1) * sizeof(TileRec), &dummy);
    HIPC(hipMemcpy(P->pr_chunk_beg, pc.chunk_beg.data(), pc.chunk_beg.size() * sizeof(int64_t),
                   hipMemcpyHostToDevice));
    if (!pc.chunk_end.empty()) {
        HIPC(hipMemcpy(P->pr_chunk_end, pc.chunk_end.data(), pc.chunk_end.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->pr_chunk_dest, pc.chunk_dest.data(), pc.chunk_dest.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
    }
    HIPC(hipMemcpy(P->pr_dest_chunk, pc.dest_chunk.data(), pc.dest_chunk.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice));
    if (!tp.empty())
        HIPC(hipMemcpy(P->pr_tiles, tp.data(), tp.size() * sizeof(TileRec), hipMemcpyHostToDevice));
    P->n_pr_chunks = pc.n_chunks;
    P->n_pr_tiles = static_cast<int64_t>(tp.size());
    P->pr_key = pr_key;
    P->pr_key_set = true;
    P->pr_all_q = !tp.empty();
    for (const Tile &t : tp) P->pr_all_q = P->pr_all_q && t.lds == 2;
}

// element (q, mode) of the plan's {hw, N} table is at q tq + mode tm
void table_strides(ephbte_plan P, int64_t *tq, int64_t *tm) {
    const bool mm = P->padq && P->tab_mm;
    *tq = mm ? 1 : P->nm;
    *tm = mm ? P->qpad_n : 1;
}

template <typename T> Tables<T> tables(ephbte_plan P, const void *nph) {
    Tables<T> t;
    t.pnu = P->pnu;
    t.g2 = static_cast<const T *>(P->g2);
    t.st = static_cast<const StateRec<T> *>(P->st);
    t.hw = static_cast<const T *>(P->hw);
    t.nph = static_cast<const T *>(nph);
    t.chunk_beg = P->chunk_beg;
    t.chunk_dest = P->chunk_dest;
    t.dest_chunk = P->dest_chunk;
    t.ent_chan = P->ent_chan;
    t.n_chunks = P->n_chunks;
    t.xcd_m = P->xcd_map ? (P->n_chunks + 7) / 8 : 0;
    t.S = P->S;
    t.nm = P->nm;
    t.nq0 = P->nq[0];
    t.nq1 = P->nq[1];
    t.nq2 = P->nq[2];
    const double s = P->sigma;
    // both precisions evaluate the Gaussian as 2^(x^2 mc)
    t.mc = static_cast<T>(-1.4426950408889634 / (2.0 * s * s));
    t.K = static_cast<T>(2.0 * kPi / (kHbar * P->nqnorm) / (s * std::sqrt(2.0 * kPi)));
    return t;
}

template <typename T> TiledArgs<T> tiled_args(ephbte_plan P) {
    TiledArgs<T> a;
    a.pnu = P->pnu;
    a.g2 = static_cast<const T *>(P->g2);
    a.st = static_cast<const StateRec<T> *>(P->st);
    a.hwN = static_cast<const Pair2<T> *>(P->hwN.p);
    table_strides(P, &a.tq, &a.tm);
    a.chunk_beg = P->chunk_beg;
    a.chunk_dest = P->chunk_dest;
    a.dest_chunk = P->dest_chunk;
    a.tiles = P->tiles;
    a.n_chunks = P->n_chunks;
    a.S = P->S;
    a.nm = P->nm;
    a.nq0 = P->nq[0];
    a.nq1 = P->nq[1];
    a.nq2 = P->nq[2];
    a.lds_states = P->lds_states;
    a.padq = P->padq ? 1 : 0;
    a.qoff = P->qoff;
    Tables<T> t = tables<T>(P, nullptr);
    a.mc = t.mc;
    a.K = t.K;
    a.e2tab = P->e2tab;
    a.mc256 = 256.0 * (-1.4426950408889634 / (2.0 * P->sigma * P->sigma));
    a.n_tiles = P->n_tiles;
    a.xcd = P->xcd_map ? 1 : 0;
    a.chunk_end = nullptr;
    a.jacc = P->jacc;
    a.nmax_bits = P->nmax_bits;
    a.gmax_bits = P->gmax_bits;
    a.fmax_bits = P->boson ? P->fmax_bits : nullptr;
    return a;
}

// arguments of the single-copy pass: its own chunks, tiles and LDS window
template <typename T> TiledArgs<T> sym_args(ephbte_plan P) {
    TiledArgs<T> a = tiled_args<T>(P);
    a.chunk_beg = P->sym_chunk_beg;
    a.chunk_end = P->sym_chunk_end;
    a.chunk_dest = P->sym_chunk_dest;
    a.dest_chunk = P->sym_dest_chunk;
    a.tiles = P->sym_tiles;
    a.n_chunks = P->n_sym_chunks;
    a.n_tiles = P->n_sym_tiles;
    a.lds_states = P->sym_lds_states;
    a.xcd = 0;   // measured: plain tile order is faster for this pass
    return a;
}

// arguments of the single-copy pass over pair records
template <typename T> TiledArgs<T> pair_args(ephbte_plan P) {
    TiledArgs<T> a = sym_args<T>(P);
    a.lds_states = P->pr_lds_states;
    a.pnu = P->pr_partner;
    a.g2 = static_cast<const T *>(P->pr_g2);
    a.pld = P->pr_ld;
    a.chunk_beg = P->pr_chunk_beg;
    a.chunk_end = P->pr_chunk_end;
    a.chunk_dest = P->pr_chunk_dest;
    a.dest_chunk = P->pr_dest_chunk;
    a.tiles = P->pr_tiles;
    a.n_chunks = P->n_pr_chunks;
    a.n_tiles = P->n_pr_tiles;
    return a;
}

// LDS of the single-copy pass: fixed-point sums, {eps, f}, packed k per window
// state, and the FP64 exponential table
size_t sym_lds_bytes(int dtype, int states) {
    const size_t es = dtype == EPHBTE_F64 ? 8 : 4;
    const size_t tab = dtype == EPHBTE_F64 ? kExpTab * sizeof(double) : 0;
    return static_cast<size_t>(states) * (8 + 2 * es + 4) + tab;
}

// LDS of the pair reverse pass: the forward's plus lam per window state
size_t vjp_pair_lds_bytes(int dtype, int states) {
    const size_t es = dtype == EPHBTE_F64 ? 8 : 4;
    return sym_lds_bytes(dtype, states) + static_cast<size_t>(states) * es;
}

// max over states of the sum of |g|^2 of the state's channels (device scalar)
void update_gmax(ephbte_plan P, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, P->gmax_bits, 1);
    if (P->S == 0) return;
    const unsigned blocks = static_cast<unsigned>((static_cast<int64_t>(P->S) * 64 + 255) / 256);
    if (P->dtype == EPHBTE_F64)
        hipLaunchKernelGGL((k_row_gmax<double>), dim3(blocks), dim3(256), 0, s,
                           static_cast<const double *>(P->g2), P->chunk_beg, P->dest_chunk, P->S, P->gmax_bits);
    else
        hipLaunchKernelGGL((k_row_gmax<float>), dim3(blocks), dim3(256), 0, s,
                           static_cast<const float *>(P->g2), P->chunk_beg, P->dest_chunk, P->S, P->gmax_bits);
    HIPC(hipGetLastError());
}

bool use_sym(ephbte_plan P, int B) {
    return B == 1 && P->layout == 2 && P->sym_ok && P->n_sym_tiles > 0;
}

// k_fwd_pairs with its mode-slot count rounded up to 1, 2, 3, 4, 6 or 8
template <typename T>
void launch_pairs(ephbte_plan P, const TiledArgs<T> &a, const T *f, T *part, size_t shm, hipStream_t s,
                  bool padq) {
    const dim3 grid(static_cast<unsigned>(P->n_pr_tiles)), block(static_cast<unsigned>(P->pr_threads));
    auto go = [&](auto nmc) {
        constexpr int NM = decltype(nmc)::value;
        const bool tab = sizeof(T) == 8 && P->exp_table;
        if (padq && tab) hipLaunchKernelGGL((k_fwd_pairs<T, true, NM, true>), grid, block, shm, s, a, f, part);
        else if (padq) hipLaunchKernelGGL((k_fwd_pairs<T, true, NM, false>), grid, block, shm, s, a, f, part);
        else if (tab) hipLaunchKernelGGL((k_fwd_pairs<T, false, NM, true>), grid, block, shm, s, a, f, part);
        else hipLaunchKernelGGL((k_fwd_pairs<T, false, NM, false>), grid, block, shm, s, a, f, part);
    };
    if (P->nm <= 1) go(std::integral_constant<int, 1>{});
    else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
    else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
    else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
    else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
    else go(std::integral_constant<int, 8>{});
}

bool use_pairs(ephbte_plan P, int B) {
    return B == 1 && P->layout == 3 && P->sym_ok && P->pr_ok && P->n_pr_tiles > 0;
}

int64_t nqm_of(ephbte_plan P) {
    return static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2] * P->nm;
}

template <typename T> Epi<T> epi_store(T *out, int64_t ld) {
    Epi<T> e{};
    e.mode = EPI_STORE;
    e.out = out;
    e.ld_out = ld;
    return e;
}

constexpr int kBatchDPW = 4;       // destinations per wave in the batched kernel
constexpr int kBatchThreads = 512;

template <typename T>
BArgs<T> batch_args(ephbte_plan P, const BTileRec *tiles, const int64_t *sub_off, int pt, int64_t n) {
    BArgs<T> a;
    a.pnu = P->pnu;
    a.g2 = static_cast<const T *>(P->g2);
    a.st = static_cast<const StateRec<T> *>(P->st);
    a.hwN = static_cast<const Pair2<T> *>(P->hwN.p);
    table_strides(P, &a.tq, &a.tm);
    a.btiles = tiles;
    a.sub_off = sub_off;
    a.S = P->S;
    a.nm = P->nm;
    a.nq0 = P->nq[0];
    a.nq1 = P->nq[1];
    a.nq2 = P->nq[2];
    a.pt = pt;
    a.padq = P->padq ? 1 : 0;
    a.qoff = P->qoff;
    a.n_btiles = n;
    a.xcd = 0;   // measured: plain order is at least as fast for the batched pass
    Tables<T> t = tables<T>(P, nullptr);
    a.mc = t.mc;
    a.K = t.K;
    return a;
}

template <typename T> BArgs<T> batch_args(ephbte_plan P) {
    return batch_args<T>(P, P->btiles, P->sub_off, P->pt, P->n_btiles);
}

// LDS of the batched kernel: f[pt][65] and the pt partner states
size_t batch_lds_bytes(ephbte_plan P, int pt) {
    const size_t es = P->dtype == EPHBTE_F64 ? 8 : 4;
    return static_cast<size_t>(pt) * (65 * es + (P->dtype == EPHBTE_F64 ? sizeof(StateRec<double>)
                                                                          : sizeof(StateRec<float>)));
}

bool capturing(hipStream_t s);

// launches timed per ephbte_kernel_timing period; later ones are not timed
constexpr size_t kTimedLaunches = 4096;

// Event before a launch of the forward kernel when timing is on (not under
// graph capture); returns the pair's index for ktime_end, or -1.
int64_t ktime_begin(ephbte_plan P, hipStream_t s) {
    if (!P->ktime_on || P->ktime_used >= kTimedLaunches || capturing(s)) return -1;
    const size_t i = P->ktime_used;
    while (P->ktime_ev.size() < 2 * (i + 1)) {
        hipEvent_t e = nullptr;
        HIPC(hipEventCreate(&e));
        P->ktime_ev.push_back(e);
    }
    HIPC(hipEventRecord(P->ktime_ev[2 * i], s));
    ++P->ktime_used;
    return static_cast<int64_t>(i);
}

void ktime_end(ephbte_plan P, hipStream_t s, int64_t i) {
    if (i >= 0) HIPC(hipEventRecord(P->ktime_ev[2 * static_cast<size_t>(i) + 1], s));
}

template <typename T>
void enqueue_forward_batched(ephbte_plan P, int B, const T *f, int64_t ldf, const Epi<T> &E,
                             hipStream_t s) {
    const size_t shm = batch_lds_bytes(P, P->pt);
    dim3 grid(static_cast<unsigned>(P->n_btiles), (B + 63) / 64);
    const int64_t kt = ktime_begin(P, s);
    hipLaunchKernelGGL((k_fwd_batched<T, kBatchDPW, 0>), grid, dim3(kBatchThreads), shm, s,
                       batch_args<T>(P), f, ldf, B, E, (const T *)nullptr, int64_t(0));
    ktime_end(P, s, kt);
    HIPC(hipGetLastError());
}

// the per-vector N of 64 vectors on the table rows, addressed by 32-bit byte
// offsets in the batched pass
bool pv_table_fits(ephbte_plan P) {
    const int64_t rows = P->padq ? P->qpad_n : static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2];
    return rows * P->nm * 64 * (P->dtype == EPHBTE_F64 ? 8 : 4) < (int64_t(1) << 31);
}

// I for B >= 8 vectors with a bath per vector (nph: B tables [Nq][n_modes]):
// per group of 64 vectors, their N on the rows of the {hw, N} table
// ([row][mode][64], in P->nvec) and one batched launch that applies each
// entry's N-free coefficients as the shared-bath pass does and its N
// coefficient with each vector's N.  The {hw, N} table must hold this plan's
// hw (its N column is not read).
template <typename T>
void enqueue_forward_batched_pv(ephbte_plan P, int B, const T *f, int64_t ldf, const T *nph, T *I, int64_t ldi,
                                hipStream_t s) {
    const size_t shm = batch_lds_bytes(P, P->pt);
    const int64_t rows = P->padq ? P->qpad_n : static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2];
    const int64_t ld = rows * P->nm * 64;
    ensure_zeroed(P, P->nvec, sizeof(T) * static_cast<size_t>(ld));
    const int64_t tab = nqm_of(P);
    T *nv = static_cast<T *>(P->nvec.p);
    const int n_rows = static_cast<int>(P->padq ? P->n_used_rows : rows);
    for (int g = 0; g * 64 < B; ++g) {
        const int nb = std::min(64, B - g * 64);
        hipLaunchKernelGGL((k_pack_nvec<T>), dim3(grid_of(static_cast<int64_t>(n_rows) * P->nm * 64)), dim3(256), 0,
                           s, nph + g * 64 * tab, nv, P->padq ? 1 : 0, P->qbox, P->nm, (const int32_t *)P->used_rows,
                           n_rows, nb);
        const Epi<T> E = epi_store<T>(I + g * 64 * ldi, ldi);
        const dim3 grid(static_cast<unsigned>(P->n_btiles), 1);
        const BArgs<T> a = batch_args<T>(P);
        const T *fg = f + g * 64 * ldf;
        auto go = [&](auto rc) {
            constexpr int RUN = decltype(rc)::value;
            hipLaunchKernelGGL((k_fwd_batched<T, kBatchDPW, RUN>), grid, dim3(kBatchThreads), shm, s, a, fg, ldf, nb,
                               E, (const T *)nv, ld);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
    }
    HIPC(hipGetLastError());
}

// Batch tiles for partner sub-tiles of pt states: shapes from the host's
// partner ranges, entry offsets searched on the device.  Synchronous.
void build_btiles(ephbte_plan P, int pt, BTileRec *&tiles, int64_t *&sub_off, int64_t &n) {
    int64_t slots = 0;
    const std::vector<BTile> bt =
        make_btiles(P->pmin, P->pmax, pt, kBatchDPW * (kBatchThreads / 64), 4096, &slots);
    static_assert(sizeof(BTile) == sizeof(BTileRec), "batch tile record layout");
    dfree(reinterpret_cast<void *&>(tiles));
    dfree(reinterpret_cast<void *&>(sub_off));
    n = 0;
    size_t dummy = 0;
    dalloc(tiles, std::max<size_t>(bt.size(), 1) * sizeof(BTileRec), &dummy);
    dalloc(sub_off, static_cast<size_t>(std::max<int64_t>(slots, 1)) * sizeof(int64_t), &dummy);
    if (!bt.empty()) {
        HIPC(hipMemcpy(tiles, bt.data(), bt.size() * sizeof(BTileRec), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_sub_offsets, dim3(static_cast<unsigned>(bt.size())), dim3(256), 0, nullptr,
                           tiles, P->pnu, P->chunk_beg, P->dest_chunk, P->S, pt, sub_off);
        HIPC(hipGetLastError());
    }
    HIPC(hipDeviceSynchronize());
    n = static_cast<int64_t>(bt.size());
}

void upload_btiles(ephbte_plan P, int pt) {
    free_graphs(P);   // captured forward passes hold the old tiles
    build_btiles(P, pt, P->btiles, P->sub_off, P->n_btiles);
    P->pt = pt;
}

// LDS of the batched reverse kernel: {f, lam}[pt][65] and the pt partner states
size_t vjp_batch_lds_bytes(ephbte_plan P, int pt) {
    const size_t es = P->dtype == EPHBTE_F64 ? 8 : 4;
    return static_cast<size_t>(pt) * (65 * 2 * es + (P->dtype == EPHBTE_F64 ? sizeof(StateRec<double>)
                                                                              : sizeof(StateRec<float>)));
}

// partners per sub-tile of the batched reverse pass (measured at B = 64 on
// 2e8 channels: 64 in FP64, 96 in FP32; LDS 68 KB and 52 KB per workgroup)
int vjp_default_pt(ephbte_plan P) { return P->dtype == EPHBTE_F64 ? 64 : 96; }

// Tiles of the batched reverse pass (at plan build).  Synchronous.
void upload_vjp_btiles(ephbte_plan P, int pt) {
    if (vjp_batch_lds_bytes(P, pt) > P->lds_max) return;   // vpt stays 0: per-vector pass
    build_btiles(P, pt, P->vbtiles, P->vsub_off, P->n_vbtiles);
    P->vpt = pt;
}

// Batched reverse pass over B vectors in groups of 64 (false: not available
// for this plan; the caller takes the per-vector pass).  The {hw, N} table
// must already be packed.
template <typename T>
bool enqueue_vjp_batched(ephbte_plan P, int B, const T *f, int64_t ldf, const T *lam, int64_t ldl,
                         T *gf, int64_t ldgf, double *gg2, int gg2_mode, hipStream_t s) {
    if (B < P->batch_min || P->vpt == 0 || P->n_vbtiles == 0) return false;
    const BArgs<T> a = batch_args<T>(P, P->vbtiles, P->vsub_off, P->vpt, P->n_vbtiles);
    const size_t shm = vjp_batch_lds_bytes(P, P->vpt);
    for (int b0 = 0; b0 < B; b0 += 64) {
        const int nb = std::min(64, B - b0);
        const int gm = gg2_mode == 0 ? 0 : (b0 == 0 ? gg2_mode : 2);
        hipLaunchKernelGGL((k_vjp_batched<T, kBatchDPW, 0>), dim3(static_cast<unsigned>(P->n_vbtiles)),
                           dim3(kBatchThreads), shm, s, a, f, ldf, lam, ldl, b0, nb, gf, ldgf,
                           (const int32_t *)P->ent_chan, gg2, gm, (const T *)nullptr, int64_t(0));
    }
    HIPC(hipGetLastError());
    return true;
}

// The reverse pass for B >= 8 vectors with a bath per vector: per group of
// 64 vectors their N on the table rows (as the forward pass) and one batched
// launch.  The {hw, N} table must hold this plan's hw.
template <typename T>
bool enqueue_vjp_batched_pv(ephbte_plan P, int B, const T *f, int64_t ldf, const T *nph, const T *lam,
                            int64_t ldl, T *gf, int64_t ldgf, double *gg2, int gg2_mode, hipStream_t s) {
    if (B < P->batch_min || P->vpt == 0 || P->n_vbtiles == 0 || !pv_table_fits(P)) return false;
    const BArgs<T> a = batch_args<T>(P, P->vbtiles, P->vsub_off, P->vpt, P->n_vbtiles);
    const size_t shm = vjp_batch_lds_bytes(P, P->vpt);
    const int64_t rows = P->padq ? P->qpad_n : static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2];
    const int64_t ld = rows * P->nm * 64;
    ensure_zeroed(P, P->nvec, sizeof(T) * static_cast<size_t>(ld));
    const int64_t tab = nqm_of(P);
    T *nv = static_cast<T *>(P->nvec.p);
    const int n_rows = static_cast<int>(P->padq ? P->n_used_rows : rows);
    for (int b0 = 0; b0 < B; b0 += 64) {
        const int nb = std::min(64, B - b0);
        hipLaunchKernelGGL((k_pack_nvec<T>), dim3(grid_of(static_cast<int64_t>(n_rows) * P->nm * 64)), dim3(256), 0,
                           s, nph + b0 * tab, nv, P->padq ? 1 : 0, P->qbox, P->nm, (const int32_t *)P->used_rows,
                           n_rows, nb);
        const int gm = gg2_mode == 0 ? 0 : (b0 == 0 ? gg2_mode : 2);
        auto go = [&](auto rc) {
            constexpr int RUN = decltype(rc)::value;
            hipLaunchKernelGGL((k_vjp_batched<T, kBatchDPW, RUN>), dim3(static_cast<unsigned>(P->n_vbtiles)),
                               dim3(kBatchThreads), shm, s, a, f, ldf, lam, ldl, b0, nb, gf, ldgf,
                               (const int32_t *)P->ent_chan, gg2, gm, (const T *)nv, ld);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
    }
    HIPC(hipGetLastError());
    return true;
}

// workgroups of the {hw, N} pack kernels
constexpr int64_t kPackBlocks = 8192;

// Interleave the plan's phonon energies with the caller's occupations into
// one {hw, N} table (one gather per entry instead of two).
template <typename T> void enqueue_pack(ephbte_plan P, const void *nph, hipStream_t s) {
    // each pack block also stores the max |N| it saw; one more workgroup reduces
    // those to the max |N| of this call (the single-copy pass's fixed-point scale)
    double *bmax = P->pack_bmax;
    unsigned nb;
    if (P->padq) {
        const int64_t n = P->n_used_rows * P->nm;
        nb = static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((n + 255) / 256, kPackBlocks), 1));
        hipLaunchKernelGGL((k_pack_hwN_pad<T>), dim3(nb), dim3(256), 0, s, static_cast<const T *>(P->hw),
                           static_cast<const T *>(nph), static_cast<Pair2<T> *>(P->hwN.p), P->qbox, P->nm,
                           static_cast<int>(P->qpad_n), (const int32_t *)P->used_rows,
                           static_cast<int>(P->n_used_rows), P->tab_mm ? 1 : 0, bmax);
    } else {
        const int64_t n = nqm_of(P);
        nb = static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((n + 255) / 256, kPackBlocks), 1));
        hipLaunchKernelGGL((k_pack_hwN<T>), dim3(nb), dim3(256), 0, s, static_cast<const T *>(P->hw),
                           static_cast<const T *>(nph), static_cast<Pair2<T> *>(P->hwN.p), n, bmax);
    }
    hipLaunchKernelGGL(k_max_blocks, dim3(1), dim3(1024), 0, s, (const double *)bmax, static_cast<int>(nb),
                       P->nmax_bits);
}

size_t tiled_lds_bytes(ephbte_plan P) {
    const size_t es = P->dtype == EPHBTE_F64 ? 8 : 4;
    const size_t tab = P->dtype == EPHBTE_F64 ? kExpTab * sizeof(double) : 0;
    return static_cast<size_t>(P->lds_states) * (2 * es + 4) + tab;
}

// Enqueue I[f] for B vectors with epilogue E (no allocation inside; the
// caller ensured P->part and P->hwN are large enough).  pack = false when the
// {hw, N} table already holds this call's occupations.
// max |f| over one vector into P->fmax_bits: the fixed-point scale of the
// single-copy passes for occupations outside [0, 1] (Bose plans)
template <typename T> void enqueue_fmax(ephbte_plan P, const T *f, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, P->fmax_bits, 1);
    hipLaunchKernelGGL((k_abs_max_bits<T>), dim3(grid_of(P->S)), dim3(256), 0, s, f, int64_t(P->S), P->fmax_bits);
}

template <typename T>
void enqueue_forward(ephbte_plan P, int B, const T *f, int64_t ldf, const void *nph,
                     const Epi<T> &E, hipStream_t s, bool pack = true) {
    if (pack) enqueue_pack<T>(P, nph, s);
    if (B >= P->batch_min && P->n_btiles > 0) {
        enqueue_forward_batched<T>(P, B, f, ldf, E, s);
        return;
    }
    if (P->boson && (use_pairs(P, B) || use_sym(P, B))) enqueue_fmax<T>(P, f, s);
    if (use_pairs(P, B)) {
        TiledArgs<T> a = pair_args<T>(P);
        T *part = static_cast<T *>(P->sym_part.p);
        const size_t shm = sym_lds_bytes(P->dtype, P->pr_lds_states);
        const int64_t kt = ktime_begin(P, s);
        launch_pairs<T>(P, a, f, part, shm, s, P->padq);
        ktime_end(P, s, kt);
        hipLaunchKernelGGL((k_sym_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a, f,
                           (const T *)part, E);
        HIPC(hipGetLastError());
        return;
    }
    if (use_sym(P, B)) {
        TiledArgs<T> a = sym_args<T>(P);
        T *part = static_cast<T *>(P->sym_part.p);
        // entries per lane and stage: 2 in FP64 keeps the pipeline in the 128
        // registers a lane has at 1024 threads per workgroup
        constexpr int U = sizeof(T) == 8 ? 2 : 4;
        const size_t shm = sym_lds_bytes(P->dtype, P->sym_lds_states);
        const int64_t kt = ktime_begin(P, s);
        if (P->padq)
            hipLaunchKernelGGL((k_fwd_sym<T, U, true>), dim3(static_cast<unsigned>(P->n_sym_tiles)), dim3(1024), shm,
                               s, a, f, part);
        else
            hipLaunchKernelGGL((k_fwd_sym<T, U, false>), dim3(static_cast<unsigned>(P->n_sym_tiles)), dim3(1024), shm,
                               s, a, f, part);
        ktime_end(P, s, kt);
        hipLaunchKernelGGL((k_sym_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a, f,
                           (const T *)part, E);
        HIPC(hipGetLastError());
        return;
    }
    TiledArgs<T> a = tiled_args<T>(P);
    T *part = static_cast<T *>(P->part.p);
    dim3 grid(tile_grid(P, P->n_tiles), B);
    const int64_t kt = ktime_begin(P, s);
    if (P->padq)
        hipLaunchKernelGGL((k_fwd_tiled<T, 4, 512, true>), grid, dim3(P->block_threads),
                           tiled_lds_bytes(P), s, a, f, ldf, part, E);
    else
        hipLaunchKernelGGL((k_fwd_tiled<T, 4, 512, false>), grid, dim3(P->block_threads),
                           tiled_lds_bytes(P), s, a, f, ldf, part, E);
    ktime_end(P, s, kt);
    if (!P->fused) {
        dim3 g2((P->S + 255) / 256, B);
        hipLaunchKernelGGL((k_tiled_finish<T>), g2, dim3(256), 0, s, a, f, ldf, (const T *)part, E);
    }
    HIPC(hipGetLastError());
}

template <typename T> void ensure_fwd(ephbte_plan P, int B) {
    if (!P->fused) ensure(P->part, sizeof(T) * 2 * static_cast<size_t>(P->n_chunks) * B, &P->ws_gen);
    if (use_sym(P, B))
        ensure(P->sym_part, sizeof(T) * 2 * static_cast<size_t>(std::max<int64_t>(P->n_sym_chunks, 1)),
               &P->ws_gen);
    if (use_pairs(P, B))
        ensure(P->sym_part, sizeof(T) * 2 * static_cast<size_t>(std::max<int64_t>(P->n_pr_chunks, 1)),
               &P->ws_gen);
    const int64_t tab = P->padq ? P->qpad_n * P->nm : nqm_of(P);
    ensure_zeroed(P, P->hwN, sizeof(Pair2<T>) * static_cast<size_t>(std::max<int64_t>(tab, 1)));
}

template <typename T> void ensure_part(ephbte_plan P, int B, int per_chunk) {
    if (!P->fused) ensure(P->part, sizeof(T) * per_chunk * static_cast<size_t>(P->n_chunks) * B, &P->ws_gen);
}

// Bytes of `scratch` the allocation-free forward pass needs: the plain
// {hw, N} table (q-major, no padding) and the partial sums of the chunks.
size_t noalloc_bytes(ephbte_plan P) {
    const size_t es = P->dtype == EPHBTE_F64 ? 8 : 4;
    const size_t tab = 2 * es * static_cast<size_t>(std::max<int64_t>(nqm_of(P), 1));
    size_t part = 0;
    if (use_pairs(P, 1)) part = 2 * es * static_cast<size_t>(std::max<int64_t>(P->n_pr_chunks, 1));
    else if (use_sym(P, 1)) part = 2 * es * static_cast<size_t>(std::max<int64_t>(P->n_sym_chunks, 1));
    else if (!P->fused) part = 2 * es * static_cast<size_t>(P->n_chunks);
    return ((tab + 255) & ~size_t(255)) + part;
}

// I[f] for one vector with every workspace inside `scratch` (base: its
// device address): the same kernels as enqueue_forward, with the plain
// {hw, N} table in place of the plan's padded one.  Allocates nothing.
template <typename T>
void enqueue_forward_noalloc(ephbte_plan P, const T *f, const void *nph, T *I, unsigned char *base,
                             hipStream_t s) {
    const int64_t n = nqm_of(P);
    Pair2<T> *tab = reinterpret_cast<Pair2<T> *>(base);
    T *part = reinterpret_cast<T *>(base + ((2 * sizeof(T) * static_cast<size_t>(std::max<int64_t>(n, 1)) + 255) &
                                            ~size_t(255)));
    const unsigned nb = static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((n + 255) / 256, kPackBlocks), 1));
    hipLaunchKernelGGL((k_pack_hwN<T>), dim3(nb), dim3(256), 0, s, static_cast<const T *>(P->hw),
                       static_cast<const T *>(nph), tab, n, P->pack_bmax);
    hipLaunchKernelGGL(k_max_blocks, dim3(1), dim3(1024), 0, s, (const double *)P->pack_bmax,
                       static_cast<int>(nb), P->nmax_bits);
    const Epi<T> E = epi_store<T>(I, P->S);
    if (use_pairs(P, 1)) {
        TiledArgs<T> a = pair_args<T>(P);
        a.hwN = tab;
        a.padq = 0;
        a.tq = P->nm;
        a.tm = 1;
        launch_pairs<T>(P, a, f, part, sym_lds_bytes(P->dtype, P->pr_lds_states), s, false);
        hipLaunchKernelGGL((k_sym_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a, f,
                           (const T *)part, E);
    } else if (use_sym(P, 1)) {
        TiledArgs<T> a = sym_args<T>(P);
        a.hwN = tab;
        a.padq = 0;
        a.tq = P->nm;
        a.tm = 1;
        constexpr int U = sizeof(T) == 8 ? 2 : 4;
        hipLaunchKernelGGL((k_fwd_sym<T, U, false>), dim3(static_cast<unsigned>(P->n_sym_tiles)), dim3(1024),
                           sym_lds_bytes(P->dtype, P->sym_lds_states), s, a, f, part);
        hipLaunchKernelGGL((k_sym_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a, f,
                           (const T *)part, E);
    } else {
        TiledArgs<T> a = tiled_args<T>(P);
        a.hwN = tab;
        a.padq = 0;
        a.tq = P->nm;
        a.tm = 1;
        hipLaunchKernelGGL((k_fwd_tiled<T, 4, 512, false>), dim3(tile_grid(P, P->n_tiles), 1),
                           dim3(P->block_threads), tiled_lds_bytes(P), s, a, f, int64_t(P->S), part, E);
        if (!P->fused)
            hipLaunchKernelGGL((k_tiled_finish<T>), dim3((P->S + 255) / 256, 1), dim3(256), 0, s, a, f,
                               int64_t(P->S), (const T *)part, E);
    }
    HIPC(hipGetLastError());
}

// gg2_mode: 0 none, 1 overwrite, 2 accumulate.  E.mode < 0: gradient of g2 only.
// The caller packed the {hw, N} table for nph and ensured P->part (n_chunks).
template <typename T>
void enqueue_vjp(ephbte_plan P, const T *f, const T *lam, const void *nph, const Epi<T> &E,
                 double *gg2, int gg2_mode, hipStream_t s) {
    (void)nph;
    if (use_pairs(P, 1) && vjp_pair_lds_bytes(P->dtype, P->pr_lds_states) <= P->lds_max) {
        // max |lam| of this call (the partner side's fixed-point scale)
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, P->lmax_bits, 1);
        hipLaunchKernelGGL((k_abs_max_bits<T>), dim3(grid_of(P->S)), dim3(256), 0, s, lam, int64_t(P->S),
                           P->lmax_bits);
        if (P->boson) enqueue_fmax<T>(P, f, s);
        TiledArgs<T> a = pair_args<T>(P);
        T *part = static_cast<T *>(P->sym_part.p);
        const int want_f = E.mode >= 0 ? 1 : 0;
        const dim3 grid(static_cast<unsigned>(P->n_pr_tiles)), block(kVjpPairThreads);
        const size_t shm = vjp_pair_lds_bytes(P->dtype, P->pr_lds_states);
        auto go = [&](auto nmc) {
            constexpr int NM = decltype(nmc)::value;
            const bool tab = sizeof(T) == 8 && P->exp_table;
            const unsigned long long *lm = P->lmax_bits;
            const int32_t *ch = P->pr_chan, *c0 = P->pr_ch0;
            if (P->padq && tab)
                hipLaunchKernelGGL((k_vjp_pairs<T, true, NM, true>), grid, block, shm, s, a, f, lam, part, want_f, lm,
                                   ch, c0, gg2, gg2_mode);
            else if (P->padq)
                hipLaunchKernelGGL((k_vjp_pairs<T, true, NM, false>), grid, block, shm, s, a, f, lam, part, want_f,
                                   lm, ch, c0, gg2, gg2_mode);
            else if (tab)
                hipLaunchKernelGGL((k_vjp_pairs<T, false, NM, true>), grid, block, shm, s, a, f, lam, part, want_f,
                                   lm, ch, c0, gg2, gg2_mode);
            else
                hipLaunchKernelGGL((k_vjp_pairs<T, false, NM, false>), grid, block, shm, s, a, f, lam, part, want_f,
                                   lm, ch, c0, gg2, gg2_mode);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
        if (want_f)
            hipLaunchKernelGGL((k_vjp_pairs_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a,
                               (const T *)part, (const unsigned long long *)P->lmax_bits, E);
        HIPC(hipGetLastError());
        return;
    }
    TiledArgs<T> a = tiled_args<T>(P);
    a.xcd = 0;   // measured: plain tile order is faster for the reverse pass
    a.tiles = P->small_tiles;
    a.n_tiles = P->n_small_tiles;
    T *part = static_cast<T *>(P->part.p);
    dim3 grid(static_cast<unsigned>(P->n_small_tiles));
    // entries per lane and pipeline stage: 2 in FP64 keeps the two stages in
    // registers at two workgroups per compute unit
    constexpr int U = sizeof(T) == 8 ? 2 : 4;
    if (P->padq)
        hipLaunchKernelGGL((k_vjp_tiled<T, U, true>), grid, dim3(P->block_threads), tiled_lds_bytes(P),
                           s, a, f, lam, part, E, (const int32_t *)P->ent_chan, gg2, gg2_mode);
    else
        hipLaunchKernelGGL((k_vjp_tiled<T, U, false>), grid, dim3(P->block_threads), tiled_lds_bytes(P),
                           s, a, f, lam, part, E, (const int32_t *)P->ent_chan, gg2, gg2_mode);
    if (!P->fused && E.mode >= 0)
        hipLaunchKernelGGL((k_vjp_tiled_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a,
                           (const T *)part, E);
    HIPC(hipGetLastError());
}

template <typename T>
__global__ void k_cast_g2(const int32_t *__restrict__ ent_chan, const double *__restrict__ g2,
                          T *__restrict__ out, int64_t E) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < E;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[e] = static_cast<T>(g2[ent_chan[e]]);
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// p[idx[x]] = 0 for x < n (the |g|^2 gradients of channels the selection removed)
__global__ void k_zero_at(double *p, const int32_t *__restrict__ idx, int64_t n) {
    for (int64_t x = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; x < n;
         x += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[idx[x]] = 0.0;
}

template <typename T>
__global__ void k_scale(const T *__restrict__ x, T *__restrict__ y, T a, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        y[i] = a * x[i];
}

template <typename T>
__global__ void k_copy_strided(const T *__restrict__ x, int64_t ldx, T *__restrict__ y,
                               int64_t ldy, int S, int B) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= S) return;
    const int b = blockIdx.y;
    y[static_cast<int64_t>(b) * ldy + d] = x[static_cast<int64_t>(b) * ldx + d];
}

// transport helpers
template <typename T>
__global__ void k_transport_prep(const T *__restrict__ f0, const T *__restrict__ vel,
                                 const T *__restrict__ tau_inv, T inv_kt, int S,
                                 T *__restrict__ tau, Vec4<T> *__restrict__ rhs,
                                 Vec4<T> *__restrict__ x0) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= S) return;
    const T ti = tau_inv[d];
    const T t = ti > T(0) ? T(1) / ti : T(0);
    const T f = f0[d];
    const T dfde = -f * (T(1) - f) * inv_kt;
    Vec4<T> r;
    r.x = vel[3 * static_cast<int64_t>(d)] * dfde;
    r.y = vel[3 * static_cast<int64_t>(d) + 1] * dfde;
    r.z = vel[3 * static_cast<int64_t>(d) + 2] * dfde;
    r.w = T(0);
    tau[d] = t;
    rhs[d] = r;
    Vec4<T> x;
    x.x = t * r.x;
    x.y = t * r.y;
    x.z = t * r.z;
    x.w = T(0);
    x0[d] = x;
}

// 10 double partial sums per block: sum v_a x_b (9) and sum f0 (only when f0 != NULL).
template <typename T>
__global__ __launch_bounds__(256) void k_mobility_partial(const T *__restrict__ vel,
                                                          const Vec4<T> *__restrict__ x,
                                                          const T *__restrict__ f0, int S,
                                                          double *__restrict__ out) {
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < S; d += gridDim.x * blockDim.x) {
        const Vec4<T> xd = x[d];
        const double xs[3] = {static_cast<double>(xd.x), static_cast<double>(xd.y),
                              static_cast<double>(xd.z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = static_cast<double>(vel[3 * static_cast<int64_t>(d) + a]);
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) acc[3 * a + bb] += v * xs[bb];
        }
        if (f0) acc[9] += static_cast<double>(f0[d]);
    }
    block_sum<double, 10>(acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 10; ++k) out[10 * blockIdx.x + k] = acc[k];
}

__global__ __launch_bounds__(256) void k_rows_sum10(const double *__restrict__ in, int rows,
                                                    double *__restrict__ out) {
    double acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[k] += in[10 * r + k];
    block_sum<double, 10>(acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 10; ++k) out[k] = acc[k];
}

template <typename T>
__global__ void k_unpack_x(const Vec4<T> *__restrict__ x, T *__restrict__ out, int S) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= S) return;
    const Vec4<T> v = x[d];
    out[3 * static_cast<int64_t>(d)] = v.x;
    out[3 * static_cast<int64_t>(d) + 1] = v.y;
    out[3 * static_cast<int64_t>(d) + 2] = v.z;
}

constexpr int kRedBlocks = 256;

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

size_t esize(ephbte_plan P) { return P->dtype == EPHBTE_F64 ? 8 : 4; }

// entries read past the end of the last chunk by the unconditional stream
// loads land in this zero padding
constexpr int64_t kEntryPad = 4096;

// Shifted k coordinates of the box table: per axis an origin o and the
// extent span of c = (k - o) mod Nq over the states.  Differences of c agree
// with those of k modulo Nq, so any origin gives the same q; placing o at the
// end of the largest unoccupied (circular) run of coordinates keeps a window
// of states around k = 0 in one run instead of split across the wrap, which
// makes span, and the box of all differences, as small as it can be.
void q_box_of(const HostLayout &L, uint32_t org[3], int span[3]) {
    for (int a = 0; a < 3; ++a) {
        const int n = L.nq[a], sh = 20 - 10 * a;
        std::vector<char> occ(n, 0);
        for (int64_t s = 0; s < L.S; ++s) occ[(L.kq[s] >> sh) & 1023u] = 1;
        int best_len = 0, best_end = 0;
        for (int c = 0; c < n; ++c) {
            if (occ[c]) continue;
            int len = 0;
            while (len < n && !occ[(c + len) % n]) ++len;
            if (len > best_len) {
                best_len = len;
                best_end = (c + len) % n;
            }
            if (len == n) break;
        }
        org[a] = best_len > 0 && best_len < n ? static_cast<uint32_t>(best_end) : 0u;
        int top = 0;
        for (int c = 0; c < n; ++c)
            if (occ[(c + static_cast<int>(org[a])) % n]) top = c;
        span[a] = top + 1;
    }
}

template <typename T> void upload_layout(ephbte_plan P, const ephbte_problem *pr, HostLayout &L) {
    size_t &acc = P->layout_bytes;
    const int64_t E = L.E, S = L.S;
    dalloc(P->pnu, sizeof(uint32_t) * (E + kEntryPad), &acc);
    dalloc(P->ent_chan, sizeof(int32_t) * E, &acc);
    dalloc(reinterpret_cast<T *&>(P->g2), sizeof(T) * (E + kEntryPad), &acc);
    HIPC(hipMemset(P->pnu + E, 0, sizeof(uint32_t) * kEntryPad));
    HIPC(hipMemset(static_cast<T *>(P->g2) + E, 0, sizeof(T) * kEntryPad));
    dalloc(reinterpret_cast<StateRec<T> *&>(P->st), sizeof(StateRec<T>) * S, &acc);
    const int64_t nqm = static_cast<int64_t>(L.nq[0]) * L.nq[1] * L.nq[2] * L.n_modes;
    dalloc(reinterpret_cast<T *&>(P->hw), sizeof(T) * nqm, &acc);
    HIPC(hipMemcpy(P->pnu, L.pnu.data(), sizeof(uint32_t) * E, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->ent_chan, L.ent_chan.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice));
    {
        std::vector<T> g(E);
        parallel_ranges(E, host_threads(), [&](int, int64_t b, int64_t e) {
            for (int64_t x = b; x < e; ++x) g[x] = static_cast<T>(pr->g2[L.ent_chan[x]]);
        });
        HIPC(hipMemcpy(P->g2, g.data(), sizeof(T) * E, hipMemcpyHostToDevice));
    }
    {
        std::vector<StateRec<T>> st(S);
        for (int64_t s = 0; s < S; ++s) {
            std::memset(&st[s], 0, sizeof(StateRec<T>));
            st[s].eps = static_cast<T>(pr->eps[s]);
            st[s].kq = L.kq[s];
            if (P->padq) {
                uint32_t c[3];
                for (int a = 0; a < 3; ++a) {
                    const uint32_t n = static_cast<uint32_t>(L.nq[a]);
                    c[a] = (((L.kq[s] >> (20 - 10 * a)) & 1023u) + n - P->qorg[a]) % n;
                }
                const uint32_t b1 = static_cast<uint32_t>(P->qbox.b[1]), b2 = static_cast<uint32_t>(P->qbox.b[2]);
                st[s].kqp = (c[0] * b1 + c[1]) * b2 + c[2];
            }
        }
        HIPC(hipMemcpy(P->st, st.data(), sizeof(StateRec<T>) * S, hipMemcpyHostToDevice));
        P->st_key.resize(static_cast<size_t>(S));
        for (int64_t s = 0; s < S; ++s) P->st_key[s] = P->padq ? st[s].kqp : st[s].kq;
        if (P->padq) {
            // box rows the entries reference (both orientations of every
            // channel, and q = 0): the only rows a call packs
            const int T_ = host_threads();
            std::vector<std::vector<uint8_t>> marks(T_, std::vector<uint8_t>(static_cast<size_t>(P->qpad_n), 0));
            parallel_ranges(S, T_, [&](int t, int64_t b, int64_t e) {
                std::vector<uint8_t> &m = marks[t];
                for (int64_t d = b; d < e; ++d)
                    for (int64_t x = L.row_ptr[d]; x < L.row_ptr[d + 1]; ++x) {
                        const int p = static_cast<int>(L.pnu[x] >> 3);
                        m[static_cast<int64_t>(static_cast<int>(st[p].kqp - st[d].kqp) + P->qoff)] = 1;
                    }
            });
            std::vector<int32_t> used;
            for (int64_t r = 0; r < P->qpad_n; ++r) {
                bool on = r == P->qoff;
                for (int t = 0; t < T_ && !on; ++t) on = marks[t][r] != 0;
                if (on) used.push_back(static_cast<int32_t>(r));
            }
            P->n_used_rows = static_cast<int64_t>(used.size());
            dalloc(P->used_rows, sizeof(int32_t) * used.size(), &acc);
            HIPC(hipMemcpy(P->used_rows, used.data(), sizeof(int32_t) * used.size(), hipMemcpyHostToDevice));
        }
    }
    {
        std::vector<T> h(nqm);
        for (int64_t x = 0; x < nqm; ++x) h[x] = static_cast<T>(pr->hw[x]);
        HIPC(hipMemcpy(P->hw, h.data(), sizeof(T) * nqm, hipMemcpyHostToDevice));
    }
}

// Pair records of the single-copy pass (see build_pair_rows), kept when at
// least half of their mode slots hold a channel (otherwise the per-entry
// single-copy pass streams fewer bytes).  The arrays are padded like the
// entry arrays, so that the kernel's stream loads need no bound.
template <typename T> void upload_pair_rows(ephbte_plan P, const ephbte_problem *pr, const HostLayout &L) {
    PairRows R = build_pair_rows(L);
    const int64_t np = R.n_pairs, nm = P->nm;
    P->pr_ok = np > 0 && 2 * R.n_filled >= np * nm;
    if (!P->pr_ok) return;
    size_t &acc = P->layout_bytes;
    P->pr_np = np;
    P->pr_ld = np + kEntryPad;
    const size_t ld = static_cast<size_t>(P->pr_ld);
    dalloc(P->pr_partner, sizeof(uint32_t) * ld, &acc);
    dalloc(reinterpret_cast<T *&>(P->pr_g2), sizeof(T) * ld * nm, &acc);
    dalloc(P->pr_chan, sizeof(int32_t) * ld * nm, &acc);
    std::vector<uint32_t> part(ld, 0u);
    std::copy(R.partner.begin(), R.partner.end(), part.begin());
    HIPC(hipMemcpy(P->pr_partner, part.data(), sizeof(uint32_t) * ld, hipMemcpyHostToDevice));
    {
        std::vector<uint32_t>().swap(part);
        std::vector<T> g(ld * nm, T(0));
        std::vector<int32_t> ch(ld * nm, -1);
        parallel_ranges(np, host_threads(), [&](int, int64_t b, int64_t e) {
            for (int64_t m = 0; m < nm; ++m)
                for (int64_t j = b; j < e; ++j) {
                    const int32_t c = R.slot_chan[static_cast<size_t>(m * np + j)];
                    ch[static_cast<size_t>(m) * ld + j] = c;
                    g[static_cast<size_t>(m) * ld + j] = c >= 0 ? static_cast<T>(pr->g2[c]) : T(0);
                }
        });
        HIPC(hipMemcpy(P->pr_g2, g.data(), sizeof(T) * g.size(), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->pr_chan, ch.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice));
        // records whose slots hold the channels c0, c0 + 1, .., c0 + n_modes - 1
        std::vector<int32_t> c0(ld, -1);
        parallel_ranges(np, host_threads(), [&](int, int64_t b, int64_t e) {
            for (int64_t j = b; j < e; ++j) {
                const int32_t first = ch[static_cast<size_t>(j)];
                bool run = first >= 0;
                for (int64_t m = 1; run && m < nm; ++m) run = ch[static_cast<size_t>(m) * ld + j] == first + m;
                c0[static_cast<size_t>(j)] = run ? first : -1;
            }
        });
        dalloc(P->pr_ch0, sizeof(int32_t) * ld, &acc);
        HIPC(hipMemcpy(P->pr_ch0, c0.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice));
    }
    P->pr_rowptr = std::move(R.row_ptr);
    P->pr_partner_host = std::move(R.partner);
    P->pr_perm.clear();
}

// The phonon pass's layout (pair records bucketed by {q, -q}, see
// build_phonon_layout) and its chunks of at most kPhChunk records.
template <typename T> void upload_phonon_layout(ephbte_plan P, const ephbte_problem *pr, const HostLayout &L) {
    size_t &acc = P->layout_bytes;
    PhononLayout ph = build_phonon_layout(L);
    const int64_t np = ph.n_pairs, nm = P->nm;
    const int64_t nb = static_cast<int64_t>(ph.bucket_q.size());
    P->ph_np = np;
    P->ph_ld = std::max<int64_t>(np, 1);
    P->ph_nbuckets = nb;
    std::vector<int64_t> cbeg;
    std::vector<int32_t> cbucket, bchunk(static_cast<size_t>(nb) + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        bchunk[b] = static_cast<int32_t>(cbucket.size());
        for (int64_t x = ph.bucket_beg[b]; x < ph.bucket_beg[b + 1]; x += kPhChunk) {
            cbeg.push_back(x);
            cbucket.push_back(static_cast<int32_t>(b));
        }
    }
    bchunk[nb] = static_cast<int32_t>(cbucket.size());
    cbeg.push_back(np);
    P->ph_nchunks = static_cast<int64_t>(cbucket.size());
    const size_t ld = static_cast<size_t>(P->ph_ld);
    dalloc(P->ph_pa, sizeof(uint32_t) * ld, &acc);
    dalloc(P->ph_pb, sizeof(uint32_t) * ld, &acc);
    dalloc(reinterpret_cast<T *&>(P->ph_g2), sizeof(T) * ld * nm, &acc);
    dalloc(P->ph_chan, sizeof(int32_t) * ld * nm, &acc);
    dalloc(P->ph_chunk_beg, sizeof(int64_t) * cbeg.size(), &acc);
    dalloc(P->ph_chunk_bucket, sizeof(int32_t) * std::max<size_t>(cbucket.size(), 1), &acc);
    dalloc(P->ph_bucket_chunk, sizeof(int32_t) * bchunk.size(), &acc);
    dalloc(P->ph_bucket_q, sizeof(int32_t) * std::max<int64_t>(nb, 1), &acc);
    dalloc(P->ph_bucket_qm, sizeof(int32_t) * std::max<int64_t>(nb, 1), &acc);
    dalloc(P->ph_bucket_modes, sizeof(uint32_t) * std::max<int64_t>(nb, 1), &acc);
    dalloc(P->ph_q_bucket, sizeof(int32_t) * ph.q_bucket.size(), &acc);
    if (np > 0) {
        HIPC(hipMemcpy(P->ph_pa, ph.pa.data(), sizeof(uint32_t) * np, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_pb, ph.pb.data(), sizeof(uint32_t) * np, hipMemcpyHostToDevice));
        std::vector<T> g(static_cast<size_t>(np) * nm);
        parallel_ranges(np * nm, host_threads(), [&](int, int64_t b, int64_t e) {
            for (int64_t x = b; x < e; ++x) {
                const int32_t c = ph.slot_chan[x];
                g[x] = c >= 0 ? static_cast<T>(pr->g2[c]) : T(0);
            }
        });
        HIPC(hipMemcpy(P->ph_g2, g.data(), sizeof(T) * g.size(), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_chan, ph.slot_chan.data(), sizeof(int32_t) * ph.slot_chan.size(),
                       hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_chunk_bucket, cbucket.data(), sizeof(int32_t) * cbucket.size(), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_bucket_q, ph.bucket_q.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_bucket_qm, ph.bucket_qm.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(P->ph_bucket_modes, ph.bucket_modes.data(), sizeof(uint32_t) * nb, hipMemcpyHostToDevice));
    }
    HIPC(hipMemcpy(P->ph_chunk_beg, cbeg.data(), sizeof(int64_t) * cbeg.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->ph_bucket_chunk, bchunk.data(), sizeof(int32_t) * bchunk.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(P->ph_q_bucket, ph.q_bucket.data(), sizeof(int32_t) * ph.q_bucket.size(), hipMemcpyHostToDevice));
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- drivers
// Field term in a stage epilogue: D[x] of the stage input x, times sign.
template <typename T> void with_drift(ephbte_plan P, Epi<T> &e, const T *x, int64_t ldx, T sign) {
    if (!P->drift_on) {
        e.nbr = nullptr;
        return;
    }
    e.nbr = P->nbr;
    e.x = x;
    e.ld_x = ldx;
    for (int a = 0; a < 3; ++a) e.rate[a] = static_cast<T>(P->drift_rate[a]);
    e.dsign = sign;
}

template <typename T>
void rk4_enqueue_step(ephbte_plan P, int B, T *f, int64_t ldf, const void *nph, T dt,
                      hipStream_t s, T *ua, T *ub, T *acc, const T *f_in, int64_t ld_in,
                      T *f_out) {
    // stage inputs: u1 = f_in, u2 -> ua, u3 -> ub, u4 -> ua; f_out = f_in + dt/6 (...)
    (void)f;
    (void)ldf;
    const int64_t S = P->S;
    Epi<T> e{};
    e.f0 = f_in;
    e.ld_f0 = ld_in;
    e.acc = acc;
    e.dt = dt;
    e.mode = EPI_RK1;
    e.u_out = ua;
    with_drift<T>(P, e, f_in, ld_in, T(1));
    enqueue_forward<T>(P, B, f_in, ld_in, nph, e, s, false);
    e.mode = EPI_RK2;
    e.u_out = ub;
    with_drift<T>(P, e, ua, S, T(1));
    enqueue_forward<T>(P, B, ua, S, nph, e, s, false);
    e.mode = EPI_RK3;
    e.u_out = ua;
    with_drift<T>(P, e, ub, S, T(1));
    enqueue_forward<T>(P, B, ub, S, nph, e, s, false);
    e.mode = EPI_RK4;
    e.f_out = f_out;
    with_drift<T>(P, e, ua, S, T(1));
    enqueue_forward<T>(P, B, ua, S, nph, e, s, false);
}

template <typename T>
ephbte_status rt_step_impl(ephbte_plan P, int B, T *f, int64_t ldf, const void *nph, double dt,
                           int n_steps, int use_graph, hipStream_t s) {
    const size_t vec = sizeof(T) * static_cast<size_t>(P->S) * B;
    ensure(P->rk_ua, vec, &P->ws_gen);
    ensure(P->rk_ub, vec, &P->ws_gen);
    ensure(P->rk_acc, vec, &P->ws_gen);
    ensure_fwd<T>(P, B);
    T *ua = static_cast<T *>(P->rk_ua.p), *ub = static_cast<T *>(P->rk_ub.p);
    T *acc = static_cast<T *>(P->rk_acc.p);
    const T tdt = static_cast<T>(dt);
    enqueue_pack<T>(P, nph, s);   // the phonon occupations hold for the whole call
    if (!use_graph || n_steps < 2) {
        for (int k = 0; k < n_steps; ++k)
            rk4_enqueue_step<T>(P, B, f, ldf, nph, tdt, s, ua, ub, acc, f, ldf, f);
        return EPHBTE_OK;
    }
    const int K = std::min(n_steps, 25);
    hipStream_t cs = s;
    if (!s) {
        if (!P->own_stream) HIPC(hipStreamCreateWithFlags(&P->own_stream, hipStreamNonBlocking));
        if (!P->ev_a) HIPC(hipEventCreateWithFlags(&P->ev_a, hipEventDisableTiming));
        if (!P->ev_b) HIPC(hipEventCreateWithFlags(&P->ev_b, hipEventDisableTiming));
        cs = P->own_stream;
        HIPC(hipEventRecord(P->ev_a, s));
        HIPC(hipStreamWaitEvent(cs, P->ev_a, 0));
    }
    hipGraphExec_t exec = nullptr;
    for (auto &g : P->graphs)
        if (g.f == f && g.nph == nph && g.ldf == ldf && g.B == B && g.steps == K && g.dt == dt &&
            g.stream == cs && g.ws_gen == P->ws_gen)
            exec = g.exec;
    if (!exec) {
        hipGraph_t graph = nullptr;
        HIPC(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            for (int k = 0; k < K; ++k)
                rk4_enqueue_step<T>(P, B, f, ldf, nph, tdt, cs, ua, ub, acc, f, ldf, f);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(cs, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        HIPC(hipStreamEndCapture(cs, &graph));
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPC(ie);
        if (P->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(P->graphs.front().exec);
            P->graphs.erase(P->graphs.begin());
        }
        P->graphs.push_back(GraphEntry{f, nph, ldf, B, K, dt, cs, P->ws_gen, exec});
    }
    int done = 0;
    for (; done + K <= n_steps; done += K) HIPC(hipGraphLaunch(exec, cs));
    for (; done < n_steps; ++done)
        rk4_enqueue_step<T>(P, B, f, ldf, nph, tdt, cs, ua, ub, acc, f, ldf, f);
    if (!s) {
        HIPC(hipEventRecord(P->ev_b, cs));
        HIPC(hipStreamWaitEvent(s, P->ev_b, 0));
    }
    return EPHBTE_OK;
}

template <typename T>
ephbte_status rt_adjoint_impl(ephbte_plan P, const T *f0, const void *nph, double dt, int n,
                              int ce, const T *gfT, T *gf0, double *gg2, int accumulate,
                              hipStream_t s) {
    const int64_t S = P->S;
    const size_t v = sizeof(T) * S;
    const int nck = (n + ce - 1) / ce;
    ensure(P->rk_ua, v, &P->ws_gen);
    ensure(P->rk_ub, v, &P->ws_gen);
    ensure(P->rk_acc, v, &P->ws_gen);
    ensure(P->adj_ck, v * nck, &P->ws_gen);
    ensure(P->adj_U, v * (4 * static_cast<size_t>(ce) + 1), &P->ws_gen);
    ensure(P->adj_la, v, &P->ws_gen);
    ensure(P->adj_lb, v, &P->ws_gen);
    ensure(P->adj_acc, v, &P->ws_gen);
    ensure(P->adj_g, v, &P->ws_gen);
    ensure(P->adj_f, v, &P->ws_gen);
    ensure_part<T>(P, 1, 2);
    ensure_fwd<T>(P, 1);
    T *ua = static_cast<T *>(P->rk_ua.p), *ub = static_cast<T *>(P->rk_ub.p);
    T *racc = static_cast<T *>(P->rk_acc.p);
    T *ck = static_cast<T *>(P->adj_ck.p), *U = static_cast<T *>(P->adj_U.p);
    T *la = static_cast<T *>(P->adj_la.p), *lb = static_cast<T *>(P->adj_lb.p);
    T *acc = static_cast<T *>(P->adj_acc.p), *gb = static_cast<T *>(P->adj_g.p);
    T *fw = static_cast<T *>(P->adj_f.p);
    const T tdt = static_cast<T>(dt);
    enqueue_pack<T>(P, nph, s);
    // forward sweep, checkpoint every ce steps
    HIPC(hipMemcpyAsync(fw, f0, v, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < n; ++k) {
        if (k % ce == 0) HIPC(hipMemcpyAsync(ck + (k / ce) * S, fw, v, hipMemcpyDeviceToDevice, s));
        rk4_enqueue_step<T>(P, 1, fw, S, nph, tdt, s, ua, ub, racc, fw, S, fw);
    }
    HIPC(hipMemcpyAsync(gb, gfT, v, hipMemcpyDeviceToDevice, s));
    int gmode = gg2 ? 2 : 0;
    if (gg2 && !accumulate) {
        hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, s, gg2, P->nch, 0.0);
        HIPC(hipGetLastError());
    }
    Epi<T> e{};
    for (int m = nck - 1; m >= 0; --m) {
        const int s0 = m * ce, s1 = std::min(n, s0 + ce);
        // recompute the segment, keeping every stage input: U[l][0..3]
        HIPC(hipMemcpyAsync(U, ck + m * S, v, hipMemcpyDeviceToDevice, s));
        for (int k = s0; k < s1; ++k) {
            T *u = U + static_cast<int64_t>(k - s0) * 4 * S;
            Epi<T> r{};
            r.f0 = u;
            r.ld_f0 = S;
            r.acc = racc;
            r.dt = tdt;
            r.mode = EPI_RK1;
            r.u_out = u + S;
            with_drift<T>(P, r, u, S, T(1));
            enqueue_forward<T>(P, 1, u, S, nph, r, s, false);
            r.mode = EPI_RK2;
            r.u_out = u + 2 * S;
            with_drift<T>(P, r, u + S, S, T(1));
            enqueue_forward<T>(P, 1, u + S, S, nph, r, s, false);
            r.mode = EPI_RK3;
            r.u_out = u + 3 * S;
            with_drift<T>(P, r, u + 2 * S, S, T(1));
            enqueue_forward<T>(P, 1, u + 2 * S, S, nph, r, s, false);
            r.mode = EPI_RK4;
            r.f_out = u + 4 * S;   // next step's u1 (one spare slot at the end)
            with_drift<T>(P, r, u + 3 * S, S, T(1));
            enqueue_forward<T>(P, 1, u + 3 * S, S, nph, r, s, false);
        }
        // reverse sweep over the segment
        for (int k = s1 - 1; k >= s0; --k) {
            T *u = U + static_cast<int64_t>(k - s0) * 4 * S;
            hipLaunchKernelGGL((k_scale<T>), dim3((S + 255) / 256), dim3(256), 0, s,
                               (const T *)gb, la, tdt / T(6), S);
            HIPC(hipGetLastError());
            e.gbar = gb;
            e.acc = acc;
            e.mode = EPI_ADJ_FIRST;   // u4: acc = v; kb3 = dt/3 g + dt v
            e.cg = tdt / T(3);
            e.cv = tdt;
            e.u_out = lb;
            with_drift<T>(P, e, la, S, T(-1));
            enqueue_vjp<T>(P, u + 3 * S, la, nph, e, gg2, gmode, s);
            e.mode = EPI_ADJ_MID;     // u3: acc += v; kb2 = dt/3 g + dt/2 v
            e.cg = tdt / T(3);
            e.cv = tdt / T(2);
            e.u_out = la;
            with_drift<T>(P, e, lb, S, T(-1));
            enqueue_vjp<T>(P, u + 2 * S, lb, nph, e, gg2, gmode, s);
            e.mode = EPI_ADJ_MID;     // u2: acc += v; kb1 = dt/6 g + dt/2 v
            e.cg = tdt / T(6);
            e.cv = tdt / T(2);
            e.u_out = lb;
            with_drift<T>(P, e, la, S, T(-1));
            enqueue_vjp<T>(P, u + S, la, nph, e, gg2, gmode, s);
            e.mode = EPI_ADJ_LAST;    // u1: g = g + acc + v
            e.gbar_out = gb;
            with_drift<T>(P, e, lb, S, T(-1));
            enqueue_vjp<T>(P, u, lb, nph, e, gg2, gmode, s);
        }
    }
    if (gf0) HIPC(hipMemcpyAsync(gf0, gb, v, hipMemcpyDeviceToDevice, s));
    return EPHBTE_OK;
}

// Coupled electron-phonon step, phonon side of a stage: x = even part in q of
// the rate (the phonons of q and -q evolve as a pair, so N stays even in q as
// Eq. 2's per-orientation evaluation assumes), then the RK4 stage update of N
// (modes as EPI_RK1 .. EPI_RK4).
template <typename T>
__global__ void k_rk_even(int mode, const T *__restrict__ N0, const T *__restrict__ rate,
                          T *__restrict__ acc, T *__restrict__ out, T dt, int n0, int n1, int n2,
                          int nm) {
    const int64_t n = static_cast<int64_t>(n0) * n1 * n2 * nm;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t q = i / nm;
        const int nu = static_cast<int>(i - q * nm);
        const int a2 = static_cast<int>(q % n2), a1 = static_cast<int>((q / n2) % n1),
                  a0 = static_cast<int>(q / (static_cast<int64_t>(n1) * n2));
        const int64_t qm = (static_cast<int64_t>((n0 - a0) % n0) * n1 + (n1 - a1) % n1) * n2 + (n2 - a2) % n2;
        const T v = T(0.5) * (rate[i] + rate[qm * nm + nu]);
        const T x0 = N0[i];
        switch (mode) {
        case EPI_RK1:
            acc[i] = v;
            out[i] = x0 + (dt * T(0.5)) * v;
            break;
        case EPI_RK2:
            acc[i] += T(2) * v;
            out[i] = x0 + (dt * T(0.5)) * v;
            break;
        case EPI_RK3:
            acc[i] += T(2) * v;
            out[i] = x0 + dt * v;
            break;
        default: out[i] = x0 + (dt / T(6)) * (acc[i] + v); break;
        }
    }
}

// Phonon-side rate of the stage input u into rate (the {hw, N} table and its
// max |N| already packed from the stage's N).
template <typename T> PhArgs<T> ph_args(ephbte_plan P) {
    PhArgs<T> a;
    a.pa = P->ph_pa;
    a.pb = P->ph_pb;
    a.g2 = static_cast<const T *>(P->ph_g2);
    a.ld = P->ph_ld;
    a.st = static_cast<const StateRec<T> *>(P->st);
    a.hw = static_cast<const T *>(P->hw);
    a.chunk_beg = P->ph_chunk_beg;
    a.chunk_bucket = P->ph_chunk_bucket;
    a.bucket_chunk = P->ph_bucket_chunk;
    a.bucket_q = P->ph_bucket_q;
    a.bucket_qm = P->ph_bucket_qm;
    a.bucket_modes = P->ph_bucket_modes;
    a.q_bucket = P->ph_q_bucket;
    a.n_chunks = P->ph_nchunks;
    a.nq = static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2];
    a.nm = P->nm;
    a.mc = static_cast<T>(-1.4426950408889634 / (2.0 * P->sigma * P->sigma));
    a.mc256 = 256.0 * (-1.4426950408889634 / (2.0 * P->sigma * P->sigma));
    a.e2tab = P->e2tab;
    a.Kp = 2.0 * kPi / (kHbar * P->nk) / (P->sigma * std::sqrt(2.0 * kPi));
    a.elastic = P->elastic;
    a.chan = P->ph_chan;
    return a;
}

// dN/dt of every (q, mode) bin into rate (the caller ensured P->ph_part)
template <typename T> void enqueue_phonon_rate(ephbte_plan P, const T *u, const T *nph, T *rate, hipStream_t s) {
    const PhArgs<T> a = ph_args<T>(P);
    T *part = static_cast<T *>(P->ph_part.p);
    if (P->ph_nchunks > 0) {
        const dim3 grid(static_cast<unsigned>((P->ph_nchunks + 3) / 4)), block(256);
        auto go = [&](auto nmc) {
            constexpr int NM = decltype(nmc)::value;
            hipLaunchKernelGGL((k_phonon_bins<T, NM>), grid, block, 0, s, a, u, nph, part);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
    }
    const int64_t nbin = a.nq * P->nm;
    const unsigned nf = static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((nbin + 255) / 256, 4096), 1));
    hipLaunchKernelGGL((k_phonon_bins_finish<T>), dim3(nf), dim3(256), 0, s, a, (const T *)part, rate);
    HIPC(hipGetLastError());
}

void ensure_phonon(ephbte_plan P) {
    ensure(P->ph_part, esize(P) * 2 * static_cast<size_t>(P->nm) * std::max<int64_t>(P->ph_nchunks, 1),
           &P->ws_gen);
}

// the electron-side constant of Eq. 2 with the Gaussian's normalisation
double k_electron(ephbte_plan P) {
    return 2.0 * kPi / (kHbar * P->nqnorm) / (P->sigma * std::sqrt(2.0 * kPi));
}

// dL/dN [Nq][n_modes] (overwritten) of L = lam . I + mu . dN/dt at (u, N),
// and the phonon-side part of dL/d|g|^2 added to gg2 (if gg2 and mu are set).
// lam or mu may be null.  The caller ensured P->ph_part.
template <typename T>
void enqueue_phonon_adj(ephbte_plan P, const T *u, const T *N, const T *lam, const T *mu, T *gN, double *gg2,
                        hipStream_t s) {
    PhArgs<T> a = ph_args<T>(P);
    T *part = static_cast<T *>(P->ph_part.p);
    if (P->ph_nchunks > 0) {
        const dim3 grid(static_cast<unsigned>((P->ph_nchunks + 3) / 4)), block(256);
        const double ke = k_electron(P);
        auto go = [&](auto nmc) {
            constexpr int NM = decltype(nmc)::value;
            hipLaunchKernelGGL((k_phonon_bins_adj<T, NM>), grid, block, 0, s, a, u, N, lam, mu, part, gg2, ke);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
    }
    a.Kp = 1.0;   // the partials already carry their constants
    hipLaunchKernelGGL((k_phonon_bins_finish<T>), dim3(grid_of(a.nq * P->nm)), dim3(256), 0, s, a,
                       (const T *)part, gN);
    HIPC(hipGetLastError());
}

// out += dL/df of L = mu . dN/dt at (u, N) (the caller ensured P->ph_tab4 and
// P->part for n_chunks values)
template <typename T>
void enqueue_phonon_vjp_f(ephbte_plan P, const T *u, const T *N, const T *mu, T *out, hipStream_t s) {
    const int64_t n = P->padq ? P->n_used_rows * P->nm : nqm_of(P);
    Vec4<T> *tab = static_cast<Vec4<T> *>(P->ph_tab4.p);
    hipLaunchKernelGGL((k_pack_hwNmu<T>), dim3(grid_of(n)), dim3(256), 0, s, static_cast<const T *>(P->hw), N, mu,
                       tab, P->padq ? 1 : 0, P->qbox, P->nm, (const int32_t *)P->used_rows, n);
    const double Kp = 2.0 * kPi / (kHbar * P->nk) / (P->sigma * std::sqrt(2.0 * kPi));
    if (P->pr_ok && P->pr_all_q && P->sym_ok && P->n_pr_tiles > 0) {
        // over the q-ordered pair records: max |N| and max |mu| of the call
        // set the fixed-point scale
        const int64_t nqm = nqm_of(P);
        // (a few hundred workgroups: fewer atomics on the one word)
        const dim3 gm(std::min<unsigned>(grid_of(nqm), 256u));
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, P->mmax_bits, 2);
        hipLaunchKernelGGL((k_abs_max_bits<T>), gm, dim3(256), 0, s, mu, nqm, P->mmax_bits);
        hipLaunchKernelGGL((k_abs_max_bits<T>), gm, dim3(256), 0, s, N, nqm, P->mmax_bits + 1);
        TiledArgs<T> a = pair_args<T>(P);
        a.nmax_bits = P->mmax_bits + 1;
        const dim3 grid(static_cast<unsigned>(P->n_pr_tiles)), block(1024);
        const size_t shm = sym_lds_bytes(P->dtype, P->pr_lds_states);
        const unsigned long long *mm = P->mmax_bits;
        auto go = [&](auto nmc) {
            constexpr int NM = decltype(nmc)::value;
            if (P->padq)
                hipLaunchKernelGGL((k_vjp_phonon_pairs<T, true, NM>), grid, block, shm, s, a, (const Vec4<T> *)tab, u,
                                   P->elastic, mm);
            else
                hipLaunchKernelGGL((k_vjp_phonon_pairs<T, false, NM>), grid, block, shm, s, a, (const Vec4<T> *)tab,
                                   u, P->elastic, mm);
        };
        if (P->nm <= 1) go(std::integral_constant<int, 1>{});
        else if (P->nm <= 2) go(std::integral_constant<int, 2>{});
        else if (P->nm <= 3) go(std::integral_constant<int, 3>{});
        else if (P->nm <= 4) go(std::integral_constant<int, 4>{});
        else if (P->nm <= 6) go(std::integral_constant<int, 6>{});
        else go(std::integral_constant<int, 8>{});
        hipLaunchKernelGGL((k_vjp_phonon_pairs_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a, mm, Kp,
                           out);
        HIPC(hipGetLastError());
        return;
    }
    TiledArgs<T> a = tiled_args<T>(P);
    T *part = static_cast<T *>(P->part.p);
    if (P->n_chunks > 0)
        hipLaunchKernelGGL((k_vjp_phonon_f<T>), dim3(static_cast<unsigned>(P->n_chunks)), dim3(256), 0, s, a,
                           (const Vec4<T> *)tab, u, P->elastic, Kp, out, part);
    if (!P->fused)
        hipLaunchKernelGGL((k_vjp_phonon_f_finish<T>), dim3((P->S + 255) / 256), dim3(256), 0, s, a,
                           (const T *)part, out);
    HIPC(hipGetLastError());
}

template <typename T> void ensure_phonon_vjp(ephbte_plan P) {
    const int64_t n = P->padq ? P->qpad_n * P->nm : nqm_of(P);
    ensure_zeroed(P, P->ph_tab4, sizeof(Vec4<T>) * static_cast<size_t>(std::max<int64_t>(n, 1)));
    ensure_part<T>(P, 1, 2);
    ensure_phonon(P);
}

template <typename T>
ephbte_status rt_coupled_impl(ephbte_plan P, T *f, T *N, double dt, int n_steps, hipStream_t s) {
    const int64_t S = P->S;
    const int64_t nbin = static_cast<int64_t>(P->nq[0]) * P->nq[1] * P->nq[2] * P->nm;
    const size_t v = sizeof(T) * static_cast<size_t>(S), vn = sizeof(T) * static_cast<size_t>(nbin);
    ensure(P->rk_ua, v, &P->ws_gen);
    ensure(P->rk_ub, v, &P->ws_gen);
    ensure(P->rk_acc, v, &P->ws_gen);
    ensure(P->cp_Ma, vn, &P->ws_gen);
    ensure(P->cp_Mb, vn, &P->ws_gen);
    ensure(P->cp_acc, vn, &P->ws_gen);
    ensure(P->cp_rate, vn, &P->ws_gen);
    ensure_fwd<T>(P, 1);
    ensure_phonon(P);
    T *ua = static_cast<T *>(P->rk_ua.p), *ub = static_cast<T *>(P->rk_ub.p);
    T *acc = static_cast<T *>(P->rk_acc.p);
    T *Ma = static_cast<T *>(P->cp_Ma.p), *Mb = static_cast<T *>(P->cp_Mb.p);
    T *nacc = static_cast<T *>(P->cp_acc.p), *rate = static_cast<T *>(P->cp_rate.p);
    const T tdt = static_cast<T>(dt);
    const unsigned ng = static_cast<unsigned>(std::max<int64_t>(std::min<int64_t>((nbin + 255) / 256, 4096), 1));
    for (int k = 0; k < n_steps; ++k) {
        // stage inputs (u, M): (f, N), (ua, Ma), (ub, Mb), (ua, Ma); outputs to
        // (ua, Ma), (ub, Mb), (ua, Ma) and finally (f, N)
        const T *uin[4] = {f, ua, ub, ua};
        const T *min_[4] = {N, Ma, Mb, Ma};
        T *uout[4] = {ua, ub, ua, nullptr};
        T *mout[4] = {Ma, Mb, Ma, N};
        for (int st = 0; st < 4; ++st) {
            enqueue_pack<T>(P, min_[st], s);
            Epi<T> e{};
            e.f0 = f;
            e.ld_f0 = S;
            e.acc = acc;
            e.dt = tdt;
            e.mode = EPI_RK1 + st;
            e.u_out = uout[st];
            e.f_out = f;
            enqueue_forward<T>(P, 1, uin[st], S, min_[st], e, s, false);
            enqueue_phonon_rate<T>(P, uin[st], min_[st], rate, s);
            hipLaunchKernelGGL((k_rk_even<T>), dim3(ng), dim3(256), 0, s, EPI_RK1 + st, (const T *)N,
                               (const T *)rate, nacc, mout[st], tdt, P->nq[0], P->nq[1], P->nq[2], P->nm);
            HIPC(hipGetLastError());
        }
    }
    return EPHBTE_OK;
}

// One coupled RK4 step whose four stage inputs (u, M) are kept: stage k reads
// U[k], M[k] (k = 0 .. 3) and writes the next stage input to U[k + 1], M[k + 1];
// the last stage writes f_next, N_next.  Same arithmetic as rt_coupled_impl.
template <typename T>
void coupled_step_stages(ephbte_plan P, T *const U[4], T *const M[4], T *f_next, T *N_next, T dt, hipStream_t s) {
    const int64_t S = P->S;
    T *acc = static_cast<T *>(P->rk_acc.p);
    T *nacc = static_cast<T *>(P->cp_acc.p), *rate = static_cast<T *>(P->cp_rate.p);
    const int64_t nbin = nqm_of(P);
    for (int st = 0; st < 4; ++st) {
        enqueue_pack<T>(P, M[st], s);
        Epi<T> e{};
        e.f0 = U[0];
        e.ld_f0 = S;
        e.acc = acc;
        e.dt = dt;
        e.mode = EPI_RK1 + st;
        e.u_out = st < 3 ? U[st + 1] : nullptr;
        e.f_out = f_next;
        enqueue_forward<T>(P, 1, U[st], S, M[st], e, s, false);
        enqueue_phonon_rate<T>(P, U[st], M[st], rate, s);
        hipLaunchKernelGGL((k_rk_even<T>), dim3(grid_of(nbin)), dim3(256), 0, s, EPI_RK1 + st, (const T *)M[0],
                           (const T *)rate, nacc, st < 3 ? M[st + 1] : N_next, dt, P->nq[0], P->nq[1], P->nq[2],
                           P->nm);
        HIPC(hipGetLastError());
    }
}

// Discrete adjoint of n coupled RK4 steps from (f0, N0), checkpointed every
// ce steps (stage inputs recomputed inside a segment).  Per stage (u, M) with
// adjoint pair (a, b), the transposed Jacobian of (I, E R) gives
//   u-bar = J_If^T a + J_Rf^T E b,  M-bar = J_IN^T a + J_RN^T E b,
//   |g|^2-bar += J_Ig^T a + J_Rg^T E b,
// and the four stages combine as in rt_adjoint_impl.
template <typename T>
ephbte_status rt_adjoint_coupled_impl(ephbte_plan P, const T *f0, const T *N0, double dt, int n, int ce,
                                      const T *gfT, const T *gNT, T *gf0, T *gN0, double *gg2, int accumulate,
                                      hipStream_t s) {
    const int64_t S = P->S, nb = nqm_of(P);
    const size_t v = sizeof(T) * S, vn = sizeof(T) * nb;
    const int nck = std::max(1, (n + ce - 1) / ce);
    ensure(P->rk_acc, v, &P->ws_gen);
    ensure(P->cp_acc, vn, &P->ws_gen);
    ensure(P->cp_rate, vn, &P->ws_gen);
    ensure(P->ca_ckf, v * nck, &P->ws_gen);
    ensure(P->ca_ckN, vn * nck, &P->ws_gen);
    ensure(P->ca_U, v * (4 * static_cast<size_t>(ce) + 1), &P->ws_gen);
    ensure(P->ca_M, vn * (4 * static_cast<size_t>(ce) + 1), &P->ws_gen);
    for (DevBuf *b : {&P->ca_gf, &P->ca_a, &P->ca_uf, &P->ca_sf}) ensure(*b, v, &P->ws_gen);
    for (DevBuf *b : {&P->ca_gN, &P->ca_b, &P->ca_uN, &P->ca_sN, &P->ca_mu}) ensure(*b, vn, &P->ws_gen);
    ensure_fwd<T>(P, 1);
    ensure_phonon_vjp<T>(P);
    T *ckf = static_cast<T *>(P->ca_ckf.p), *ckN = static_cast<T *>(P->ca_ckN.p);
    T *U = static_cast<T *>(P->ca_U.p), *M = static_cast<T *>(P->ca_M.p);
    T *gf = static_cast<T *>(P->ca_gf.p), *gN = static_cast<T *>(P->ca_gN.p);
    T *a = static_cast<T *>(P->ca_a.p), *b = static_cast<T *>(P->ca_b.p);
    T *uf = static_cast<T *>(P->ca_uf.p), *uN = static_cast<T *>(P->ca_uN.p);
    T *sf = static_cast<T *>(P->ca_sf.p), *sN = static_cast<T *>(P->ca_sN.p);
    T *mu = static_cast<T *>(P->ca_mu.p);
    const T tdt = static_cast<T>(dt);
    auto copy = [&](T *dst, const T *src, int64_t cnt) {
        hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(cnt)), dim3(256), 0, s, cnt, T(1), src, T(0),
                           (const T *)nullptr, dst);
    };
    auto stage_ptrs = [&](int64_t l, T *Ul[4], T *Ml[4]) {
        for (int k = 0; k < 4; ++k) {
            Ul[k] = U + (l * 4 + k) * S;
            Ml[k] = M + (l * 4 + k) * nb;
        }
    };
    // forward sweep: checkpoints of (f, N) every ce steps
    copy(U, f0, S);
    copy(M, N0, nb);
    for (int k = 0; k < n; ++k) {
        if (k % ce == 0) {
            copy(ckf + static_cast<int64_t>(k / ce) * S, U, S);
            copy(ckN + static_cast<int64_t>(k / ce) * nb, M, nb);
        }
        T *Ul[4], *Ml[4];
        stage_ptrs(0, Ul, Ml);
        coupled_step_stages<T>(P, Ul, Ml, U, M, tdt, s);
    }
    if (gfT) copy(gf, gfT, S);
    else hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(S)), dim3(256), 0, s, S, T(0), (const T *)U, T(0),
                            (const T *)nullptr, gf);
    if (gNT) copy(gN, gNT, nb);
    else hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(nb)), dim3(256), 0, s, nb, T(0), (const T *)M, T(0),
                            (const T *)nullptr, gN);
    const int gmode = gg2 ? 2 : 0;
    if (gg2 && !accumulate) hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, s, gg2, P->nch, 0.0);
    HIPC(hipGetLastError());
    // (cg, cv) of the stages 4, 3, 2, 1: a_k = cg gbar + cv u-bar_{k+1}
    const T cg[4] = {tdt / T(6), tdt / T(3), tdt / T(3), tdt / T(6)};
    const T cv[4] = {T(0), tdt, tdt / T(2), tdt / T(2)};
    for (int m = nck - 1; m >= 0; --m) {
        const int s0 = m * ce, s1 = std::min(n, s0 + ce);
        copy(U, ckf + static_cast<int64_t>(m) * S, S);
        copy(M, ckN + static_cast<int64_t>(m) * nb, nb);
        for (int k = s0; k < s1; ++k) {
            T *Ul[4], *Ml[4];
            stage_ptrs(k - s0, Ul, Ml);
            coupled_step_stages<T>(P, Ul, Ml, U + (static_cast<int64_t>(k - s0) + 1) * 4 * S,
                                   M + (static_cast<int64_t>(k - s0) + 1) * 4 * nb, tdt, s);
        }
        for (int k = s1 - 1; k >= s0; --k) {
            T *Ul[4], *Ml[4];
            stage_ptrs(k - s0, Ul, Ml);
            copy(sf, gf, S);
            copy(sN, gN, nb);
            for (int r = 0; r < 4; ++r) {
                const int st = 3 - r;
                hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(S)), dim3(256), 0, s, S, cg[r], (const T *)gf, cv[r],
                                   r ? (const T *)uf : nullptr, a);
                hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(nb)), dim3(256), 0, s, nb, cg[r], (const T *)gN,
                                   cv[r], r ? (const T *)uN : nullptr, b);
                // electron side: u-bar = J_If^T a, and J_Ig^T a into gg2
                enqueue_pack<T>(P, Ml[st], s);
                enqueue_vjp<T>(P, Ul[st], a, Ml[st], epi_store<T>(uf, S), gg2, gmode, s);
                // phonon side through the even part: mu = E b
                hipLaunchKernelGGL((k_even_q<T>), dim3(grid_of(nb)), dim3(256), 0, s, (const T *)b, mu, P->nq[0],
                                   P->nq[1], P->nq[2], P->nm);
                enqueue_phonon_vjp_f<T>(P, Ul[st], Ml[st], mu, uf, s);
                enqueue_phonon_adj<T>(P, Ul[st], Ml[st], a, mu, uN, gg2, s);
                hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(S)), dim3(256), 0, s, S, T(1), (const T *)sf, T(1),
                                   (const T *)uf, sf);
                hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(nb)), dim3(256), 0, s, nb, T(1), (const T *)sN, T(1),
                                   (const T *)uN, sN);
                HIPC(hipGetLastError());
            }
            copy(gf, sf, S);
            copy(gN, sN, nb);
        }
    }
    if (gf0) copy(gf0, gf, S);
    if (gN0) copy(gN0, gN, nb);
    HIPC(hipGetLastError());
    return EPHBTE_OK;
}

// iterations without a new smallest relative change after which the
// transport iteration stops at its precision floor
constexpr int kStall = 5;

template <typename T>
ephbte_status transport_impl(ephbte_plan P, const T *f0, const T *vel, double T_K,
                             const void *nph, double tol, int max_iter, T *x_out, double *mob,
                             int32_t *iters, double *resid, hipStream_t s) {
    const int64_t S = P->S;
    ensure(P->tr_W, sizeof(T) * (P->E + kEntryPad), &P->ws_gen);
    ensure(P->tr_tau_inv, sizeof(T) * S, &P->ws_gen);
    ensure(P->tr_tau, sizeof(T) * S, &P->ws_gen);
    ensure(P->tr_rhs, sizeof(Vec4<T>) * S, &P->ws_gen);
    ensure(P->tr_xa, sizeof(Vec4<T>) * S, &P->ws_gen);
    ensure(P->tr_xb, sizeof(Vec4<T>) * S, &P->ws_gen);
    ensure(P->tr_part, sizeof(Vec4<T>) * std::max<int64_t>(P->n_chunks, 1), &P->ws_gen);
    ensure(P->tr_red, sizeof(double) * 10 * kRedBlocks, &P->ws_gen);
    ensure(P->tr_red2, sizeof(double) * 10, &P->ws_gen);
    if (!P->host_red) HIPC(hipHostMalloc(reinterpret_cast<void **>(&P->host_red), sizeof(double) * 10, 0));
    Tables<T> t = tables<T>(P, nph);
    T *W = static_cast<T *>(P->tr_W.p), *tinv = static_cast<T *>(P->tr_tau_inv.p);
    T *tau = static_cast<T *>(P->tr_tau.p);
    Vec4<T> *rhs = static_cast<Vec4<T> *>(P->tr_rhs.p);
    Vec4<T> *xa = static_cast<Vec4<T> *>(P->tr_xa.p), *xb = static_cast<Vec4<T> *>(P->tr_xb.p);
    Vec4<T> *part = static_cast<Vec4<T> *>(P->tr_part.p);
    double *red = static_cast<double *>(P->tr_red.p), *red2 = static_cast<double *>(P->tr_red2.p);
    dim3 grid(static_cast<unsigned>(grid_x(P))), block(P->block_threads);
    dim3 sg((S + 255) / 256);
    if (P->fused)
        hipLaunchKernelGGL((k_transport_setup<T, true>), grid, block, 0, s, t, f0, W, (T *)nullptr,
                           tinv);
    else {
        hipLaunchKernelGGL((k_transport_setup<T, false>), grid, block, 0, s, t, f0, W,
                           reinterpret_cast<T *>(part), tinv);
        hipLaunchKernelGGL((k_transport_setup_finish<T>), sg, dim3(256), 0, s, t,
                           (const T *)reinterpret_cast<T *>(part), tinv);
    }
    hipLaunchKernelGGL((k_transport_prep<T>), sg, dim3(256), 0, s, f0, vel, (const T *)tinv,
                       static_cast<T>(1.0 / (kKb * T_K)), (int)S, tau, rhs, xa);
    HIPC(hipGetLastError());
    auto mobility = [&](const Vec4<T> *x, bool with_f0, double out[10]) {
        hipLaunchKernelGGL((k_mobility_partial<T>), dim3(kRedBlocks), dim3(256), 0, s, vel, x,
                           with_f0 ? f0 : (const T *)nullptr, (int)S, red);
        hipLaunchKernelGGL(k_rows_sum10, dim3(1), dim3(256), 0, s, (const double *)red,
                           kRedBlocks, red2);
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(P->host_red, red2, sizeof(double) * 10, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        std::memcpy(out, P->host_red, sizeof(double) * 10);
    };
    double r0[10];
    mobility(xa, true, r0);
    const double sum_f0 = r0[9];
    if (!(sum_f0 > 0.0)) throw HipError{hipErrorInvalidValue, "sum of f0 is not positive"};
    const double unit = -1e-15 * 1e4 / sum_f0;   // fs -> s, m^2 -> cm^2, e = 1
    double mu[9];
    for (int k = 0; k < 9; ++k) mu[k] = unit * r0[k];
    double rel = INFINITY, best = INFINITY;
    int it = 0, since_best = 0;
    bool conv = false, stalled = false;
    for (it = 1; it <= max_iter; ++it) {
        {
            TiledArgs<T> ta = tiled_args<T>(P);
            ta.xcd = 0;
            // half-size tiles: measured 3 % faster than the forward's here
            ta.tiles = P->small_tiles;
            ta.n_tiles = P->n_small_tiles;
            const size_t shm = static_cast<size_t>(P->lds_states) * 3 * sizeof(T);
            const int use_lds = shm <= P->lds_max ? 1 : 0;
            hipLaunchKernelGGL((k_tr_tiled<T>), dim3(static_cast<unsigned>(P->n_small_tiles)),
                               dim3(P->block_threads), use_lds ? shm : 0, s, ta, use_lds,
                               (const T *)W, (const Vec4<T> *)xa, (const Vec4<T> *)rhs,
                               (const T *)tau, part, xb);
            if (!P->fused)
                hipLaunchKernelGGL((k_tr_tiled_finish<T>), sg, dim3(256), 0, s, ta,
                                   (const Vec4<T> *)part, (const Vec4<T> *)rhs, (const T *)tau, xb);
        }
        HIPC(hipGetLastError());
        double r[10];
        mobility(xb, false, r);
        double num = 0.0, den = 0.0, nm[9];
        for (int k = 0; k < 9; ++k) {
            nm[k] = unit * r[k];
            num = std::max(num, std::fabs(nm[k] - mu[k]));
            den = std::max(den, std::fabs(nm[k]));
        }
        rel = den > 0 ? num / den : 0.0;
        std::memcpy(mu, nm, sizeof(mu));
        std::swap(xa, xb);
        if (rel <= tol) {
            conv = true;
            break;
        }
        // the working precision's floor: no new smallest change in kStall iterations
        if (rel < best) {
            best = rel;
            since_best = 0;
        } else if (++since_best >= kStall) {
            stalled = true;
            break;
        }
    }
    if (it > max_iter) it = max_iter;
    if (x_out) {
        hipLaunchKernelGGL((k_unpack_x<T>), sg, dim3(256), 0, s, (const Vec4<T> *)xa, x_out, (int)S);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));
    }
    std::memcpy(mob, mu, sizeof(mu));
    if (iters) *iters = it;
    if (resid) *resid = rel;
    if (stalled)
        return fail(EPHBTE_NOT_CONVERGED,
                    "transport iteration stagnated: the relative change stopped decreasing above "
                    "the tolerance (the working precision's floor)");
    if (!conv) return fail(EPHBTE_NOT_CONVERGED, "transport iteration did not reach the tolerance");
    return EPHBTE_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// Orders this call's work after the previous call on the plan (if that ran
// on another stream) and records completion for the next call.
struct PlanUse {
    ephbte_plan P;
    hipStream_t s;
    bool active = false;
    PlanUse(ephbte_plan p, hipStream_t st) : P(p), s(st) {
        if (capturing(s)) return;
        if (!P->ev_last) HIPC(hipEventCreateWithFlags(&P->ev_last, hipEventDisableTiming));
        if (P->has_last && P->last_stream != s) HIPC(hipStreamWaitEvent(s, P->ev_last, 0));
        active = true;
    }
    void done() {
        if (!active) return;
        HIPC(hipEventRecord(P->ev_last, s));
        P->last_stream = s;
        P->has_last = true;
    }
};

template <typename F> ephbte_status guarded(ephbte_plan P, void *stream, F &&fn) {
    if (!P) return fail(EPHBTE_INVALID_ARGUMENT, "plan is NULL");
    try {
        DeviceGuard g(P->device);
        PlanUse use(P, static_cast<hipStream_t>(stream));
        ephbte_status st = fn();
        use.done();
        return st;
    } catch (const HipError &e) {
        return fail(EPHBTE_HIP_ERROR, std::string(e.where) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc &) {
        return fail(EPHBTE_OUT_OF_MEMORY, "device or host memory allocation failed");
    } catch (...) {
        return fail(EPHBTE_HIP_ERROR, "unexpected exception");
    }
}

// ---------------------------------------------------------------- autotune cache
// A JSON object mapping a plan key to the tuning chosen for it:
//   {"<key>": {"chunk_entries": 65536, "block_threads": 512, ...}, ...}
using TuneEntry = std::map<std::string, long long>;
using TuneCache = std::map<std::string, TuneEntry>;

// 1: parsed, 0: no file, -1: not a cache of this form
int read_tune_cache(const char *path, TuneCache &out) {
    std::ifstream in(path, std::ios::binary);
    if (!in) return 0;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    auto ws = [&]() { while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i; };
    auto str = [&](std::string &o) -> bool {
        ws();
        if (i >= t.size() || t[i] != '"') return false;
        ++i;
        o.clear();
        while (i < t.size() && t[i] != '"') {
            if (t[i] == '\\') return false;   // keys and names are written without escapes
            o += t[i++];
        }
        if (i >= t.size()) return false;
        ++i;
        return true;
    };
    auto ch = [&](char c) -> bool {
        ws();
        if (i < t.size() && t[i] == c) {
            ++i;
            return true;
        }
        return false;
    };
    auto num = [&](long long &v) -> bool {
        ws();
        const size_t b = i;
        if (i < t.size() && t[i] == '-') ++i;
        while (i < t.size() && std::isdigit(static_cast<unsigned char>(t[i]))) ++i;
        if (i == b || (i == b + 1 && t[b] == '-')) return false;
        v = std::stoll(t.substr(b, i - b));
        return true;
    };
    if (!ch('{')) return -1;
    if (ch('}')) return 1;
    do {
        std::string key;
        if (!str(key) || !ch(':') || !ch('{')) return -1;
        TuneEntry e;
        if (!ch('}')) {
            do {
                std::string name;
                long long v;
                if (!str(name) || !ch(':') || !num(v)) return -1;
                e[name] = v;
            } while (ch(','));
            if (!ch('}')) return -1;
        }
        out[key] = e;
    } while (ch(','));
    if (!ch('}')) return -1;
    ws();
    return i == t.size() ? 1 : -1;
}

bool write_tune_cache(const char *path, const TuneCache &c) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::binary | std::ios::trunc);
        if (!o) return false;
        o << "{\n";
        size_t k = 0;
        for (const auto &kv : c) {
            o << "  \"" << kv.first << "\": {";
            size_t n = 0;
            for (const auto &f : kv.second) o << (n++ ? ", " : "") << "\"" << f.first << "\": " << f.second;
            o << "}" << (++k < c.size() ? "," : "") << "\n";
        }
        o << "}\n";
        if (!o) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

std::string tune_key(ephbte_plan P, int batch) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == '"' || c == '\\') c = '_';
    std::ostringstream k;
    k << arch << "|cu=" << P->n_cu << "|" << (P->dtype == EPHBTE_F64 ? "f64" : "f32") << "|S=" << P->S
      << "|E=" << P->E << "|modes=" << P->nm << "|q=" << P->nq[0] << "x" << P->nq[1] << "x" << P->nq[2]
      << "|" << (batch >= P->batch_min ? "batched" : "single");
    return k.str();
}

}  // namespace

// =================================================================== C ABI
// Bose plans.  With the blocking factors (1 + n) in place of (1 - f), every
// term of Eq. 2 at occupations n is minus the Fermi term at f = -n, so
// I_B(n) = -I_F(-n): the entry points run the Fermi kernels on -n and negate
// what comes back (gradients follow by the chain rule, see each entry point).
template <typename T>
const T *boson_neg(ephbte_plan P, DevBuf &buf, const void *src, int64_t lds, int B, hipStream_t s) {
    ensure(buf, sizeof(T) * static_cast<size_t>(P->S) * B, &P->ws_gen);
    T *dst = static_cast<T *>(buf.p);
    hipLaunchKernelGGL((k_neg_rows<T>), dim3(grid_of(static_cast<int64_t>(P->S) * B)), dim3(256), 0, s,
                       static_cast<const T *>(src), lds, dst, int64_t(P->S), B, P->S);
    return dst;
}
template <typename T> void neg_in_place(ephbte_plan P, void *x, int64_t ld, int B, hipStream_t s) {
    T *p = static_cast<T *>(x);
    hipLaunchKernelGGL((k_neg_rows<T>), dim3(grid_of(static_cast<int64_t>(P->S) * B)), dim3(256), 0, s,
                       (const T *)p, ld, p, ld, B, P->S);
}

ephbte_status boson_unsupported(const char *what) {
    return fail(EPHBTE_INVALID_ARGUMENT,
                std::string(what) + " is defined for Fermi statistics only (this plan was built with statistics = 1)");
}

extern "C" {

const char *ephbte_status_string(ephbte_status s) {
    switch (s) {
    case EPHBTE_OK: return "ok";
    case EPHBTE_INVALID_ARGUMENT: return "invalid argument";
    case EPHBTE_UNSUPPORTED_DTYPE: return "unsupported dtype";
    case EPHBTE_OUT_OF_MEMORY: return "out of memory";
    case EPHBTE_HIP_ERROR: return "HIP error";
    case EPHBTE_NOT_CONVERGED: return "not converged";
    case EPHBTE_NONFINITE: return "non-finite value";
    case EPHBTE_PLAN_MISMATCH: return "plan mismatch";
    default: return "unknown status";
    }
}

const char *ephbte_last_error(void) { return g_last_error.c_str(); }

ephbte_status ephbte_layout_host(const ephbte_problem *problem, const ephbte_build_opts *opts,
                                 int64_t *row_ptr, int32_t *entry_partner, int8_t *entry_mode,
                                 int32_t *entry_channel) {
    try {
        HostLayout L;
        std::string err;
        ephbte_status st = build_host_layout(problem, opts, &L, &err);
        if (st != EPHBTE_OK) return fail(st, err);
        if (row_ptr) std::memcpy(row_ptr, L.row_ptr.data(), sizeof(int64_t) * (L.S + 1));
        for (int64_t e = 0; e < L.E; ++e) {
            if (entry_partner) entry_partner[e] = static_cast<int32_t>(L.pnu[e] >> 3);
            if (entry_mode) entry_mode[e] = static_cast<int8_t>(L.pnu[e] & 7u);
            if (entry_channel) entry_channel[e] = L.ent_chan[e];
        }
        return EPHBTE_OK;
    } catch (const std::bad_alloc &) {
        return fail(EPHBTE_OUT_OF_MEMORY, "host memory allocation failed");
    } catch (...) {
        return fail(EPHBTE_INVALID_ARGUMENT, "unexpected exception while building the layout");
    }
}

ephbte_status ephbte_build_channels(const ephbte_problem *problem, const ephbte_build_opts *opts,
                                    ephbte_plan *out) {
    if (!out) return fail(EPHBTE_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    HostLayout L;
    std::string err;
    try {
        ephbte_status st = build_host_layout(problem, opts, &L, &err);
        if (st != EPHBTE_OK) return fail(st, err);
    } catch (const std::bad_alloc &) {
        return fail(EPHBTE_OUT_OF_MEMORY, "host memory allocation failed");
    }
    ephbte_plan P = new (std::nothrow) ephbte_plan_s();
    if (!P) return fail(EPHBTE_OUT_OF_MEMORY, "host memory allocation failed");
    try {
        int dev = problem->device;
        if (dev < 0) HIPC(hipGetDevice(&dev));
        int ndev = 0;
        HIPC(hipGetDeviceCount(&ndev));
        if (dev >= ndev) {
            delete P;
            return fail(EPHBTE_INVALID_ARGUMENT, "device ordinal out of range");
        }
        P->device = dev;
        DeviceGuard g(dev);
        // set-up of this device: the address of its copy of the allocation-free
        // pass's scratch, and the event that orders consecutive calls on the plan
        (void)scratch_base(dev);
        HIPC(hipEventCreateWithFlags(&P->ev_last, hipEventDisableTiming));
        P->dtype = problem->dtype;
        P->S = L.S;
        P->nm = L.n_modes;
        P->nch = L.n_input;
        P->nch_kept = L.n_channels;
        P->E = L.E;
        P->elastic = opts ? opts->elastic_modes : 0u;
        P->boson = opts && opts->statistics == 1;
        P->nk = static_cast<double>(problem->kgrid[0]) * problem->kgrid[1] * problem->kgrid[2];
        P->nbr_ok = !L.nbr.empty();
        if (P->nbr_ok) {
            dalloc(P->nbr, sizeof(int32_t) * L.nbr.size(), &P->layout_bytes);
            HIPC(hipMemcpy(P->nbr, L.nbr.data(), sizeof(int32_t) * L.nbr.size(), hipMemcpyHostToDevice));
        }
        P->n_drop = static_cast<int64_t>(L.dropped.size());
        if (P->n_drop > 0) {
            dalloc(P->drop_idx, sizeof(int32_t) * P->n_drop, &P->layout_bytes);
            HIPC(hipMemcpy(P->drop_idx, L.dropped.data(), sizeof(int32_t) * P->n_drop,
                           hipMemcpyHostToDevice));
        }
        for (int a = 0; a < 3; ++a) P->nq[a] = L.nq[a];
        P->sigma = problem->sigma;
        P->nqnorm = problem->n_q_norm;
        {
            int span[3];
            q_box_of(L, P->qorg, span);
            int64_t rows = 1;
            for (int a = 0; a < 3; ++a) {
                P->qbox.n[a] = L.nq[a];
                P->qbox.b[a] = 2 * span[a] - 1;
                P->qbox.h[a] = span[a] - 1;
                rows *= P->qbox.b[a];
            }
            const size_t pair_bytes = P->dtype == EPHBTE_F64 ? 16 : 8;
            if (rows * L.n_modes * static_cast<int64_t>(pair_bytes) <= (int64_t(256) << 20)) {
                P->padq = true;
                P->qpad_n = rows;
                P->qoff = (P->qbox.h[0] * P->qbox.b[1] + P->qbox.h[1]) * P->qbox.b[2] + P->qbox.h[2];
            }
        }
        P->row_ptr = L.row_ptr;
        P->pmin = L.pmin;
        P->pmax = L.pmax;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            ncu > 0)
            P->n_cu = ncu;
        // LDS window per workgroup: {eps, f} + packed k = 20 B (FP64) / 12 B (FP32) per
        // state, kept under 64 KB so two (FP64) or three (FP32) workgroups share a CU
        P->lds_states = P->dtype == EPHBTE_F64 ? 3072 : 4096;
        int shm = 0;
        if (hipDeviceGetAttribute(&shm, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            shm > 0)
            P->lds_max = static_cast<size_t>(shm);
        if (P->dtype == EPHBTE_F64) {
            upload_layout<double>(P, problem, L);
            upload_phonon_layout<double>(P, problem, L);
            upload_pair_rows<double>(P, problem, L);
        } else {
            upload_layout<float>(P, problem, L);
            upload_phonon_layout<float>(P, problem, L);
            upload_pair_rows<float>(P, problem, L);
        }
        {
            // 2^(j/256) rounded from extended precision
            double tab[kExpTab];
            for (int j = 0; j < kExpTab; ++j)
                tab[j] = static_cast<double>(std::exp2(static_cast<long double>(j) / kExpTab));
            dalloc(P->e2tab, sizeof(tab), &P->layout_bytes);
            HIPC(hipMemcpy(P->e2tab, tab, sizeof(tab), hipMemcpyHostToDevice));
        }
        {
            // single-copy pass: the part p > d of each row (entries are sorted by
            // partner inside a row, so it is a suffix) and its partner range
            P->upper_beg.resize(P->S);
            P->pmin_up.resize(P->S);
            P->pmax_up.resize(P->S);
            parallel_ranges(P->S, host_threads(), [&](int, int64_t b, int64_t e) {
                for (int64_t d = b; d < e; ++d) {
                    const auto lo = L.pnu.begin() + L.row_ptr[d], hi = L.pnu.begin() + L.row_ptr[d + 1];
                    const auto u = std::lower_bound(lo, hi, static_cast<uint32_t>(d + 1) << 3);
                    P->upper_beg[d] = u - L.pnu.begin();
                    const bool has = u != hi;
                    P->pmin_up[d] = has ? static_cast<int32_t>(*u >> 3) : 1;
                    P->pmax_up[d] = has ? L.pmax[d] : 0;
                }
            });
            P->sym_lds_states = P->dtype == EPHBTE_F64 ? 3072 : 4096;
            P->pr_lds_states = P->sym_lds_states;
            P->sym_ok = sym_lds_bytes(P->dtype, P->sym_lds_states) <= P->lds_max;
            if (P->sym_ok && P->pr_ok) P->layout = 3;
            dalloc(P->jacc, sizeof(unsigned long long) * std::max(P->S, 1), &P->layout_bytes);
            HIPC(hipMemset(P->jacc, 0, sizeof(unsigned long long) * std::max(P->S, 1)));
            dalloc(P->nmax_bits, sizeof(unsigned long long), &P->layout_bytes);
            dalloc(P->gmax_bits, sizeof(unsigned long long), &P->layout_bytes);
            dalloc(P->pack_bmax, sizeof(double) * kPackBlocks, &P->layout_bytes);
            dalloc(P->lmax_bits, sizeof(unsigned long long), &P->layout_bytes);
            dalloc(P->mmax_bits, 2 * sizeof(unsigned long long), &P->layout_bytes);
            dalloc(P->fmax_bits, sizeof(unsigned long long), &P->layout_bytes);
            HIPC(hipMemset(P->nmax_bits, 0, sizeof(unsigned long long)));
            HIPC(hipMemset(P->fmax_bits, 0, sizeof(unsigned long long)));
        }
        { HostLayout tmp; std::swap(tmp, L); }
        P->block_threads = 512;
        upload_chunks(P, 65536);
        upload_btiles(P, P->dtype == EPHBTE_F64 ? 96 : 192);
        upload_vjp_btiles(P, vjp_default_pt(P));
        update_gmax(P, nullptr);
        HIPC(hipDeviceSynchronize());
    } catch (const HipError &e) {
        free_plan(P);
        return fail(EPHBTE_HIP_ERROR, std::string(e.where) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc &) {
        free_plan(P);
        return fail(EPHBTE_OUT_OF_MEMORY, "device or host memory allocation failed");
    }
    *out = P;
    return EPHBTE_OK;
}

ephbte_status ephbte_collision_integral(ephbte_plan plan, int32_t batch, const void *f,
                                        int64_t ldf, const void *nph, int32_t nph_per_batch,
                                        void *I, int64_t ldi, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (batch < 1 || batch > 65535) return fail(EPHBTE_INVALID_ARGUMENT, "batch must be in [1, 65535]");
        if (!f || !nph || !I) return fail(EPHBTE_INVALID_ARGUMENT, "f, nph and I must be non-NULL");
        if (ldf < plan->S || ldi < plan->S)
            return fail(EPHBTE_INVALID_ARGUMENT, "ldf and ldi must be >= n_states");
        const size_t es = esize(plan);
        if (overlaps(f, es * ldf * batch, I, es * ldi * batch))
            return fail(EPHBTE_INVALID_ARGUMENT, "I must not overlap f");
        hipStream_t s = as_stream(stream);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            const T *ft = static_cast<const T *>(f);
            int64_t ldft = ldf;
            T *It = static_cast<T *>(I);
            if (plan->boson) {   // I_B(n) = -I_F(-n)
                ft = boson_neg<T>(plan, plan->bs_x, f, ldf, batch, s);
                ldft = plan->S;
            }
            if (!nph_per_batch || batch == 1) {
                ensure_fwd<T>(plan, batch);
                enqueue_forward<T>(plan, batch, ft, ldft, nph, epi_store<T>(It, ldi), s);
            } else if (batch >= plan->batch_min && plan->n_btiles > 0 && pv_table_fits(plan)) {
                // a bath per vector, batched: the table's hw from the first bath's pack
                ensure_fwd<T>(plan, batch);
                enqueue_pack<T>(plan, nph, s);
                enqueue_forward_batched_pv<T>(plan, batch, ft, ldft, static_cast<const T *>(nph), It, ldi, s);
            } else {
                // one bath per vector: the {hw, N} table differs per vector, so
                // each vector is a single-vector pass after its own pack
                ensure_fwd<T>(plan, 1);
                const int64_t tab = nqm_of(plan);
                for (int b = 0; b < batch; ++b)
                    enqueue_forward<T>(plan, 1, ft + b * ldft, ldft, static_cast<const T *>(nph) + b * tab,
                                       epi_store<T>(It + b * ldi, ldi), s);
            }
            if (plan->boson) neg_in_place<T>(plan, It, ldi, batch, s);
        };
        if (plan->dtype == EPHBTE_F64) run(double{});
        else run(float{});
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_collision_integral_noalloc(ephbte_plan plan, const void *f, const void *nph,
                                                void *I, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (!f || !nph || !I) return fail(EPHBTE_INVALID_ARGUMENT, "f, nph and I must be non-NULL");
        if (plan->boson) return boson_unsupported("the allocation-free pass");
        const size_t es = esize(plan);
        if (overlaps(f, es * plan->S, I, es * plan->S))
            return fail(EPHBTE_INVALID_ARGUMENT, "I must not overlap f");
        const size_t need = noalloc_bytes(plan);
        if (need > kScratchBytes)
            return fail(EPHBTE_INVALID_ARGUMENT,
                        "the allocation-free pass needs " + std::to_string(need) +
                            " bytes of scratch for this plan; it holds " + std::to_string(kScratchBytes));
        unsigned char *base = static_cast<unsigned char *>(scratch_base(plan->device));
        hipStream_t s = as_stream(stream);
        if (plan->dtype == EPHBTE_F64)
            enqueue_forward_noalloc<double>(plan, static_cast<const double *>(f), nph, static_cast<double *>(I),
                                            base, s);
        else
            enqueue_forward_noalloc<float>(plan, static_cast<const float *>(f), nph, static_cast<float *>(I), base,
                                           s);
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_collision_vjp(ephbte_plan plan, int32_t batch, const void *f_in, int64_t ldf_in,
                                   const void *nph, int32_t nph_per_batch, const void *gI_in,
                                   int64_t ldg_in, void *gf, int64_t ldgf, double *gg2,
                                   int32_t accumulate_gg2, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        const void *f = f_in, *gI = gI_in;
        const int64_t ldf = ldf_in, ldg = ldg_in;
        if (batch < 1 || batch > 65535) return fail(EPHBTE_INVALID_ARGUMENT, "batch must be in [1, 65535]");
        if (!f || !nph || !gI) return fail(EPHBTE_INVALID_ARGUMENT, "f, nph and gI must be non-NULL");
        if (ldf < plan->S || ldg < plan->S || (gf && ldgf < plan->S))
            return fail(EPHBTE_INVALID_ARGUMENT, "leading dimensions must be >= n_states");
        const size_t es = esize(plan);
        if (gf && (overlaps(gf, es * ldgf * batch, f, es * ldf * batch) ||
                   overlaps(gf, es * ldgf * batch, gI, es * ldg * batch)))
            return fail(EPHBTE_INVALID_ARGUMENT, "gf must not overlap f or gI");
        if (!gf && !gg2) return EPHBTE_OK;
        hipStream_t s = as_stream(stream);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            ensure_part<T>(plan, 1, 1);
            ensure_fwd<T>(plan, 1);
            const int64_t S = plan->S, tab = nqm_of(plan);
            const bool per_batch = nph_per_batch && batch > 1;
            const void *f = f_in, *gI = gI_in;
            int64_t ldf = ldf_in, ldg = ldg_in;
            if (plan->boson) {
                // L = sum lam I_B(n) = sum (-lam) I_F(-n): the Fermi pass on
                // (-n, -lam) gives dL/d|g|^2 as it is and -dL/dn
                f = boson_neg<T>(plan, plan->bs_x, f_in, ldf_in, batch, s);
                gI = boson_neg<T>(plan, plan->bs_y, gI_in, ldg_in, batch, s);
                ldf = ldg = S;
            }
            if (gg2 && !accumulate_gg2 && plan->n_drop > 0) {
                const unsigned nb = static_cast<unsigned>(std::min<int64_t>((plan->n_drop + 255) / 256, 1024));
                hipLaunchKernelGGL(k_zero_at, dim3(nb), dim3(256), 0, s, gg2, (const int32_t *)plan->drop_idx,
                                   plan->n_drop);
            }
            bool done = false;
            if (!per_batch) {
                enqueue_pack<T>(plan, nph, s);
                done = enqueue_vjp_batched<T>(plan, batch, static_cast<const T *>(f), ldf,
                                              static_cast<const T *>(gI), ldg, static_cast<T *>(gf), ldgf,
                                              gg2, gg2 ? (accumulate_gg2 ? 2 : 1) : 0, s);
            } else if (batch >= plan->batch_min) {
                // a bath per vector, batched: the table's hw from the first bath's pack
                enqueue_pack<T>(plan, nph, s);
                done = enqueue_vjp_batched_pv<T>(plan, batch, static_cast<const T *>(f), ldf,
                                                 static_cast<const T *>(nph), static_cast<const T *>(gI), ldg,
                                                 static_cast<T *>(gf), ldgf, gg2, gg2 ? (accumulate_gg2 ? 2 : 1) : 0,
                                                 s);
            }
            // the kernels take unit-stride vectors of length S; strided
            // batch members are addressed one vector at a time
            for (int b = 0; b < batch && !done; ++b) {
                const T *nb = static_cast<const T *>(nph) + (per_batch ? b * tab : 0);
                if (per_batch) enqueue_pack<T>(plan, nb, s);
                const T *fb = static_cast<const T *>(f) + b * ldf;
                const T *lb = static_cast<const T *>(gI) + b * ldg;
                Epi<T> e{};
                if (gf) {
                    e = epi_store<T>(static_cast<T *>(gf) + b * ldgf, S);
                } else {
                    e.mode = -1;
                }
                const int gmode = gg2 ? ((accumulate_gg2 || b > 0) ? 2 : 1) : 0;
                enqueue_vjp<T>(plan, fb, lb, nb, e, gg2, gmode, s);
            }
            if (plan->boson && gf) neg_in_place<T>(plan, gf, ldgf, batch, s);
        };
        if (plan->dtype == EPHBTE_F64) run(double{});
        else run(float{});
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_rt_step(ephbte_plan plan, int32_t batch, void *f, int64_t ldf,
                             const void *nph, double dt_fs, int32_t n_steps, int32_t use_graph,
                             void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (batch < 1 || batch > 65535) return fail(EPHBTE_INVALID_ARGUMENT, "batch must be in [1, 65535]");
        if (!f || !nph) return fail(EPHBTE_INVALID_ARGUMENT, "f and nph must be non-NULL");
        if (ldf < plan->S) return fail(EPHBTE_INVALID_ARGUMENT, "ldf must be >= n_states");
        if (n_steps < 0) return fail(EPHBTE_INVALID_ARGUMENT, "n_steps must be >= 0");
        if (!std::isfinite(dt_fs)) return fail(EPHBTE_INVALID_ARGUMENT, "dt must be finite");
        if (n_steps == 0) return EPHBTE_OK;
        hipStream_t s = as_stream(stream);
        // Bose plans: u = -n obeys du/dt = -I_B(n) = I_F(u), the Fermi steps
        auto run = [&](auto tag) -> ephbte_status {
            using T = decltype(tag);
            if (plan->boson) neg_in_place<T>(plan, f, ldf, batch, s);
            const ephbte_status st =
                rt_step_impl<T>(plan, batch, static_cast<T *>(f), ldf, nph, dt_fs, n_steps, use_graph, s);
            if (plan->boson) neg_in_place<T>(plan, f, ldf, batch, s);
            return st;
        };
        if (plan->dtype == EPHBTE_F64) return run(double{});
        return run(float{});
    });
}

ephbte_status ephbte_rt_adjoint(ephbte_plan plan, const void *f0, const void *nph, double dt_fs,
                                int32_t n_steps, int32_t checkpoint_every, const void *gfT,
                                void *gf0, double *gg2, int32_t accumulate_gg2, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (!f0 || !nph || !gfT) return fail(EPHBTE_INVALID_ARGUMENT, "f0, nph and gfT must be non-NULL");
        if (n_steps < 1) return fail(EPHBTE_INVALID_ARGUMENT, "n_steps must be >= 1");
        if (checkpoint_every < 1) return fail(EPHBTE_INVALID_ARGUMENT, "checkpoint_every must be >= 1");
        if (!std::isfinite(dt_fs)) return fail(EPHBTE_INVALID_ARGUMENT, "dt must be finite");
        hipStream_t s = as_stream(stream);
        const int ce = std::min(checkpoint_every, n_steps);
        // Bose plans: n(T) = -u(T) with u the Fermi trajectory from -n(0), so
        // the Fermi adjoint of -dL/dn(T) gives dL/d|g|^2 and -dL/dn(0)
        auto run = [&](auto tag) -> ephbte_status {
            using T = decltype(tag);
            const T *x0 = static_cast<const T *>(f0), *gx = static_cast<const T *>(gfT);
            if (plan->boson) {
                x0 = boson_neg<T>(plan, plan->bs_x, f0, plan->S, 1, s);
                gx = boson_neg<T>(plan, plan->bs_y, gfT, plan->S, 1, s);
            }
            const ephbte_status st = rt_adjoint_impl<T>(plan, x0, nph, dt_fs, n_steps, ce, gx,
                                                        static_cast<T *>(gf0), gg2, accumulate_gg2, s);
            if (plan->boson && gf0) neg_in_place<T>(plan, gf0, plan->S, 1, s);
            return st;
        };
        if (plan->dtype == EPHBTE_F64) return run(double{});
        return run(float{});
    });
}

ephbte_status ephbte_iterate_transport(ephbte_plan plan, const void *f0, const void *vel,
                                       double T_K, const void *nph, double tol, int32_t max_iter,
                                       void *x_out, double *mobility, int32_t *iters,
                                       double *resid, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (plan->boson) return boson_unsupported("the transport iteration");
        if (!f0 || !vel || !nph || !mobility)
            return fail(EPHBTE_INVALID_ARGUMENT, "f0, vel, nph and mobility must be non-NULL");
        if (!(T_K > 0.0) || !std::isfinite(T_K)) return fail(EPHBTE_INVALID_ARGUMENT, "T_K must be > 0");
        if (max_iter < 0) return fail(EPHBTE_INVALID_ARGUMENT, "max_iter must be >= 0");
        if (!(tol >= 0.0)) return fail(EPHBTE_INVALID_ARGUMENT, "tol must be >= 0");
        hipStream_t s = as_stream(stream);
        if (plan->dtype == EPHBTE_F64)
            return transport_impl<double>(plan, static_cast<const double *>(f0),
                                          static_cast<const double *>(vel), T_K, nph, tol, max_iter,
                                          static_cast<double *>(x_out), mobility, iters, resid, s);
        return transport_impl<float>(plan, static_cast<const float *>(f0),
                                     static_cast<const float *>(vel), T_K, nph, tol, max_iter,
                                     static_cast<float *>(x_out), mobility, iters, resid, s);
    });
}

ephbte_status ephbte_update_g2(ephbte_plan plan, const double *g2, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (!g2) return fail(EPHBTE_INVALID_ARGUMENT, "g2 must be non-NULL");
        hipStream_t s = as_stream(stream);
        if (plan->E == 0) return EPHBTE_OK;
        if (plan->dtype == EPHBTE_F64)
            hipLaunchKernelGGL((k_cast_g2<double>), dim3(4096), dim3(256), 0, s,
                               (const int32_t *)plan->ent_chan, g2, static_cast<double *>(plan->g2),
                               plan->E);
        else
            hipLaunchKernelGGL((k_cast_g2<float>), dim3(4096), dim3(256), 0, s,
                               (const int32_t *)plan->ent_chan, g2, static_cast<float *>(plan->g2),
                               plan->E);
        HIPC(hipGetLastError());
        update_gmax(plan, s);
        if (plan->pr_ok) {
            const int64_t np = plan->pr_ld * plan->nm;
            if (plan->dtype == EPHBTE_F64)
                hipLaunchKernelGGL((k_ph_gather_g2<double>), dim3(4096), dim3(256), 0, s,
                                   (const int32_t *)plan->pr_chan, g2, static_cast<double *>(plan->pr_g2), np);
            else
                hipLaunchKernelGGL((k_ph_gather_g2<float>), dim3(4096), dim3(256), 0, s,
                                   (const int32_t *)plan->pr_chan, g2, static_cast<float *>(plan->pr_g2), np);
            HIPC(hipGetLastError());
        }
        const int64_t ns = plan->ph_ld * plan->nm;
        if (ns > 0) {
            if (plan->dtype == EPHBTE_F64)
                hipLaunchKernelGGL((k_ph_gather_g2<double>), dim3(4096), dim3(256), 0, s,
                                   (const int32_t *)plan->ph_chan, g2, static_cast<double *>(plan->ph_g2), ns);
            else
                hipLaunchKernelGGL((k_ph_gather_g2<float>), dim3(4096), dim3(256), 0, s,
                                   (const int32_t *)plan->ph_chan, g2, static_cast<float *>(plan->ph_g2), ns);
            HIPC(hipGetLastError());
        }
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_phonon_rate(ephbte_plan plan, const void *f, const void *nph, void *dN,
                                 void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (plan->boson) return boson_unsupported("the phonon-side rate");
        if (!f || !nph || !dN) return fail(EPHBTE_INVALID_ARGUMENT, "f, nph and dN must be non-NULL");
        const int64_t nbin = static_cast<int64_t>(plan->nq[0]) * plan->nq[1] * plan->nq[2] * plan->nm;
        if (overlaps(dN, esize(plan) * nbin, f, esize(plan) * plan->S))
            return fail(EPHBTE_INVALID_ARGUMENT, "dN must not overlap f");
        hipStream_t s = as_stream(stream);
        ensure_phonon(plan);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            enqueue_phonon_rate<T>(plan, static_cast<const T *>(f), static_cast<const T *>(nph),
                                   static_cast<T *>(dN), s);
        };
        if (plan->dtype == EPHBTE_F64) run(double{});
        else run(float{});
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_rt_step_coupled(ephbte_plan plan, void *f, void *nph, double dt_fs,
                                     int32_t n_steps, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (plan->boson) return boson_unsupported("the coupled electron-phonon step");
        if (!f || !nph) return fail(EPHBTE_INVALID_ARGUMENT, "f and nph must be non-NULL");
        if (n_steps < 0) return fail(EPHBTE_INVALID_ARGUMENT, "n_steps must be >= 0");
        if (!std::isfinite(dt_fs)) return fail(EPHBTE_INVALID_ARGUMENT, "dt_fs must be finite");
        const int64_t nbin = static_cast<int64_t>(plan->nq[0]) * plan->nq[1] * plan->nq[2] * plan->nm;
        if (overlaps(nph, esize(plan) * nbin, f, esize(plan) * plan->S))
            return fail(EPHBTE_INVALID_ARGUMENT, "nph must not overlap f");
        if (n_steps == 0) return EPHBTE_OK;
        hipStream_t s = as_stream(stream);
        if (plan->dtype == EPHBTE_F64)
            return rt_coupled_impl<double>(plan, static_cast<double *>(f), static_cast<double *>(nph), dt_fs,
                                           n_steps, s);
        return rt_coupled_impl<float>(plan, static_cast<float *>(f), static_cast<float *>(nph), dt_fs, n_steps, s);
    });
}

ephbte_status ephbte_collision_vjp_nph(ephbte_plan plan, const void *f, const void *nph, const void *gI,
                                       void *gnph, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (!f || !nph || !gI || !gnph)
            return fail(EPHBTE_INVALID_ARGUMENT, "f, nph, gI and gnph must be non-NULL");
        const size_t es = esize(plan);
        const int64_t nbin = nqm_of(plan);
        if (overlaps(gnph, es * nbin, f, es * plan->S) || overlaps(gnph, es * nbin, gI, es * plan->S) ||
            overlaps(gnph, es * nbin, nph, es * nbin))
            return fail(EPHBTE_INVALID_ARGUMENT, "gnph must not overlap f, gI or nph");
        hipStream_t s = as_stream(stream);
        ensure_phonon(plan);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            const T *x = static_cast<const T *>(f), *l = static_cast<const T *>(gI);
            if (plan->boson) {   // dL/dN of sum (-lam) I_F(-n)
                x = boson_neg<T>(plan, plan->bs_x, f, plan->S, 1, s);
                l = boson_neg<T>(plan, plan->bs_y, gI, plan->S, 1, s);
            }
            enqueue_phonon_adj<T>(plan, x, static_cast<const T *>(nph), l, (const T *)nullptr, static_cast<T *>(gnph),
                                  nullptr, s);
        };
        if (plan->dtype == EPHBTE_F64) run(double{});
        else run(float{});
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_phonon_rate_vjp(ephbte_plan plan, const void *f, const void *nph, const void *gR, void *gf,
                                     void *gnph, double *gg2, int32_t accumulate_gg2, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (plan->boson) return boson_unsupported("the reverse of the phonon-side rate");
        if (!f || !nph || !gR) return fail(EPHBTE_INVALID_ARGUMENT, "f, nph and gR must be non-NULL");
        const size_t es = esize(plan);
        const int64_t nbin = nqm_of(plan);
        if (gf && (overlaps(gf, es * plan->S, f, es * plan->S) || overlaps(gf, es * plan->S, gR, es * nbin)))
            return fail(EPHBTE_INVALID_ARGUMENT, "gf must not overlap f or gR");
        if (gnph && (overlaps(gnph, es * nbin, nph, es * nbin) || overlaps(gnph, es * nbin, gR, es * nbin)))
            return fail(EPHBTE_INVALID_ARGUMENT, "gnph must not overlap nph or gR");
        hipStream_t s = as_stream(stream);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            const T *ft = static_cast<const T *>(f), *nt = static_cast<const T *>(nph), *mt = static_cast<const T *>(gR);
            if (gf) {
                ensure_phonon_vjp<T>(plan);
                hipLaunchKernelGGL((k_axpby<T>), dim3(grid_of(plan->S)), dim3(256), 0, s, int64_t(plan->S), T(0), ft,
                                   T(0), (const T *)nullptr, static_cast<T *>(gf));
                enqueue_phonon_vjp_f<T>(plan, ft, nt, mt, static_cast<T *>(gf), s);
            }
            if (gnph || gg2) {
                ensure_phonon(plan);
                if (gg2 && !accumulate_gg2)
                    hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, s, gg2, plan->nch, 0.0);
                T *out = static_cast<T *>(gnph);
                if (!out) {
                    ensure(plan->ca_mu, es * static_cast<size_t>(std::max<int64_t>(nbin, 1)), &plan->ws_gen);
                    out = static_cast<T *>(plan->ca_mu.p);
                }
                enqueue_phonon_adj<T>(plan, ft, nt, (const T *)nullptr, mt, out, gg2, s);
            }
        };
        if (plan->dtype == EPHBTE_F64) run(double{});
        else run(float{});
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_rt_adjoint_coupled(ephbte_plan plan, const void *f0, const void *nph0, double dt_fs,
                                        int32_t n_steps, int32_t checkpoint_every, const void *gfT,
                                        const void *gNT, void *gf0, void *gN0, double *gg2,
                                        int32_t accumulate_gg2, void *stream) {
    return guarded(plan, stream, [&]() -> ephbte_status {
        if (plan->boson) return boson_unsupported("the adjoint of the coupled step");
        if (!f0 || !nph0) return fail(EPHBTE_INVALID_ARGUMENT, "f0 and nph0 must be non-NULL");
        if (n_steps < 1) return fail(EPHBTE_INVALID_ARGUMENT, "n_steps must be >= 1");
        if (checkpoint_every < 1) return fail(EPHBTE_INVALID_ARGUMENT, "checkpoint_every must be >= 1");
        if (!std::isfinite(dt_fs)) return fail(EPHBTE_INVALID_ARGUMENT, "dt_fs must be finite");
        const size_t es = esize(plan);
        const int64_t nbin = nqm_of(plan);
        if (gf0 && overlaps(gf0, es * plan->S, f0, es * plan->S))
            return fail(EPHBTE_INVALID_ARGUMENT, "gf0 must not overlap f0");
        if (gN0 && overlaps(gN0, es * nbin, nph0, es * nbin))
            return fail(EPHBTE_INVALID_ARGUMENT, "gN0 must not overlap nph0");
        hipStream_t s = as_stream(stream);
        const int ce = std::min(checkpoint_every, n_steps);
        auto run = [&](auto tag) {
            using T = decltype(tag);
            return rt_adjoint_coupled_impl<T>(plan, static_cast<const T *>(f0), static_cast<const T *>(nph0), dt_fs,
                                              n_steps, ce, static_cast<const T *>(gfT), static_cast<const T *>(gNT),
                                              static_cast<T *>(gf0), static_cast<T *>(gN0), gg2, accumulate_gg2, s);
        };
        if (plan->dtype == EPHBTE_F64) return run(double{});
        return run(float{});
    });
}

ephbte_status ephbte_set_tuning(ephbte_plan plan, const ephbte_tuning *tuning) {
    return guarded(plan, nullptr, [&]() -> ephbte_status {
        if (!tuning) return fail(EPHBTE_INVALID_ARGUMENT, "tuning is NULL");
        int bt = tuning->block_threads ? tuning->block_threads : plan->block_threads;
        if (bt != 64 && bt != 128 && bt != 256 && bt != 512)
            return fail(EPHBTE_INVALID_ARGUMENT, "block_threads must be 64, 128, 256 or 512");
        int ce = tuning->chunk_entries ? tuning->chunk_entries : plan->chunk_entries;
        if (ce < 0) return fail(EPHBTE_INVALID_ARGUMENT, "chunk_entries must be >= 0");
        if (tuning->xcd_map < 0 || tuning->xcd_map > 2)
            return fail(EPHBTE_INVALID_ARGUMENT, "xcd_map must be 0, 1 or 2");
        const int pt = tuning->batch_partners;
        if (pt != 0 && (pt < 16 || pt > 1024 || batch_lds_bytes(plan, pt) > plan->lds_max))
            return fail(EPHBTE_INVALID_ARGUMENT,
                        "batch_partners must be in [16, 1024] and fit the LDS of one workgroup");
        if (tuning->table_order < 0 || tuning->table_order > 2)
            return fail(EPHBTE_INVALID_ARGUMENT, "table_order must be 0 (keep), 1 or 2");
        const int pw = tuning->pair_window;
        if (pw != 0 && (pw < 64 || vjp_pair_lds_bytes(plan->dtype, pw) > plan->lds_max))
            return fail(EPHBTE_INVALID_ARGUMENT,
                        "pair_window must be >= 64 and fit the reverse pass's LDS of one workgroup");
        const int pth = tuning->pair_threads;
        if (pth != 0 && pth != 256 && pth != 512 && pth != 768 && pth != 1024)
            return fail(EPHBTE_INVALID_ARGUMENT, "pair_threads must be 0 (keep), 256, 512, 768 or 1024");
        if (tuning->pair_order < 0 || tuning->pair_order > 2)
            return fail(EPHBTE_INVALID_ARGUMENT, "pair_order must be 0 (keep), 1 or 2");
        const int prow = tuning->pair_rows;
        if (prow < 0 || prow > 65536 || (prow & (prow - 1)) != 0)
            return fail(EPHBTE_INVALID_ARGUMENT, "pair_rows must be 0 (keep) or a power of 2 up to 65536");
        if (tuning->tile_entries < -1)
            return fail(EPHBTE_INVALID_ARGUMENT, "tile_entries must be -1 (default), 0 (keep) or > 0");
        if (tuning->fp64_exp < 0 || tuning->fp64_exp > 2)
            return fail(EPHBTE_INVALID_ARGUMENT, "fp64_exp must be 0 (keep), 1 or 2");
        if (tuning->layout < 0 || tuning->layout > 3)
            return fail(EPHBTE_INVALID_ARGUMENT, "layout must be 0 (keep), 1, 2 or 3");
        if (tuning->layout >= 2 && !plan->sym_ok)
            return fail(EPHBTE_INVALID_ARGUMENT,
                        "the single-copy pass needs more LDS per workgroup than this device has");
        if (tuning->layout == 3 && !plan->pr_ok)
            return fail(EPHBTE_INVALID_ARGUMENT,
                        "this plan has no pair records (fewer than half of their mode slots would hold a channel)");
        HIPC(hipDeviceSynchronize());
        plan->block_threads = bt;
        if (tuning->xcd_map) plan->xcd_map = tuning->xcd_map == 1;
        if (tuning->tile_entries) plan->tile_entries = tuning->tile_entries > 0 ? tuning->tile_entries : 0;
        if (tuning->layout) plan->layout = tuning->layout;
        if (tuning->fp64_exp) plan->exp_table = tuning->fp64_exp == 1;
        if (tuning->table_order) plan->tab_mm = tuning->table_order == 2;
        if (pw) plan->pr_lds_states = pw;
        if (pth) plan->pr_threads = pth;
        if (tuning->pair_order) plan->pair_order = tuning->pair_order;
        if (prow) plan->pair_shift = __builtin_ctz(static_cast<unsigned>(prow));
        upload_chunks(plan, ce);
        if (pt != 0) upload_btiles(plan, pt);
        free_graphs(plan);
        return EPHBTE_OK;
    });
}

// Times the candidate tunings on this plan and applies the fastest.
static ephbte_status autotune_timed(ephbte_plan plan, int32_t batch, ephbte_tuning *chosen) {
    {
        const size_t es = esize(plan);
        const int64_t S = plan->S;
        const int64_t nqm = static_cast<int64_t>(plan->nq[0]) * plan->nq[1] * plan->nq[2] * plan->nm;
        void *f = nullptr, *I = nullptr, *nph = nullptr;
        size_t dummy = 0;
        dalloc(f, es * S * batch, &dummy);
        dalloc(I, es * S * batch, &dummy);
        dalloc(nph, es * nqm, &dummy);
        struct Freer {
            void *a, *b, *c;
            ~Freer() { (void)hipFree(a); (void)hipFree(b); (void)hipFree(c); }
        } fr{f, I, nph};
        // half-filled states and phonons: the kernels' cost does not depend on values
        if (es == 8) {
            std::vector<double> h(std::max<int64_t>(S * batch, nqm), 0.5);
            HIPC(hipMemcpy(f, h.data(), es * S * batch, hipMemcpyHostToDevice));
            HIPC(hipMemcpy(nph, h.data(), es * nqm, hipMemcpyHostToDevice));
        } else {
            std::vector<float> h(std::max<int64_t>(S * batch, nqm), 0.5f);
            HIPC(hipMemcpy(f, h.data(), es * S * batch, hipMemcpyHostToDevice));
            HIPC(hipMemcpy(nph, h.data(), es * nqm, hipMemcpyHostToDevice));
        }
        hipEvent_t e0, e1;
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        auto once = [&]() {
            if (plan->dtype == EPHBTE_F64) {
                ensure_fwd<double>(plan, batch);
                enqueue_forward<double>(plan, batch, (const double *)f, S, nph,
                                        epi_store<double>((double *)I, S), nullptr);
            } else {
                ensure_fwd<float>(plan, batch);
                enqueue_forward<float>(plan, batch, (const float *)f, S, nph,
                                       epi_store<float>((float *)I, S), nullptr);
            }
        };
        auto time_it = [&]() -> float {
            once();
            HIPC(hipEventRecord(e0, nullptr));
            for (int r = 0; r < 3; ++r) once();
            HIPC(hipEventRecord(e1, nullptr));
            HIPC(hipEventSynchronize(e1));
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        if (batch >= plan->batch_min) {
            // batched pass: partner sub-tile sizes that fit the LDS of a workgroup
            const int pt64[] = {48, 64, 96, 128, 160};
            const int pt32[] = {96, 128, 192, 256, 320};
            const int *cand = plan->dtype == EPHBTE_F64 ? pt64 : pt32;
            float best = INFINITY;
            int best_pt = plan->pt;
            for (int i = 0; i < 5; ++i) {
                if (batch_lds_bytes(plan, cand[i]) > plan->lds_max) continue;
                upload_btiles(plan, cand[i]);
                const float ms = time_it();
                if (ms < best) {
                    best = ms;
                    best_pt = cand[i];
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            upload_btiles(plan, best_pt);
            if (chosen) {
                std::memset(chosen, 0, sizeof(*chosen));
                chosen->chunk_entries = plan->chunk_entries;
                chosen->block_threads = plan->block_threads;
                chosen->xcd_map = plan->xcd_map ? 1 : 2;
                chosen->batch_partners = best_pt;
            }
            return EPHBTE_OK;
        }
        // chunk size x tile size (default target, and about 4 and 12 tiles per
        // compute unit) at 512 threads, plus the default tiles at 256 threads
        const int chunk_c[] = {8192, 16384, 32768, 65536};
        const int64_t cu = static_cast<int64_t>(plan->n_cu);
        const int64_t tile_c[] = {0, plan->E / (4 * cu) + 1, plan->E / (12 * cu) + 1};
        float best = INFINITY;
        int best_ce = plan->chunk_entries, best_bt = plan->block_threads;
        int64_t best_te = plan->tile_entries;
        for (int bt : {512, 256})
            for (int ce : chunk_c)
                for (int64_t te : tile_c) {
                    if (bt == 256 && te != 0) continue;
                    plan->block_threads = bt;
                    plan->tile_entries = te;
                    upload_chunks(plan, ce);
                    const float ms = time_it();
                    if (ms < best) {
                        best = ms;
                        best_ce = ce;
                        best_bt = bt;
                        best_te = te;
                    }
                }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan->block_threads = best_bt;
        plan->tile_entries = best_te;
        upload_chunks(plan, best_ce);
        if (chosen) {
            std::memset(chosen, 0, sizeof(*chosen));
            chosen->chunk_entries = best_ce;
            chosen->block_threads = best_bt;
            chosen->xcd_map = plan->xcd_map ? 1 : 2;
            chosen->batch_partners = plan->pt;
            chosen->tile_entries = best_te > 0 ? static_cast<int32_t>(std::min<int64_t>(best_te, INT32_MAX)) : -1;
        }
        return EPHBTE_OK;
    }
}

ephbte_status ephbte_autotune(ephbte_plan plan, int32_t batch, ephbte_tuning *chosen,
                              const char *cache_path) {
    return guarded(plan, nullptr, [&]() -> ephbte_status {
        if (batch < 1 || batch > 65535) return fail(EPHBTE_INVALID_ARGUMENT, "batch must be in [1, 65535]");
        HIPC(hipDeviceSynchronize());
        TuneCache cache;
        std::string key;
        if (cache_path) {
            const int r = read_tune_cache(cache_path, cache);
            if (r < 0) return fail(EPHBTE_INVALID_ARGUMENT, "cache_path holds something other than an autotune cache");
            key = tune_key(plan, batch);
            const auto it = cache.find(key);
            if (it != cache.end()) {
                const TuneEntry &e = it->second;
                auto get = [&](const char *n, long long d) {
                    const auto f = e.find(n);
                    return f == e.end() ? d : f->second;
                };
                const bool batched = batch >= plan->batch_min;
                const long long pt = get("batch_partners", plan->pt);
                const long long bt = get("block_threads", plan->block_threads);
                const long long ce = get("chunk_entries", plan->chunk_entries);
                const long long te = get("tile_entries", -1);
                const bool ok = batched ? (pt >= 16 && pt <= 1024 && batch_lds_bytes(plan, static_cast<int>(pt)) <= plan->lds_max)
                                        : ((bt == 64 || bt == 128 || bt == 256 || bt == 512) && ce >= 0 && te >= -1);
                if (ok) {
                    if (batched) {
                        if (pt != plan->pt) upload_btiles(plan, static_cast<int>(pt));
                    } else {
                        plan->block_threads = static_cast<int>(bt);
                        plan->tile_entries = te > 0 ? te : 0;
                        upload_chunks(plan, static_cast<int64_t>(ce));
                        free_graphs(plan);
                    }
                    if (chosen) {
                        std::memset(chosen, 0, sizeof(*chosen));
                        chosen->chunk_entries = plan->chunk_entries;
                        chosen->block_threads = plan->block_threads;
                        chosen->xcd_map = plan->xcd_map ? 1 : 2;
                        chosen->batch_partners = plan->pt;
                        chosen->tile_entries = plan->tile_entries > 0
                                                   ? static_cast<int32_t>(std::min<int64_t>(plan->tile_entries, INT32_MAX))
                                                   : -1;
                    }
                    return EPHBTE_OK;
                }
                // a stale or foreign entry: tune again and replace it
            }
        }
        ephbte_tuning got{};
        const ephbte_status st = autotune_timed(plan, batch, &got);
        if (st != EPHBTE_OK) return st;
        if (chosen) *chosen = got;
        if (cache_path) {
            TuneEntry e;
            if (batch >= plan->batch_min) {
                e["batch_partners"] = got.batch_partners;
            } else {
                e["block_threads"] = got.block_threads;
                e["chunk_entries"] = got.chunk_entries;
                e["tile_entries"] = got.tile_entries;
            }
            cache[key] = e;
            if (!write_tune_cache(cache_path, cache))
                return fail(EPHBTE_INVALID_ARGUMENT, "could not write cache_path (the plan keeps the tuning)");
        }
        return EPHBTE_OK;
    });
}

ephbte_status ephbte_set_field(ephbte_plan plan, const double rate[3]) {
    if (!plan || !rate) return fail(EPHBTE_INVALID_ARGUMENT, "plan and rate must be non-NULL");
    bool on = false;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(rate[a])) return fail(EPHBTE_INVALID_ARGUMENT, "field rates must be finite");
        on = on || rate[a] != 0.0;
    }
    if (on && plan->boson) return boson_unsupported("the field term");
    if (on && !plan->nbr_ok)
        return fail(EPHBTE_INVALID_ARGUMENT,
                    "the field term needs each (k, band) held by one state (give state_band)");
    try {
        DeviceGuard g(plan->device);
        HIPC(hipDeviceSynchronize());
        free_graphs(plan);   // captured steps hold the previous rates
    } catch (const HipError &e) {
        return fail(EPHBTE_HIP_ERROR, std::string(e.where) + ": " + hipGetErrorString(e.e));
    }
    for (int a = 0; a < 3; ++a) plan->drift_rate[a] = rate[a];
    plan->drift_on = on;
    return EPHBTE_OK;
}

ephbte_status ephbte_kernel_timing(ephbte_plan plan, int32_t mode, double *mean_ms, int64_t *launches) {
    if (!plan) return fail(EPHBTE_INVALID_ARGUMENT, "plan is NULL");
    if (mode != 0 && mode != 1) return fail(EPHBTE_INVALID_ARGUMENT, "mode must be 0 (stop) or 1 (start)");
    try {
        DeviceGuard g(plan->device);
        double total = 0.0;
        const size_t n = plan->ktime_used;
        if (mode == 0) {
            for (size_t i = 0; i < n; ++i) {
                HIPC(hipEventSynchronize(plan->ktime_ev[2 * i + 1]));
                float ms = 0.0f;
                HIPC(hipEventElapsedTime(&ms, plan->ktime_ev[2 * i], plan->ktime_ev[2 * i + 1]));
                total += ms;
            }
        }
        if (mean_ms) *mean_ms = mode == 0 && n > 0 ? total / static_cast<double>(n) : 0.0;
        if (launches) *launches = mode == 0 ? static_cast<int64_t>(n) : 0;
        plan->ktime_used = 0;
        plan->ktime_on = mode == 1;
        return EPHBTE_OK;
    } catch (const HipError &e) {
        return fail(EPHBTE_HIP_ERROR, std::string(e.where) + ": " + hipGetErrorString(e.e));
    }
}

ephbte_status ephbte_plan_info(ephbte_plan plan, int64_t out[12]) {
    if (!plan || !out) return fail(EPHBTE_INVALID_ARGUMENT, "plan and out must be non-NULL");
    out[0] = plan->S;
    out[1] = plan->nch;
    out[2] = plan->E;
    out[3] = plan->n_chunks;
    out[4] = plan->dtype;
    out[5] = plan->device;
    out[6] = static_cast<int64_t>(plan->bytes());
    out[7] = plan->chunk_entries;
    out[8] = plan->block_threads;
    out[9] = plan->nch_kept;
    out[10] = plan->layout;
    out[11] = plan->pr_ok ? plan->pr_np : 0;
    return EPHBTE_OK;
}

int64_t ephbte_plan_bytes(ephbte_plan plan) { return plan ? static_cast<int64_t>(plan->bytes()) : 0; }

void ephbte_destroy(ephbte_plan plan) {
    if (!plan) return;
    try {
        (void)hipDeviceSynchronize();
        free_plan(plan);
    } catch (...) {
    }
}

}  // extern "C"
