// Runs one entry point of the library, built for the CPU with the runtime
// stand-in of hip/hip_runtime.h, on inputs that a test wrote into a folder:
//   driver <mode> <folder>
// The folder holds meta.txt ("key value" lines) and raw little-endian arrays;
// results are written back as FP64 arrays named out_*.bin.  Test
// infrastructure: it links the library's sources directly.
#include "api.hip"

#include <fstream>
#include <map>

namespace {

std::string g_dir;
std::map<std::string, std::vector<double>> g_meta;

void load_meta() {
    std::ifstream in(g_dir + "/meta.txt");
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string key;
        ss >> key;
        double v;
        while (ss >> v) g_meta[key].push_back(v);
    }
}
double meta(const std::string &k, double def = NAN) {
    auto it = g_meta.find(k);
    if (it == g_meta.end() || it->second.empty()) {
        if (std::isnan(def)) {
            fprintf(stderr, "meta key %s missing\n", k.c_str());
            exit(2);
        }
        return def;
    }
    return it->second[0];
}
template <class T> std::vector<T> rd(const std::string &name, size_t n) {
    std::vector<T> v(n);
    std::ifstream in(g_dir + "/" + name, std::ios::binary);
    in.read(reinterpret_cast<char *>(v.data()), static_cast<std::streamsize>(n * sizeof(T)));
    if (!in) {
        fprintf(stderr, "reading %s (%zu values) failed\n", name.c_str(), n);
        exit(2);
    }
    return v;
}
void wr(const std::string &name, const std::vector<double> &v) {
    std::ofstream o(g_dir + "/" + name, std::ios::binary);
    o.write(reinterpret_cast<const char *>(v.data()), static_cast<std::streamsize>(v.size() * 8));
}
void check(ephbte_status st, const char *what) {
    if (st != EPHBTE_OK) {
        fprintf(stderr, "%s: status %d: %s\n", what, st, ephbte_last_error());
        exit(3);
    }
}

// device buffers in the plan's working precision
struct Dev {
    bool f32;
    void *alloc(size_t n) {
        void *p = nullptr;
        hipMalloc(&p, (f32 ? 4 : 8) * std::max<size_t>(n, 1));
        return p;
    }
    void *up(const std::vector<double> &h) {
        void *p = alloc(h.size());
        if (f32) {
            std::vector<float> t(h.begin(), h.end());
            hipMemcpy(p, t.data(), 4 * h.size(), hipMemcpyHostToDevice);
        } else {
            hipMemcpy(p, h.data(), 8 * h.size(), hipMemcpyHostToDevice);
        }
        return p;
    }
    std::vector<double> down(const void *p, size_t n) {
        std::vector<double> h(n);
        if (f32) {
            std::vector<float> t(n);
            hipMemcpy(t.data(), p, 4 * n, hipMemcpyDeviceToHost);
            h.assign(t.begin(), t.end());
        } else {
            hipMemcpy(h.data(), p, 8 * n, hipMemcpyDeviceToHost);
        }
        return h;
    }
};

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: driver <mode> <folder>\n");
        return 2;
    }
    const std::string mode = argv[1];
    g_dir = argv[2];
    emu::verbose = getenv("CPU_BUILD_VERBOSE") != nullptr;
    load_meta();
    const int S = static_cast<int>(meta("S"));
    const int nm = static_cast<int>(meta("nm"));
    const int64_t nch = static_cast<int64_t>(meta("nch"));
    const int q0 = static_cast<int>(g_meta["qgrid"].at(0)), q1 = static_cast<int>(g_meta["qgrid"].at(1)),
              q2 = static_cast<int>(g_meta["qgrid"].at(2));
    const size_t nqm = static_cast<size_t>(q0) * q1 * q2 * nm;
    const bool f32 = meta("dtype") == 1;
    const int B = static_cast<int>(meta("B", 1));

    auto sk = rd<int32_t>("state_k.bin", S);
    auto sb = rd<int8_t>("state_band.bin", S);
    auto eps = rd<double>("eps.bin", S);
    auto hw = rd<double>("hw.bin", nqm);
    auto ci = rd<int32_t>("ci.bin", nch), cj = rd<int32_t>("cj.bin", nch);
    auto cn = rd<int8_t>("cn.bin", nch);
    auto g2 = rd<double>("g2.bin", nch);
    ephbte_problem p{};
    p.n_states = S;
    p.state_k = sk.data();
    p.state_band = sb.data();
    p.eps = eps.data();
    for (int a = 0; a < 3; ++a) {
        p.kgrid[a] = static_cast<int32_t>(g_meta["kgrid"].at(a));
        p.qgrid[a] = static_cast<int32_t>(g_meta["qgrid"].at(a));
    }
    p.n_modes = nm;
    p.hw = hw.data();
    p.n_channels = nch;
    p.ch_i = ci.data();
    p.ch_j = cj.data();
    p.ch_nu = cn.data();
    p.g2 = g2.data();
    p.sigma = meta("sigma");
    p.n_q_norm = meta("nq");
    p.dtype = f32 ? EPHBTE_F32 : EPHBTE_F64;
    p.device = 0;
    ephbte_build_opts opts{};
    opts.energy_nsigma = meta("energy_nsigma", 0.0);
    opts.g2_min = meta("g2_min", 0.0);
    opts.elastic_modes = static_cast<uint32_t>(meta("elastic_modes", 0));
    opts.statistics = static_cast<int32_t>(meta("statistics", 0));
    ephbte_plan plan = nullptr;
    check(ephbte_build_channels(&p, &opts, &plan), "build_channels");
    // tuning knobs (0 keeps the plan's value)
    ephbte_tuning t{};
    t.layout = static_cast<int32_t>(meta("layout", 0));
    t.chunk_entries = static_cast<int32_t>(meta("chunk_entries", 0));
    t.block_threads = static_cast<int32_t>(meta("block_threads", 0));
    t.xcd_map = static_cast<int32_t>(meta("xcd_map", 0));
    t.batch_partners = static_cast<int32_t>(meta("batch_partners", 0));
    t.tile_entries = static_cast<int32_t>(meta("tile_entries", 0));
    t.fp64_exp = static_cast<int32_t>(meta("fp64_exp", 0));
    t.table_order = static_cast<int32_t>(meta("table_order", 0));
    t.pair_window = static_cast<int32_t>(meta("pair_window", 0));
    t.pair_threads = static_cast<int32_t>(meta("pair_threads", 0));
    t.pair_order = static_cast<int32_t>(meta("pair_order", 0));
    t.pair_rows = static_cast<int32_t>(meta("pair_rows", 0));
    if (t.layout || t.chunk_entries || t.block_threads || t.xcd_map || t.batch_partners || t.tile_entries ||
        t.fp64_exp || t.table_order || t.pair_window || t.pair_threads || t.pair_order || t.pair_rows)
        check(ephbte_set_tuning(plan, &t), "set_tuning");
    // empty_windows: every LDS tile whose chunks hold no entries gets an empty
    // partner window (nothing staged), the shape that once made masked lanes
    // read an unwritten LDS slot; the kernels must not depend on that slot
    if (meta("empty_windows", 0.0) != 0.0) {
        double emptied = 0;
        struct Set { TileRec *t; int64_t n; const int64_t *beg, *end; };
        const Set sets[3] = {{plan->tiles, plan->n_tiles, plan->chunk_beg, nullptr},
                             {plan->small_tiles, plan->n_small_tiles, plan->chunk_beg, nullptr},
                             {plan->sym_tiles, plan->n_sym_tiles, plan->sym_chunk_beg, plan->sym_chunk_end}};
        for (const Set &x : sets) {
            for (int64_t i = 0; i < x.n; ++i) {
                TileRec &t = x.t[i];
                if (!t.lds) continue;
                int64_t ents = 0;
                for (int64_t c = t.c0; c < t.c1; ++c) ents += (x.end ? x.end[c] : x.beg[c + 1]) - x.beg[c];
                if (ents == 0) {
                    t.p_hi = t.p_lo - 1;
                    emptied += 1;
                }
            }
        }
        wr("out_emptied.bin", {emptied});
    }
    Dev dv{f32};
    // per-vector baths: nph holds B tables of [Nq][n_modes]
    const int per_batch = static_cast<int>(meta("nph_per_batch", 0));
    auto nph = rd<double>("nph.bin", per_batch ? nqm * B : nqm);
    void *dN = dv.up(nph);

    if (mode == "forward") {
        auto f = rd<double>("f.bin", static_cast<size_t>(B) * S);
        void *df = dv.up(f), *dI = dv.alloc(static_cast<size_t>(B) * S);
        check(ephbte_kernel_timing(plan, 1, nullptr, nullptr), "kernel_timing start");
        check(ephbte_collision_integral(plan, B, df, S, dN, per_batch, dI, S, nullptr), "collision_integral");
        double kms = 0;
        int64_t kn = 0;
        check(ephbte_kernel_timing(plan, 0, &kms, &kn), "kernel_timing stop");
        wr("out_I.bin", dv.down(dI, static_cast<size_t>(B) * S));
        wr("out_timing.bin", {kms, static_cast<double>(kn)});
    } else if (mode == "noalloc") {
        // the allocation-free pass after the plain one, on scratch that holds
        // fresh-memory bytes; it must make no hipMalloc call
        fill_unwritten(ephbte::scratch, sizeof(ephbte::scratch), 0xA5);
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dI = dv.alloc(static_cast<size_t>(S)), *dJ = dv.alloc(static_cast<size_t>(S));
        check(ephbte_collision_integral(plan, 1, df, S, dN, 0, dI, S, nullptr), "collision_integral");
        const long long m0 = emu::n_malloc;
        check(ephbte_collision_integral_noalloc(plan, df, dN, dJ, nullptr), "collision_integral_noalloc");
        const long long m1 = emu::n_malloc;
        wr("out_I.bin", dv.down(dI, static_cast<size_t>(S)));
        wr("out_J.bin", dv.down(dJ, static_cast<size_t>(S)));
        wr("out_mallocs.bin", {static_cast<double>(m1 - m0)});
    } else if (mode == "vjp") {
        auto f = rd<double>("f.bin", static_cast<size_t>(B) * S);
        auto lam = rd<double>("lam.bin", static_cast<size_t>(B) * S);
        void *df = dv.up(f), *dl = dv.up(lam), *dg = dv.alloc(static_cast<size_t>(B) * S);
        // the |g|^2 gradient starts at gg2_fill: overwritten, and 0 for removed channels
        std::vector<double> fill(static_cast<size_t>(nch), meta("gg2_fill", 0.0));
        double *dgg = nullptr;
        hipMalloc(reinterpret_cast<void **>(&dgg), 8 * static_cast<size_t>(nch));
        hipMemcpy(dgg, fill.data(), 8 * static_cast<size_t>(nch), hipMemcpyHostToDevice);
        check(ephbte_collision_vjp(plan, B, df, S, dN, per_batch, dl, S, dg, S, dgg, 0, nullptr), "collision_vjp");
        wr("out_gf.bin", dv.down(dg, static_cast<size_t>(B) * S));
        std::vector<double> gg(static_cast<size_t>(nch));
        hipMemcpy(gg.data(), dgg, 8 * static_cast<size_t>(nch), hipMemcpyDeviceToHost);
        wr("out_gg2.bin", gg);
    } else if (mode == "rt" || mode == "field") {
        const double dt = meta("dt");
        const int n = static_cast<int>(meta("steps"));
        if (mode == "field") {
            const double rates[3] = {g_meta["rates"].at(0), g_meta["rates"].at(1), g_meta["rates"].at(2)};
            check(ephbte_set_field(plan, rates), "set_field");
        }
        auto f = rd<double>("f.bin", static_cast<size_t>(B) * S);
        void *fe = dv.up(f), *fg = dv.up(f);
        check(ephbte_rt_step(plan, B, fe, S, dN, dt, n, 0, nullptr), "rt_step eager");
        check(ephbte_rt_step(plan, B, fg, S, dN, dt, n, 1, nullptr), "rt_step graph");
        wr("out_f.bin", dv.down(fe, static_cast<size_t>(B) * S));
        wr("out_f_graph.bin", dv.down(fg, static_cast<size_t>(B) * S));
    } else if (mode == "coupled") {
        const double dt = meta("dt");
        const int n = static_cast<int>(meta("steps"));
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        void *df = dv.up(f);
        check(ephbte_rt_step_coupled(plan, df, dN, dt, n, nullptr), "rt_step_coupled");
        wr("out_f.bin", dv.down(df, static_cast<size_t>(S)));
        wr("out_N.bin", dv.down(dN, nqm));
    } else if (mode == "update_g2") {
        // new |g|^2 (caller order, FP64 on the device), then the forward pass
        auto g2n = rd<double>("g2_new.bin", static_cast<size_t>(nch));
        double *dg = nullptr;
        hipMalloc(reinterpret_cast<void **>(&dg), 8 * static_cast<size_t>(nch));
        hipMemcpy(dg, g2n.data(), 8 * static_cast<size_t>(nch), hipMemcpyHostToDevice);
        check(ephbte_update_g2(plan, dg, nullptr), "update_g2");
        auto f = rd<double>("f.bin", static_cast<size_t>(B) * S);
        void *df = dv.up(f), *dI = dv.alloc(static_cast<size_t>(B) * S);
        check(ephbte_collision_integral(plan, B, df, S, dN, 0, dI, S, nullptr), "collision_integral");
        wr("out_I.bin", dv.down(dI, static_cast<size_t>(B) * S));
        void *dr = dv.alloc(nqm);
        check(ephbte_phonon_rate(plan, df, dN, dr, nullptr), "phonon_rate");
        wr("out_rate.bin", dv.down(dr, nqm));
    } else if (mode == "autotune") {
        // tune twice with one cache file: the second call reads the entry back
        const std::string cache = g_dir + "/tune.json";
        ephbte_tuning a{}, b{};
        check(ephbte_autotune(plan, B, &a, cache.c_str()), "autotune");
        check(ephbte_autotune(plan, B, &b, cache.c_str()), "autotune (cached)");
        wr("out_tune.bin", {double(a.chunk_entries), double(a.block_threads), double(a.batch_partners),
                            double(b.chunk_entries), double(b.block_threads), double(b.batch_partners)});
        auto f = rd<double>("f.bin", static_cast<size_t>(B) * S);
        void *df = dv.up(f), *dI = dv.alloc(static_cast<size_t>(B) * S);
        check(ephbte_collision_integral(plan, B, df, S, dN, 0, dI, S, nullptr), "collision_integral");
        wr("out_I.bin", dv.down(dI, static_cast<size_t>(B) * S));
    } else if (mode == "tiles") {
        // tile tables of the plan (device memory is host memory here): every
        // LDS tile has a window of 1 .. cap states that holds every partner of
        // its chunks, and the tiles cover the chunks in order
        struct Set { const TileRec *t; int64_t n; const int64_t *beg, *end; int64_t nch; int cap; };
        const Set sets[3] = {
            {plan->tiles, plan->n_tiles, plan->chunk_beg, nullptr, plan->n_chunks, plan->lds_states},
            {plan->small_tiles, plan->n_small_tiles, plan->chunk_beg, nullptr, plan->n_chunks, plan->lds_states},
            {plan->sym_tiles, plan->n_sym_tiles, plan->sym_chunk_beg, plan->sym_chunk_end, plan->n_sym_chunks,
             plan->sym_lds_states}};
        std::vector<double> bad(3, 0.0);
        for (int k = 0; k < 3; ++k) {
            const Set &x = sets[k];
            int64_t next = 0;
            for (int64_t i = 0; i < x.n; ++i) {
                const TileRec t = x.t[i];
                if (t.c0 != next || t.c1 < t.c0) bad[k] += 1;
                next = t.c1;
                if (!t.lds) continue;
                if (t.p_hi < t.p_lo || t.p_hi - t.p_lo + 1 > x.cap || t.p_lo < 0 || t.p_hi >= S) bad[k] += 1;
                for (int64_t c = t.c0; c < t.c1; ++c) {
                    const int64_t e1 = x.end ? x.end[c] : x.beg[c + 1];
                    for (int64_t e = x.beg[c]; e < e1; ++e) {
                        const int p = static_cast<int>(plan->pnu[e] >> 3);
                        if (p < t.p_lo || p > t.p_hi) bad[k] += 1;
                    }
                }
            }
            if (next != x.nch) bad[k] += 1;
        }
        // pair-record tiles: the same, and in a q-ordered tile (lds = 2) every
        // word decodes to a pair (d, p), p_lo <= d < p <= p_hi, that is the
        // record the host permutation names, the rows of q = k_p - k_d are
        // non-decreasing, and the permutation is one
        double bad_pr = 0, n_q = 0;
        if (plan->pr_ok) {
            const int64_t np = plan->pr_np;
            std::vector<int64_t> row_of_rec(static_cast<size_t>(np));
            for (int64_t d = 0; d < S; ++d)
                for (int64_t y = plan->pr_rowptr[d]; y < plan->pr_rowptr[d + 1]; ++y) row_of_rec[y] = d;
            std::vector<char> seen(static_cast<size_t>(np), 0);
            ephbte::RowKey rk;
            rk.key = plan->st_key.data();
            rk.padq = plan->padq;
            rk.qoff = plan->qoff;
            for (int a = 0; a < 3; ++a) rk.n[a] = plan->nq[a];
            const int shift = plan->pair_shift;
            int64_t next = 0;
            for (int64_t i = 0; i < plan->n_pr_tiles; ++i) {
                const TileRec t = plan->pr_tiles[i];
                if (t.c0 != next || t.c1 < t.c0) bad_pr += 1;
                next = t.c1;
                if (t.lds && (t.p_hi < t.p_lo || t.p_hi - t.p_lo + 1 > plan->pr_lds_states || t.p_lo < 0 ||
                              t.p_hi >= S))
                    bad_pr += 1;
                n_q += t.lds == 2;
                int64_t last_row = -1;
                for (int64_t c = t.c0; c < t.c1; ++c)
                    for (int64_t x = plan->pr_chunk_beg[c]; x < plan->pr_chunk_end[c]; ++x) {
                        const uint32_t w = plan->pr_partner[x];
                        const int64_t y = plan->pr_perm.empty() ? x : plan->pr_perm[x];
                        if (y < 0 || y >= np || seen[y]) {
                            bad_pr += 1;
                            continue;
                        }
                        seen[y] = 1;
                        int64_t d, p;
                        if (t.lds == 2) {
                            d = t.p_lo + static_cast<int64_t>(w & 0xffffu);
                            p = t.p_lo + static_cast<int64_t>(w >> 16);
                            const int64_t r =
                                ephbte::row_of(rk, static_cast<int32_t>(d), static_cast<int32_t>(p)) >> shift;
                            if (r < last_row) bad_pr += 1;
                            last_row = r;
                            if (d < t.p_lo || p > t.p_hi || d >= p) bad_pr += 1;
                        } else {
                            d = row_of_rec[y];
                            p = w;
                            if (t.lds && (p < t.p_lo || p > t.p_hi)) bad_pr += 1;
                        }
                        if (d != row_of_rec[y] || p != static_cast<int64_t>(plan->pr_partner_host[y])) bad_pr += 1;
                    }
            }
            if (next != plan->n_pr_chunks) bad_pr += 1;
            for (int64_t y = 0; y < np; ++y) bad_pr += seen[y] ? 0 : 1;
        }
        bad.push_back(bad_pr);
        bad.push_back(-n_q);
        bad.push_back(plan->pr_all_q ? 1.0 : 0.0);
        wr("out_tiles.bin", bad);
    } else if (mode == "phonon") {
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dr = dv.alloc(nqm);
        check(ephbte_phonon_rate(plan, df, dN, dr, nullptr), "phonon_rate");
        wr("out_rate.bin", dv.down(dr, nqm));
    } else if (mode == "vjp_nph") {
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        auto lam = rd<double>("lam.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dl = dv.up(lam), *dg = dv.alloc(nqm);
        check(ephbte_collision_vjp_nph(plan, df, dN, dl, dg, nullptr), "collision_vjp_nph");
        wr("out_gN.bin", dv.down(dg, nqm));
    } else if (mode == "phonon_vjp") {
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        auto mu = rd<double>("mu.bin", nqm);
        void *df = dv.up(f), *dm = dv.up(mu), *dgf = dv.alloc(static_cast<size_t>(S)), *dgN = dv.alloc(nqm);
        std::vector<double> fill(static_cast<size_t>(nch), 0.25);
        double *dgg = nullptr;
        hipMalloc(reinterpret_cast<void **>(&dgg), 8 * static_cast<size_t>(nch));
        hipMemcpy(dgg, fill.data(), 8 * static_cast<size_t>(nch), hipMemcpyHostToDevice);
        check(ephbte_phonon_rate_vjp(plan, df, dN, dm, dgf, dgN, dgg, 1, nullptr), "phonon_rate_vjp");
        wr("out_gf.bin", dv.down(dgf, static_cast<size_t>(S)));
        wr("out_gN.bin", dv.down(dgN, nqm));
        std::vector<double> gg(static_cast<size_t>(nch));
        hipMemcpy(gg.data(), dgg, 8 * static_cast<size_t>(nch), hipMemcpyDeviceToHost);
        wr("out_gg2.bin", gg);   // accumulated onto 0.25
    } else if (mode == "coupled_adjoint") {
        const double dt = meta("dt");
        const int n = static_cast<int>(meta("steps"));
        const int ce = static_cast<int>(meta("ce"));
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        auto gfT = rd<double>("gT.bin", static_cast<size_t>(S));
        auto gNT = rd<double>("gNT.bin", nqm);
        void *df = dv.up(f), *dgT = dv.up(gfT), *dgNT = dv.up(gNT);
        void *dgf = dv.alloc(static_cast<size_t>(S)), *dgN = dv.alloc(nqm);
        double *dgg = nullptr;
        hipMalloc(reinterpret_cast<void **>(&dgg), 8 * static_cast<size_t>(nch));
        check(ephbte_rt_adjoint_coupled(plan, df, dN, dt, n, ce, dgT, dgNT, dgf, dgN, dgg, 0, nullptr),
              "rt_adjoint_coupled");
        wr("out_gf.bin", dv.down(dgf, static_cast<size_t>(S)));
        wr("out_gN.bin", dv.down(dgN, nqm));
        std::vector<double> gg(static_cast<size_t>(nch));
        hipMemcpy(gg.data(), dgg, 8 * static_cast<size_t>(nch), hipMemcpyDeviceToHost);
        wr("out_gg2.bin", gg);
    } else if (mode == "adjoint") {
        if (g_meta.count("rates")) {
            const double rates[3] = {g_meta["rates"].at(0), g_meta["rates"].at(1), g_meta["rates"].at(2)};
            check(ephbte_set_field(plan, rates), "set_field");
        }
        const double dt = meta("dt");
        const int n = static_cast<int>(meta("steps"));
        const int ce = static_cast<int>(meta("ce"));
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        auto gT = rd<double>("gT.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dgT = dv.up(gT), *dgf = dv.alloc(static_cast<size_t>(S));
        double *dgg = nullptr;
        hipMalloc(reinterpret_cast<void **>(&dgg), 8 * static_cast<size_t>(nch));
        check(ephbte_rt_adjoint(plan, df, dN, dt, n, ce, dgT, dgf, dgg, 0, nullptr), "rt_adjoint");
        wr("out_gf.bin", dv.down(dgf, static_cast<size_t>(S)));
        std::vector<double> gg(static_cast<size_t>(nch));
        hipMemcpy(gg.data(), dgg, 8 * static_cast<size_t>(nch), hipMemcpyDeviceToHost);
        wr("out_gg2.bin", gg);
    } else if (mode == "bose_rejects") {
        // entry points defined for Fermi statistics only: status of each call
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dx = dv.alloc(static_cast<size_t>(S)), *dr = dv.alloc(nqm);
        std::vector<double> st;
        st.push_back(ephbte_collision_integral_noalloc(plan, df, dN, dx, nullptr));
        st.push_back(ephbte_phonon_rate(plan, df, dN, dr, nullptr));
        st.push_back(ephbte_rt_step_coupled(plan, df, dr, 1.0, 1, nullptr));
        const double rates[3] = {0.01, 0.0, 0.0};
        st.push_back(ephbte_set_field(plan, rates));
        double mob[9];
        st.push_back(ephbte_iterate_transport(plan, df, dx, 300.0, dN, 0.0, 1, nullptr, mob, nullptr, nullptr,
                                              nullptr));
        wr("out_status.bin", st);
    } else if (mode == "tuning_rejects") {
        // out-of-range tuning knobs are rejected and leave the plan as it was;
        // then the forward pass still gives I
        std::vector<double> st;
        auto one = [&](auto setf) {
            ephbte_tuning t{};
            setf(t);
            st.push_back(ephbte_set_tuning(plan, &t));
        };
        one([](ephbte_tuning &t) { t.pair_order = 3; });
        one([](ephbte_tuning &t) { t.pair_order = -1; });
        one([](ephbte_tuning &t) { t.pair_rows = 3; });
        one([](ephbte_tuning &t) { t.pair_rows = 131072; });
        one([](ephbte_tuning &t) { t.pair_rows = -2; });
        one([](ephbte_tuning &t) { t.pair_threads = 640; });
        one([](ephbte_tuning &t) { t.pair_window = 32; });
        one([](ephbte_tuning &t) { t.table_order = 3; });
        wr("out_status.bin", st);
        auto f = rd<double>("f.bin", static_cast<size_t>(S));
        void *df = dv.up(f), *dI = dv.alloc(static_cast<size_t>(S));
        check(ephbte_collision_integral(plan, 1, df, S, dN, 0, dI, S, nullptr), "collision_integral");
        wr("out_I.bin", dv.down(dI, static_cast<size_t>(S)));
    } else if (mode == "transport") {
        auto f0 = rd<double>("f.bin", static_cast<size_t>(S));
        auto vel = rd<double>("vel.bin", static_cast<size_t>(S) * 3);
        void *df = dv.up(f0), *dv3 = dv.up(vel), *dx = dv.alloc(static_cast<size_t>(S) * 3);
        double mob[9], resid = 0;
        int32_t iters = 0;
        const ephbte_status st = ephbte_iterate_transport(plan, df, dv3, meta("T"), dN, meta("tol"),
                                                          static_cast<int32_t>(meta("max_iter")), dx,
                                                          mob, &iters, &resid, nullptr);
        if (st != EPHBTE_OK && st != EPHBTE_NOT_CONVERGED) check(st, "iterate_transport");
        wr("out_mob.bin", std::vector<double>(mob, mob + 9));
        wr("out_x.bin", dv.down(dx, static_cast<size_t>(S) * 3));
        wr("out_iters.bin", {static_cast<double>(iters), resid});
    } else {
        fprintf(stderr, "unknown mode %s\n", mode.c_str());
        return 2;
    }
    printf("%s: %lld launches, %lld workgroups\n", mode.c_str(), emu::n_launch, emu::n_blocks);
    ephbte_destroy(plan);
    return 0;
}
