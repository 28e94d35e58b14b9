// Host-side channel layout builder (see layout.hpp).
#include "layout.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <sstream>
#include <thread>
#include <unordered_map>

namespace ephbte {

int host_threads() {
    const char *env = std::getenv("EPHBTE_HOST_THREADS");
    if (env && std::atoi(env) > 0) return std::atoi(env);
    unsigned hc = std::thread::hardware_concurrency();
    int t = hc ? static_cast<int>(hc) : 1;
    return std::min(t, 16);
}

void parallel_ranges(int64_t n, int threads,
                     const std::function<void(int, int64_t, int64_t)> &fn) {
    if (threads < 1) threads = 1;
    if (n < 4096 || threads == 1) {
        fn(0, 0, n);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) {
        int64_t b = n * t / threads, e = n * (t + 1) / threads;
        pool.emplace_back([&, t, b, e] { fn(t, b, e); });
    }
    for (auto &th : pool) th.join();
}

namespace {

void k_coords(int64_t lin, const int32_t g[3], int32_t c[3]) {
    c[2] = static_cast<int32_t>(lin % g[2]);
    lin /= g[2];
    c[1] = static_cast<int32_t>(lin % g[1]);
    c[0] = static_cast<int32_t>(lin / g[1]);
}

std::string fmt_channel(int64_t c, int32_t i, int32_t j, int nu) {
    std::ostringstream os;
    os << "channel " << c << " (i=" << i << ", j=" << j << ", nu=" << nu << ")";
    return os.str();
}

}  // namespace

ephbte_status build_host_layout(const ephbte_problem *p, const ephbte_build_opts *opts,
                                HostLayout *out, std::string *err) {
    auto bad = [&](const std::string &m) {
        *err = m;
        return EPHBTE_INVALID_ARGUMENT;
    };
    if (!p) return bad("problem is NULL");
    double e_nsig = 0.0, g2_min = 0.0;
    uint32_t elastic = 0;
    if (opts) {
        e_nsig = opts->energy_nsigma;
        g2_min = opts->g2_min;
        elastic = opts->elastic_modes;
        if (!std::isfinite(e_nsig) || e_nsig < 0.0) return bad("energy_nsigma must be finite and >= 0");
        if (!std::isfinite(g2_min) || g2_min < 0.0) return bad("g2_min must be finite and >= 0");
        if (opts->statistics != 0 && opts->statistics != 1)
            return bad("statistics must be 0 (Fermi) or 1 (Bose)");
        for (int32_t x : opts->reserved)
            if (x != 0) return bad("reserved build options must be 0");
    }
    if (p->dtype != EPHBTE_F32 && p->dtype != EPHBTE_F64) {
        *err = "dtype must be EPHBTE_F32 (1) or EPHBTE_F64 (2)";
        return EPHBTE_UNSUPPORTED_DTYPE;
    }
    const int32_t S = p->n_states;
    if (S < 1 || S >= (1 << 29)) return bad("n_states must be in [1, 2^29)");
    if (!p->state_k || !p->eps) return bad("state_k and eps must be non-NULL");
    if (p->n_modes < 1 || p->n_modes > 8) return bad("n_modes must be in [1, 8]");
    if (!p->hw) return bad("hw must be non-NULL");
    if (p->n_channels < 0 || p->n_channels >= (int64_t(1) << 30))
        return bad("n_channels must be in [0, 2^30)");
    if (p->n_channels > 0 && (!p->ch_i || !p->ch_j || !p->ch_nu || !p->g2))
        return bad("channel arrays must be non-NULL when n_channels > 0");
    if (!(p->sigma > 0.0) || !std::isfinite(p->sigma)) return bad("sigma must be finite and > 0");
    if (!(p->n_q_norm > 0.0) || !std::isfinite(p->n_q_norm))
        return bad("n_q_norm must be finite and > 0");
    int64_t nk = 1, nq = 1;
    int32_t r[3];
    for (int a = 0; a < 3; ++a) {
        if (p->kgrid[a] < 1 || p->qgrid[a] < 1) return bad("grid sizes must be >= 1");
        if (p->qgrid[a] > 1024) return bad("q grid sizes must be <= 1024");
        if (p->kgrid[a] % p->qgrid[a] != 0) return bad("q grid must divide the k grid");
        r[a] = p->kgrid[a] / p->qgrid[a];
        nk *= p->kgrid[a];
        nq *= p->qgrid[a];
    }
    if (nk >= (int64_t(1) << 31)) return bad("k grid has too many points");
    const int nm = p->n_modes;
    if (elastic >> nm) return bad("elastic_modes names a mode >= n_modes");
    for (int64_t x = 0; x < nq * nm; ++x) {
        if (!std::isfinite(p->hw[x]) || p->hw[x] < 0.0) return bad("hw must be finite and >= 0");
        if (((elastic >> (x % nm)) & 1u) && p->hw[x] != 0.0) return bad("hw of an elastic mode must be 0");
    }
    // both orientations of a channel use their own q (q and -q); the two
    // contributions cancel exactly only for tables even in q
    for (int32_t a0 = 0; a0 < p->qgrid[0]; ++a0)
        for (int32_t a1 = 0; a1 < p->qgrid[1]; ++a1)
            for (int32_t a2 = 0; a2 < p->qgrid[2]; ++a2) {
                int64_t q = (int64_t(a0) * p->qgrid[1] + a1) * p->qgrid[2] + a2;
                int64_t m = (int64_t((p->qgrid[0] - a0) % p->qgrid[0]) * p->qgrid[1] +
                             (p->qgrid[1] - a1) % p->qgrid[1]) * p->qgrid[2] +
                            (p->qgrid[2] - a2) % p->qgrid[2];
                for (int nu = 0; nu < nm; ++nu) {
                    double x = p->hw[q * nm + nu], y = p->hw[m * nm + nu];
                    if (std::fabs(x - y) > 1e-9 * std::max(std::fabs(x), std::fabs(y)))
                        return bad("hw must be even in q (hw(-q) = hw(q))");
                }
            }

    HostLayout &L = *out;
    L.S = S;
    L.n_modes = nm;
    for (int a = 0; a < 3; ++a) L.nq[a] = p->qgrid[a];
    L.kq.resize(S);
    std::vector<int32_t> kc(3 * static_cast<size_t>(S));
    for (int32_t s = 0; s < S; ++s) {
        int64_t k = p->state_k[s];
        if (k < 0 || k >= nk) return bad("state_k out of range for the k grid");
        if (!std::isfinite(p->eps[s])) return bad("eps must be finite");
        int32_t c[3];
        k_coords(k, p->kgrid, c);
        for (int a = 0; a < 3; ++a) kc[3 * s + a] = c[a];
        L.kq[s] = (static_cast<uint32_t>(c[0] / r[0]) << 20) |
                  (static_cast<uint32_t>(c[1] / r[1]) << 10) | static_cast<uint32_t>(c[2] / r[2]);
    }

    // neighbours of the field term: the state of the same band at k +/- one
    // grid step along each axis
    L.nbr.clear();
    {
        std::unordered_map<int64_t, int32_t> at;
        at.reserve(static_cast<size_t>(S) * 2);
        bool unique = true;
        auto key = [&](int64_t k, int band) { return k * 256 + (band + 128); };
        for (int32_t s = 0; s < S; ++s) {
            const int band = p->state_band ? p->state_band[s] : 0;
            if (!at.emplace(key(p->state_k[s], band), s).second) {
                // a k point held twice in one band (two states without bands,
                // or block-diagonal subsystems drawn from one grid): the field
                // term has no single neighbour and is not available
                unique = false;
                break;
            }
        }
        if (unique) {
            L.nbr.assign(static_cast<size_t>(S) * 6, -1);
            for (int32_t s = 0; s < S; ++s) {
                const int band = p->state_band ? p->state_band[s] : 0;
                for (int a = 0; a < 3; ++a)
                    for (int u = 0; u < 2; ++u) {
                        int32_t c[3] = {kc[3 * s], kc[3 * s + 1], kc[3 * s + 2]};
                        c[a] = (c[a] + (u == 0 ? 1 : p->kgrid[a] - 1)) % p->kgrid[a];
                        const int64_t k = (int64_t(c[0]) * p->kgrid[1] + c[1]) * p->kgrid[2] + c[2];
                        const auto it = at.find(key(k, band));
                        L.nbr[static_cast<size_t>(s) * 6 + 2 * a + u] = it == at.end() ? -1 : it->second;
                    }
            }
        }
    }

    const int64_t nch = p->n_channels;
    const int T = host_threads();
    // --- validate channels (parallel, first error by lowest channel index)
    std::atomic<int64_t> first_bad{INT64_MAX};
    std::vector<std::string> msgs(T);
    // channel selection (paper: scattering-channel paragraph after Eq. 2):
    // approximate energy conservation keeps a channel when one of its two
    // Gaussians, at Delta + hw or Delta - hw, lies within e_nsig standard
    // deviations; couplings below g2_min are discarded
    std::vector<uint8_t> keep(static_cast<size_t>(nch), 1);
    const double e_cut = e_nsig * p->sigma;
    auto q_of = [&](int32_t d, int32_t pp) {
        int32_t q[3];
        for (int a = 0; a < 3; ++a) {
            int32_t dk = kc[3 * pp + a] - kc[3 * d + a];
            if (dk < 0) dk += p->kgrid[a];
            if (dk % r[a] != 0) return int64_t(-1);
            q[a] = dk / r[a];
        }
        return (int64_t(q[0]) * p->qgrid[1] + q[1]) * p->qgrid[2] + q[2];
    };
    parallel_ranges(nch, T, [&](int t, int64_t b, int64_t e) {
        for (int64_t c = b; c < e; ++c) {
            if (c >= first_bad.load(std::memory_order_relaxed)) return;
            int32_t i = p->ch_i[c], j = p->ch_j[c];
            int nu = p->ch_nu[c];
            std::string m;
            if (i < 0 || i >= S || j < 0 || j >= S) m = "state index out of range";
            else if (i == j) m = "i == j (a state cannot scatter into itself)";
            else if (nu < 0 || nu >= nm) m = "mode index out of range";
            else if (!std::isfinite(p->g2[c]) || p->g2[c] < 0.0) m = "|g|^2 must be finite and >= 0";
            else {
                int64_t q1 = q_of(i, j), q2 = q_of(j, i);
                if (q1 < 0 || q2 < 0) m = "k_j - k_i is not a q-grid vector";
                else if (!((elastic >> nu) & 1u) && (p->hw[q1 * nm + nu] < 1e-6 || p->hw[q2 * nm + nu] < 1e-6))
                    m = "phonon energy below 1e-6 eV (divergent occupation)";
                else {
                    const double dl = p->eps[i] - p->eps[j], w = p->hw[q1 * nm + nu];
                    const bool e_ok = e_nsig == 0.0 || std::min(std::fabs(dl + w), std::fabs(dl - w)) < e_cut;
                    keep[c] = (e_ok && p->g2[c] >= g2_min) ? 1 : 0;
                }
            }
            if (!m.empty()) {
                int64_t cur = first_bad.load();
                while (c < cur && !first_bad.compare_exchange_weak(cur, c)) {
                }
                msgs[t] = fmt_channel(c, i, j, nu) + ": " + m;
                return;
            }
        }
    });
    if (first_bad.load() != INT64_MAX) {
        int64_t c = first_bad.load();
        for (auto &m : msgs)
            if (m.rfind(fmt_channel(c, p->ch_i[c], p->ch_j[c], p->ch_nu[c]), 0) == 0) return bad(m);
        return bad("invalid channel");
    }

    L.n_input = nch;
    L.dropped.clear();
    for (int64_t c = 0; c < nch; ++c)
        if (!keep[c]) L.dropped.push_back(static_cast<int32_t>(c));
    const int64_t nkeep = nch - static_cast<int64_t>(L.dropped.size());

    // --- count entries per destination (per-thread histograms)
    L.n_channels = nkeep;
    L.E = 2 * nkeep;
    std::vector<std::vector<int64_t>> cnt(T, std::vector<int64_t>(S, 0));
    parallel_ranges(nch, T, [&](int t, int64_t b, int64_t e) {
        auto &h = cnt[t];
        for (int64_t c = b; c < e; ++c) {
            if (!keep[c]) continue;
            h[p->ch_i[c]]++;
            h[p->ch_j[c]]++;
        }
    });
    L.row_ptr.assign(S + 1, 0);
    for (int32_t d = 0; d < S; ++d) {
        int64_t tot = 0;
        for (int t = 0; t < T; ++t) tot += cnt[t][d];
        L.row_ptr[d + 1] = L.row_ptr[d] + tot;
    }
    // per-thread write cursors: thread t writes after threads 0..t-1
    for (int32_t d = 0; d < S; ++d) {
        int64_t pos = L.row_ptr[d];
        for (int t = 0; t < T; ++t) {
            int64_t n = cnt[t][d];
            cnt[t][d] = pos;
            pos += n;
        }
    }
    L.pnu.resize(L.E);
    L.ent_chan.resize(L.E);
    // stable scatter: inside a destination, entries keep channel order
    parallel_ranges(nch, T, [&](int t, int64_t b, int64_t e) {
        auto &cur = cnt[t];
        for (int64_t c = b; c < e; ++c) {
            if (!keep[c]) continue;
            int32_t i = p->ch_i[c], j = p->ch_j[c];
            int nu = p->ch_nu[c];
            int64_t ei = cur[i]++, ej = cur[j]++;
            L.pnu[ei] = pack_pnu(j, nu);
            L.ent_chan[ei] = static_cast<int32_t>(c);
            L.pnu[ej] = pack_pnu(i, nu);
            L.ent_chan[ej] = static_cast<int32_t>(c);
        }
    });
    cnt.clear();

    // --- sort each destination by (partner, mode); detect duplicates
    std::atomic<int32_t> dup_dest{-1};
    parallel_ranges(S, T, [&](int, int64_t b, int64_t e) {
        std::vector<int64_t> idx;
        std::vector<uint32_t> kb;
        std::vector<int32_t> cb;
        for (int64_t d = b; d < e; ++d) {
            int64_t lo = L.row_ptr[d], hi = L.row_ptr[d + 1];
            bool sorted = true;
            for (int64_t x = lo + 1; x < hi; ++x)
                if (L.pnu[x] <= L.pnu[x - 1]) {
                    sorted = false;
                    break;
                }
            if (sorted) continue;
            idx.resize(hi - lo);
            std::iota(idx.begin(), idx.end(), lo);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int64_t a, int64_t bb) { return L.pnu[a] < L.pnu[bb]; });
            kb.resize(hi - lo);
            cb.resize(hi - lo);
            for (int64_t x = 0; x < hi - lo; ++x) {
                kb[x] = L.pnu[idx[x]];
                cb[x] = L.ent_chan[idx[x]];
            }
            for (int64_t x = 0; x < hi - lo; ++x) {
                L.pnu[lo + x] = kb[x];
                L.ent_chan[lo + x] = cb[x];
                if (x > 0 && kb[x] == kb[x - 1]) dup_dest.store(static_cast<int32_t>(d));
            }
        }
    });
    if (dup_dest.load() >= 0) {
        std::ostringstream os;
        os << "duplicate (i, j, nu) channel at state " << dup_dest.load();
        return bad(os.str());
    }
    // partners are sorted, so the range of destination d is its first and last entry
    L.pmin.assign(S, 0);
    L.pmax.assign(S, -1);
    for (int32_t d = 0; d < S; ++d) {
        if (L.row_ptr[d + 1] > L.row_ptr[d]) {
            L.pmin[d] = static_cast<int32_t>(L.pnu[L.row_ptr[d]] >> 3);
            L.pmax[d] = static_cast<int32_t>(L.pnu[L.row_ptr[d + 1] - 1] >> 3);
        }
    }
    return EPHBTE_OK;
}

ChunkTable make_chunks_seg(const std::vector<int64_t> &seg_beg, const std::vector<int64_t> &seg_end,
                           int64_t chunk_entries) {
    ChunkTable t;
    const int32_t S = static_cast<int32_t>(seg_beg.size());
    if (chunk_entries < 1) chunk_entries = INT64_MAX;
    t.dest_chunk.resize(S + 1);
    t.chunk_beg.reserve(S + 1);
    t.chunk_end.reserve(S);
    for (int32_t d = 0; d < S; ++d) {
        t.dest_chunk[d] = static_cast<int32_t>(t.chunk_dest.size());
        const int64_t lo = seg_beg[d], len = seg_end[d] - seg_beg[d];
        const int64_t nc = len <= chunk_entries ? 1 : (len + chunk_entries - 1) / chunk_entries;
        for (int64_t c = 0; c < nc; ++c) {
            t.chunk_beg.push_back(lo + len * c / nc);
            t.chunk_end.push_back(lo + len * (c + 1) / nc);
            t.chunk_dest.push_back(d);
        }
        if (nc > 1) t.one_per_dest = false;
    }
    t.dest_chunk[S] = static_cast<int32_t>(t.chunk_dest.size());
    t.chunk_beg.push_back(S > 0 ? seg_end[S - 1] : 0);
    t.n_chunks = static_cast<int64_t>(t.chunk_dest.size());
    return t;
}

ChunkTable make_chunks(const std::vector<int64_t> &row_ptr, int64_t chunk_entries) {
    const std::vector<int64_t> beg(row_ptr.begin(), row_ptr.end() - 1), end(row_ptr.begin() + 1, row_ptr.end());
    return make_chunks_seg(beg, end, chunk_entries);
}

std::vector<Tile> make_tiles(const ChunkTable &ct, const std::vector<int64_t> &row_ptr,
                             const std::vector<int32_t> &pmin, const std::vector<int32_t> &pmax,
                             int32_t lds_states, int64_t target_entries) {
    (void)row_ptr;
    std::vector<Tile> tiles;
    if (target_entries < 1) target_entries = 1;
    const int64_t n = ct.n_chunks;
    int64_t c = 0;
    while (c < n) {
        Tile t{c, c, 0, -1, 1, 0};
        int32_t lo = INT32_MAX, hi = -1;
        int64_t ent = 0;
        int kind = -1;   // 1 LDS, 0 global
        while (c < n) {
            const int32_t d = ct.chunk_dest[c];
            const int64_t ce = ct.chunk_end[c] - ct.chunk_beg[c];
            const bool has = pmax[d] >= pmin[d];
            const int32_t nlo = has ? std::min(lo, pmin[d]) : lo;
            const int32_t nhi = has ? std::max(hi, pmax[d]) : hi;
            const int ckind = (!has || int64_t(pmax[d]) - pmin[d] + 1 <= lds_states) ? 1 : 0;
            if (c > t.c0) {
                if (ckind != kind || ent + ce > target_entries) break;
                if (kind == 1 && has && int64_t(nhi) - nlo + 1 > lds_states) break;
            } else {
                kind = ckind;
            }
            if (kind == 1) {
                lo = nlo;
                hi = nhi;
            }
            ent += ce;
            ++c;
        }
        t.c1 = c;
        t.lds = kind;
        if (kind == 1) {
            // a tile whose destinations have no partners still stages one state
            // (state 0): its chunks are empty, but their masked lanes read window
            // slot 0, which must hold a state, not whatever the LDS held before
            t.p_lo = hi >= lo ? lo : 0;
            t.p_hi = hi >= lo ? hi : 0;
        }
        tiles.push_back(t);
    }
    return tiles;
}

std::vector<BTile> make_btiles(const std::vector<int32_t> &pmin, const std::vector<int32_t> &pmax,
                               int32_t pt, int32_t dmax, int32_t window_cap, int64_t *slots) {
    std::vector<BTile> tiles;
    const int32_t S = static_cast<int32_t>(pmin.size());
    int64_t off = 0;
    int32_t d = 0;
    while (d < S) {
        BTile t{d, d, 0, 0, off};
        int32_t lo = INT32_MAX, hi = -1;
        while (d < S && d - t.d0 < dmax) {
            const bool has = pmax[d] >= pmin[d];
            const int32_t nlo = has ? std::min(lo, pmin[d]) : lo;
            const int32_t nhi = has ? std::max(hi, pmax[d]) : hi;
            if (d > t.d0 && has && int64_t(nhi) - nlo + 1 > window_cap) break;
            lo = nlo;
            hi = nhi;
            ++d;
        }
        t.d1 = d;
        if (hi >= lo) {
            t.p_lo = lo;
            t.n_sub = static_cast<int32_t>((int64_t(hi) - lo + pt) / pt);
        }
        off += int64_t(t.d1 - t.d0) * (t.n_sub + 1);
        tiles.push_back(t);
    }
    *slots = off;
    return tiles;
}

}  // namespace ephbte

namespace ephbte {

PhononLayout build_phonon_layout(const HostLayout &L) {
    PhononLayout out;
    const int64_t n0 = L.nq[0], n1 = L.nq[1], n2 = L.nq[2];
    const int64_t nq = n0 * n1 * n2;
    const int nm = L.n_modes;
    // q = k_b - k_a on the q grid (both in q-grid units, 10 bits per axis)
    auto qlin = [&](uint32_t ka, uint32_t kb) {
        int64_t a0 = int64_t(kb >> 20) - int64_t(ka >> 20);
        int64_t a1 = int64_t((kb >> 10) & 1023u) - int64_t((ka >> 10) & 1023u);
        int64_t a2 = int64_t(kb & 1023u) - int64_t(ka & 1023u);
        a0 += a0 < 0 ? n0 : 0;
        a1 += a1 < 0 ? n1 : 0;
        a2 += a2 < 0 ? n2 : 0;
        return (a0 * n1 + a1) * n2 + a2;
    };
    auto neg = [&](int64_t q) {
        const int64_t c2 = q % n2, c1 = (q / n2) % n1, c0 = q / (n1 * n2);
        return (((n0 - c0) % n0) * n1 + (n1 - c1) % n1) * n2 + (n2 - c2) % n2;
    };
    // each channel once: row d, partners p > d; a pair is a run of equal p
    const int T = host_threads();
    const int64_t S = L.S;
    std::vector<int64_t> ranges(T + 1);
    for (int t = 0; t <= T; ++t) ranges[t] = S * t / T;
    std::vector<std::vector<int64_t>> cnt(T, std::vector<int64_t>(static_cast<size_t>(nq), 0));
    auto for_pairs = [&](int64_t d0, int64_t d1, auto &&fn) {
        for (int64_t d = d0; d < d1; ++d) {
            int64_t x = L.row_ptr[d];
            const int64_t e = L.row_ptr[d + 1];
            while (x < e && static_cast<int64_t>(L.pnu[x] >> 3) <= d) ++x;
            while (x < e) {
                const uint32_t p = L.pnu[x] >> 3;
                int64_t y = x;
                uint32_t modes = 0;
                while (y < e && (L.pnu[y] >> 3) == p) {
                    modes |= 1u << (L.pnu[y] & 7u);
                    ++y;
                }
                if (modes) {
                    const int64_t q = qlin(L.kq[d], L.kq[p]), qm = neg(q);
                    fn(d, static_cast<int64_t>(p), x, y, std::min(q, qm), q <= qm);
                }
                x = y;
            }
        }
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t)
        pool.emplace_back([&, t] {
            for_pairs(ranges[t], ranges[t + 1],
                      [&](int64_t, int64_t, int64_t, int64_t, int64_t qc, bool) { ++cnt[t][qc]; });
        });
    for (auto &th : pool) th.join();
    pool.clear();
    // buckets in order of qc; thread t's pairs of a bucket follow those of
    // threads < t, and each thread walks its rows in order, so every bucket is
    // ordered by (d, p) whatever the split
    std::vector<int64_t> qbeg(static_cast<size_t>(nq) + 1, 0);
    for (int64_t q = 0; q < nq; ++q) {
        int64_t c = 0;
        for (int t = 0; t < T; ++t) c += cnt[t][q];
        qbeg[q + 1] = qbeg[q] + c;
    }
    out.n_pairs = qbeg[nq];
    for (int64_t q = 0; q < nq; ++q) {
        int64_t o = qbeg[q];
        for (int t = 0; t < T; ++t) {
            const int64_t c = cnt[t][q];
            cnt[t][q] = o;
            o += c;
        }
    }
    const int64_t np = out.n_pairs;
    out.pa.resize(np);
    out.pb.resize(np);
    out.slot_chan.assign(static_cast<size_t>(nm) * np, -1);
    std::vector<uint32_t> qmodes(static_cast<size_t>(nq), 0);
    std::vector<std::vector<uint32_t>> tmodes(T);
    for (int t = 0; t < T; ++t)
        pool.emplace_back([&, t] {
            auto &pos = cnt[t];
            for_pairs(ranges[t], ranges[t + 1],
                      [&](int64_t d, int64_t p, int64_t x, int64_t y, int64_t qc, bool fwd) {
                          const int64_t i = pos[qc]++;
                          out.pa[i] = static_cast<uint32_t>(fwd ? d : p);
                          out.pb[i] = static_cast<uint32_t>(fwd ? p : d);
                          for (int64_t z = x; z < y; ++z)
                              out.slot_chan[static_cast<size_t>(L.pnu[z] & 7u) * np + i] = L.ent_chan[z];
                      });
        });
    for (auto &th : pool) th.join();
    // modes present per bucket (from the slots, in one pass)
    out.q_bucket.assign(static_cast<size_t>(nq), -1);
    out.bucket_beg.push_back(0);
    for (int64_t q = 0; q < nq; ++q) {
        if (qbeg[q + 1] == qbeg[q]) continue;
        uint32_t modes = 0;
        for (int m = 0; m < nm; ++m)
            for (int64_t i = qbeg[q]; i < qbeg[q + 1]; ++i)
                if (out.slot_chan[static_cast<size_t>(m) * np + i] >= 0) {
                    modes |= 1u << m;
                    break;
                }
        const int64_t b = static_cast<int64_t>(out.bucket_q.size());
        const int64_t qm = neg(q);
        out.bucket_q.push_back(static_cast<int32_t>(q));
        out.bucket_qm.push_back(static_cast<int32_t>(qm));
        out.bucket_modes.push_back(modes);
        out.bucket_beg.push_back(qbeg[q + 1]);
        out.q_bucket[q] = static_cast<int32_t>(2 * b);
        if (qm != q) out.q_bucket[qm] = static_cast<int32_t>(2 * b + 1);
    }
    return out;
}

}  // namespace ephbte

namespace ephbte {

PairRows build_pair_rows(const HostLayout &L) {
    PairRows out;
    const int64_t S = L.S;
    const int nm = L.n_modes;
    out.row_ptr.assign(static_cast<size_t>(S) + 1, 0);
    // first entry of row d with partner > d: entries are sorted by (partner, mode)
    auto upper = [&](int64_t d) {
        const auto lo = L.pnu.begin() + L.row_ptr[d], hi = L.pnu.begin() + L.row_ptr[d + 1];
        return static_cast<int64_t>(std::lower_bound(lo, hi, static_cast<uint32_t>(d + 1) << 3) - L.pnu.begin());
    };
    std::vector<int64_t> cnt(static_cast<size_t>(S), 0);
    parallel_ranges(S, host_threads(), [&](int, int64_t b, int64_t e) {
        for (int64_t d = b; d < e; ++d) {
            int64_t n = 0;
            uint32_t last = 0xffffffffu;
            for (int64_t x = upper(d); x < L.row_ptr[d + 1]; ++x) {
                const uint32_t p = L.pnu[x] >> 3;
                n += p != last;
                last = p;
            }
            cnt[d] = n;
        }
    });
    for (int64_t d = 0; d < S; ++d) out.row_ptr[d + 1] = out.row_ptr[d] + cnt[d];
    const int64_t np = out.row_ptr[S];
    out.n_pairs = np;
    out.partner.resize(static_cast<size_t>(np));
    out.slot_chan.assign(static_cast<size_t>(nm) * np, -1);
    std::vector<int64_t> filled(static_cast<size_t>(host_threads()) + 1, 0);
    parallel_ranges(S, host_threads(), [&](int t, int64_t b, int64_t e) {
        int64_t f = 0;
        for (int64_t d = b; d < e; ++d) {
            int64_t j = out.row_ptr[d] - 1;
            uint32_t last = 0xffffffffu;
            for (int64_t x = upper(d); x < L.row_ptr[d + 1]; ++x) {
                const uint32_t p = L.pnu[x] >> 3;
                if (p != last) out.partner[++j] = p;
                last = p;
                out.slot_chan[static_cast<size_t>(L.pnu[x] & 7u) * np + j] = L.ent_chan[x];
                ++f;
            }
        }
        filled[t] = f;
    });
    for (int64_t f : filled) out.n_filled += f;
    return out;
}

int64_t row_of(const RowKey &k, int32_t d, int32_t p) {
    const uint32_t kd = k.key[d], kp = k.key[p];
    if (k.padq) return static_cast<int64_t>(static_cast<int32_t>(kp - kd)) + k.qoff;
    int64_t q = 0;
    for (int a = 0; a < 3; ++a) {
        const int sh = 20 - 10 * a;
        int v = static_cast<int>((kp >> sh) & 1023u) - static_cast<int>((kd >> sh) & 1023u);
        v += v < 0 ? k.n[a] : 0;
        q = q * k.n[a] + v;
    }
    return q;
}

PairOrder order_pair_tiles(const ChunkTable &pc, const std::vector<Tile> &tiles,
                           const std::vector<uint32_t> &partner, const RowKey &rk, int chunks_per_tile,
                           int64_t max_chunk) {
    PairOrder o;
    const int64_t np = static_cast<int64_t>(partner.size());
    const int64_t nt = static_cast<int64_t>(tiles.size());
    const int32_t S = static_cast<int32_t>(pc.dest_chunk.size()) - 1;
    if (chunks_per_tile < 1) chunks_per_tile = 1;
    if (max_chunk < 1) max_chunk = 1;
    o.perm.resize(static_cast<size_t>(np));
    o.word.resize(static_cast<size_t>(np));
    parallel_ranges(np, host_threads(), [&](int, int64_t b, int64_t e) {
        for (int64_t x = b; x < e; ++x) {
            o.perm[x] = static_cast<uint32_t>(x);
            o.word[x] = partner[x];
        }
    });
    // the tiles that go to q order, and their record ranges
    std::vector<int64_t> r0(static_cast<size_t>(nt), 0), r1(static_cast<size_t>(nt), 0);
    std::vector<char> qt(static_cast<size_t>(nt), 0);
    for (int64_t i = 0; i < nt; ++i) {
        const Tile &t = tiles[i];
        if (t.c1 <= t.c0) continue;
        r0[i] = pc.chunk_beg[t.c0];
        r1[i] = pc.chunk_end[t.c1 - 1];
        qt[i] = t.lds == 1 && int64_t(t.p_hi) - t.p_lo < 65536;
    }
    parallel_ranges(nt, host_threads(), [&](int, int64_t b, int64_t e) {
        std::vector<std::pair<uint64_t, uint32_t>> keys;
        for (int64_t i = b; i < e; ++i) {
            if (!qt[i]) continue;
            const Tile &t = tiles[i];
            keys.clear();
            bool ok = true;
            for (int64_t c = t.c0; c < t.c1 && ok; ++c) {
                const int32_t d = pc.chunk_dest[c];
                for (int64_t x = pc.chunk_beg[c]; x < pc.chunk_end[c]; ++x) {
                    const int32_t p = static_cast<int32_t>(partner[x]);
                    if (d < t.p_lo || d > t.p_hi || p < t.p_lo || p > t.p_hi) {
                        ok = false;
                        break;
                    }
                    const uint64_t row = static_cast<uint64_t>(row_of(rk, d, p) >> rk.shift);
                    keys.emplace_back((row << 32) | (static_cast<uint64_t>(d - t.p_lo) << 16) |
                                          static_cast<uint64_t>(p - t.p_lo),
                                      static_cast<uint32_t>(x));
                }
            }
            if (!ok) {
                qt[i] = 0;   // window does not hold the destinations: destination order
                continue;
            }
            std::sort(keys.begin(), keys.end());
            for (size_t j = 0; j < keys.size(); ++j) {
                const size_t at = static_cast<size_t>(r0[i]) + j;
                const uint64_t k = keys[j].first;
                o.perm[at] = keys[j].second;
                o.word[at] = (static_cast<uint32_t>(k & 0xffffu) << 16) | static_cast<uint32_t>((k >> 16) & 0xffffu);
            }
        }
    });
    // the renumbered chunk table
    ChunkTable &ct = o.chunks;
    ct.dest_chunk.assign(static_cast<size_t>(S) + 1, 0);
    std::vector<int32_t> new_of_old(static_cast<size_t>(pc.n_chunks), 0);
    o.tiles = tiles;
    bool any_q = false;
    for (int64_t i = 0; i < nt; ++i) {
        Tile &t = o.tiles[i];
        const int64_t c0 = static_cast<int64_t>(ct.chunk_dest.size());
        if (qt[i]) {
            any_q = true;
            const int64_t len = r1[i] - r0[i];
            const int64_t per = static_cast<int64_t>(chunks_per_tile) * max_chunk;
            const int64_t k = static_cast<int64_t>(chunks_per_tile) * std::max<int64_t>(1, (len + per - 1) / per);
            for (int64_t j = 0; j < k; ++j) {
                ct.chunk_beg.push_back(r0[i] + len * j / k);
                ct.chunk_end.push_back(r0[i] + len * (j + 1) / k);
                ct.chunk_dest.push_back(pc.chunk_dest[t.c0]);
            }
            for (int64_t c = t.c0; c < t.c1; ++c) new_of_old[c] = static_cast<int32_t>(c0);
            t.lds = 2;
        } else {
            for (int64_t c = t.c0; c < t.c1; ++c) {
                new_of_old[c] = static_cast<int32_t>(ct.chunk_dest.size());
                ct.chunk_beg.push_back(pc.chunk_beg[c]);
                ct.chunk_end.push_back(pc.chunk_end[c]);
                ct.chunk_dest.push_back(pc.chunk_dest[c]);
            }
        }
        t.c0 = c0;
        t.c1 = static_cast<int64_t>(ct.chunk_dest.size());
    }
    ct.n_chunks = static_cast<int64_t>(ct.chunk_dest.size());
    for (int32_t d = 0; d < S; ++d) {
        const int32_t c = pc.dest_chunk[d];
        ct.dest_chunk[d] = c < pc.n_chunks ? new_of_old[c] : static_cast<int32_t>(ct.n_chunks);
    }
    ct.dest_chunk[S] = static_cast<int32_t>(ct.n_chunks);
    ct.chunk_beg.push_back(pc.chunk_beg.empty() ? 0 : pc.chunk_beg.back());
    ct.one_per_dest = pc.one_per_dest && !any_q;
    return o;
}

}  // namespace ephbte

