// HIP kernels (gfx950) for the e-ph collision integral and its consumers.
//
// Data layout in HBM (built once by layout.cpp, uploaded by api.hip):
//   pnu [E]  u32   partner << 3 | mode, sorted by (destination, partner, mode)
//   g2  [E]  T     |g|^2 of the entry's channel (each channel stored twice)
//   st  [S]  {T eps; u32 kq}   state energy and k in q-grid units (10 bits/axis)
//   hw  [Nq][n_modes] T, nph [Nq][n_modes] T (caller's occupations)
//   chunk_beg [n_chunks+1] i64, chunk_dest [n_chunks] i32: workgroup work items,
//   each a contiguous run of one destination's entries.
//
// One workgroup reduces one chunk: its threads stride the chunk's entries
// (coalesced pnu/g2 streams), gather the partner's state record, occupation
// and phonon data (cache resident), evaluate the two Gaussians and fold the
// entry into two running sums, then combine lanes with a fixed
// shuffle tree and waves through LDS in fixed order.  Floating-point sums
// never use atomics; the single-copy pass and the phonon-side rate add
// 64-bit fixed-point integers with integer atomics, which are associative,
// so every result is bitwise reproducible.
//
// Entry algebra (Eq. 2 with the golden-rule occupation factors).  With
// da = exp(-(e_d - e_p + hw)^2 / 2 s^2), de = exp(-(e_d - e_p - hw)^2 / 2 s^2)
// (evaluated as powers of two),
// t = N (da + de):
//   a = g2 (t + de)  (weight of the out-scattering product f_d (1 - f_p))
//   b = g2 (t + da)  (weight of the in-scattering product  f_p (1 - f_d))
// and I_d = K [ (1 - f_d) sum b f_p  -  f_d sum a (1 - f_p) ] with
// K = 2 pi / (hbar N_q) / (s sqrt(2 pi)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ephbte {

// kq:  k in q-grid units, 10 bits per axis (a0 << 20 | a1 << 10 | a2)
// kqp: the same k in shifted coordinates c (0 .. span - 1 per axis) as the
//      linear index (c0 b1 + c1) b2 + c2 on the (b0, b1, b2) = 2 span - 1 box
//      of QBox, so that kqp_p - kqp_d + offset is the box row of q = k_p - k_d
//      (each axis difference + span - 1 lies in [0, b), so no borrow crosses axes)
template <typename T> struct StateRec;
template <> struct alignas(16) StateRec<double> {
    double eps;
    uint32_t kq;
    uint32_t kqp;
};
template <> struct alignas(16) StateRec<float> {
    float eps;
    uint32_t kq;
    uint32_t kqp;
    uint32_t pad;
};

// Base-2 exponential of the (pre-scaled, never positive) Gaussian exponent;
// the log2(e) factor is folded into the exponent scale on the host.
// FP32: the hardware exponential.  FP64: y = n + r with n = rint(y), which
// is exact, so |r| <= 1/2; 2^r = exp(r ln2) by its Taylor series to degree
// 12 (truncation below 2e-16 relative for |r ln2| <= 0.347, Horner form);
// 2^n by ldexp.  y is clamped at -1100, where the result is already 0.
__device__ __forceinline__ double gauss_exp2(double y) {
    y = fmax(y, -1100.0);
    const double n = __builtin_rint(y);
    const double r = y - n;
    // coefficients (ln 2)^k / k!, k = 12 .. 0
    double p = 2.5678435993488196e-11;
    p = fma(p, r, 4.44553827187081e-10);
    p = fma(p, r, 7.054911620801121e-09);
    p = fma(p, r, 1.0178086009239696e-07);
    p = fma(p, r, 1.3215486790144305e-06);
    p = fma(p, r, 1.5252733804059838e-05);
    p = fma(p, r, 0.00015403530393381606);
    p = fma(p, r, 0.0013333558146428441);
    p = fma(p, r, 0.009618129107628477);
    p = fma(p, r, 0.055504108664821576);
    p = fma(p, r, 0.2402265069591007);
    p = fma(p, r, 0.6931471805599453);
    p = fma(p, r, 1.0);
    return ldexp(p, static_cast<int>(n));
}
// Table-driven base-2 exponential (Tang, ACM TOMS 15(2), 1989) for the
// streaming kernels.  Takes y256 = 256 y.  With n = rint(y256) and
// r = y256 - n (exact, |r| <= 1/2): 2^y = 2^(n >> 8) 2^((n & 255)/256) 2^(r/256).
// The middle factor comes from a 256-entry table of 2^(j/256) held in LDS;
// the last is exp(r ln2/256) by its Taylor series to degree 4
// (|r ln2/256| <= 1.36e-3, truncation below 4e-17 relative); coefficients
// (ln2/256)^k / k!.  y256 is clamped where the result is already 0, which
// keeps the integer conversion in range.
__device__ __forceinline__ double gauss_exp2_tab(double y256, const double *tab) {
    y256 = fmax(y256, -300000.0);
    const double n = __builtin_rint(y256);
    const double r = y256 - n;
    double p = 2.239395190875157e-12;
    p = fma(p, r, 3.3083026805413713e-09);
    p = fma(p, r, 3.6655655969101062e-06);
    p = fma(p, r, 0.0027076061740622863);
    p = fma(p, r, 1.0);
    const int i = static_cast<int>(n);
    return ldexp(tab[i & 255] * p, i >> 8);
}

__device__ __forceinline__ double gauss_exp(double a) { return gauss_exp2(a); }
__device__ __forceinline__ float gauss_exp(float a) { return __builtin_amdgcn_exp2f(a); }

template <typename T> struct alignas(4 * sizeof(T)) Vec4 {
    T x, y, z, w;
};

// linear q index of k_p - k_d (both given in q-grid units, 10 bits per axis)
__device__ __forceinline__ int q_linear(uint32_t kd, uint32_t kp, int n0, int n1, int n2) {
    int a0 = static_cast<int>(kp >> 20) - static_cast<int>(kd >> 20);
    int a1 = static_cast<int>((kp >> 10) & 1023u) - static_cast<int>((kd >> 10) & 1023u);
    int a2 = static_cast<int>(kp & 1023u) - static_cast<int>(kd & 1023u);
    a0 += (a0 < 0) ? n0 : 0;
    a1 += (a1 < 0) ? n1 : 0;
    a2 += (a2 < 0) ? n2 : 0;
    return (a0 * n1 + a1) * n2 + a2;
}

// chunk served by this workgroup; with xcd_m > 0 the 8 XCDs (which receive
// workgroups round-robin) each get a contiguous range of chunks, so every
// L2 sees neighbouring destinations
__device__ __forceinline__ int64_t chunk_of_block(int64_t n_chunks, int64_t xcd_m) {
    int64_t b = blockIdx.x;
    if (xcd_m > 0) return (b & 7) * xcd_m + (b >> 3);
    return b;
}

// Tile served by this workgroup.  Workgroups are dispatched to the 8 XCDs
// round-robin (block b runs on XCD b % 8); with xcd set, each XCD gets a
// contiguous range of tiles, so the workgroups sharing one L2 work on
// neighbouring destinations, whose partner and {hw, N} gathers overlap.
// The grid then has 8 ceil(n / 8) blocks; the extra ones get -1.
__device__ __forceinline__ int64_t tile_of_block(int64_t n, int xcd) {
    const int64_t b = blockIdx.x;
    if (!xcd) return b;
    const int64_t t = (b & 7) * ((n + 7) / 8) + (b >> 3);
    return t < n ? t : -1;
}

template <typename T> struct Tables {
    const uint32_t *__restrict__ pnu;
    const T *__restrict__ g2;
    const StateRec<T> *__restrict__ st;
    const T *__restrict__ hw;
    const T *__restrict__ nph;
    const int64_t *__restrict__ chunk_beg;
    const int32_t *__restrict__ chunk_dest;
    const int32_t *__restrict__ dest_chunk;
    const int32_t *__restrict__ ent_chan;
    int64_t n_chunks;
    int64_t xcd_m;
    int S, nm, nq0, nq1, nq2;
    T mc;   // Gaussian exponent scale, base 2: -log2(e) / (2 s^2)
    T K;    // 2 pi / (hbar N_q) / (s sqrt(2 pi))
};

// Per-destination epilogue applied to the value v = I_d (forward) or
// v = dL/df_d (reverse), for vector b.
template <typename T> struct Epi {
    int mode;              // see apply_epi
    T *out;                // mode 0: output [B][ld_out]
    int64_t ld_out;
    const T *f0;           // RK4: step start f (caller layout, ld_f0)
    int64_t ld_f0;
    T *u_out;              // RK4: next stage input [B][S]
    T *acc;                // RK4: k1 + 2k2 + 2k3 accumulator [B][S]
    T *f_out;              // RK4 stage 4: f at the end of the step (ld_f0)
    T dt;
    // adjoint stages: lam_out = cg * gbar + cv * v
    const T *gbar;
    T *gbar_out;
    T cg, cv;
    // field term of Eq. 1 (RK and adjoint modes, when nbr is set): v gains
    // dsign * D[x], D[x]_d = -sum_a rate[a] (x[up_a] - x[down_a]) / 2, with x the
    // stage input (forward: the stage's f, dsign = 1; adjoint: the stage's
    // lambda, dsign = -1, since D^T = -D for a symmetric neighbour relation)
    const int32_t *nbr;    // [S][3][2], -1: not in the list (x = 0 there)
    const T *x;
    int64_t ld_x;
    T rate[3];
    T dsign;
};

template <typename T>
__device__ __forceinline__ T drift_term(const Epi<T> &E, int b, int d) {
    const int32_t *nb = E.nbr + 6 * static_cast<int64_t>(d);
    const T *xb = E.x + static_cast<int64_t>(b) * E.ld_x;
    T s = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int up = nb[2 * a], dn = nb[2 * a + 1];
        const T xu = up >= 0 ? xb[up] : T(0);
        const T xd = dn >= 0 ? xb[dn] : T(0);
        s += E.rate[a] * (xu - xd);
    }
    return E.dsign * (T(-0.5) * s);
}

enum EpiMode {
    EPI_STORE = 0,
    EPI_RK1 = 1,     // acc = v;       u = f0 + dt/2 v
    EPI_RK2 = 2,     // acc += 2v;     u = f0 + dt/2 v
    EPI_RK3 = 3,     // acc += 2v;     u = f0 + dt v
    EPI_RK4 = 4,     // f_out = f0 + dt/6 (acc + v)
    EPI_ADJ_FIRST = 5,   // acc = v;   u = cg gbar + cv v
    EPI_ADJ_MID = 6,     // acc += v;  u = cg gbar + cv v
    EPI_ADJ_LAST = 7,    // gbar_out = gbar + acc + v
};

template <typename T>
__device__ __forceinline__ void apply_epi(const Epi<T> &E, int b, int d, int S, T v) {
    const int64_t iw = static_cast<int64_t>(b) * S + d;
    if (E.mode > EPI_STORE && E.nbr) v += drift_term(E, b, d);
    switch (E.mode) {
    case EPI_STORE: E.out[static_cast<int64_t>(b) * E.ld_out + d] = v; break;
    case EPI_RK1: {
        T f = E.f0[static_cast<int64_t>(b) * E.ld_f0 + d];
        E.acc[iw] = v;
        E.u_out[iw] = f + (E.dt * T(0.5)) * v;
    } break;
    case EPI_RK2: {
        T f = E.f0[static_cast<int64_t>(b) * E.ld_f0 + d];
        E.acc[iw] += T(2) * v;
        E.u_out[iw] = f + (E.dt * T(0.5)) * v;
    } break;
    case EPI_RK3: {
        T f = E.f0[static_cast<int64_t>(b) * E.ld_f0 + d];
        E.acc[iw] += T(2) * v;
        E.u_out[iw] = f + E.dt * v;
    } break;
    case EPI_RK4: {
        int64_t i = static_cast<int64_t>(b) * E.ld_f0 + d;
        T f = E.f0[i];
        E.f_out[i] = f + (E.dt / T(6)) * (E.acc[iw] + v);
    } break;
    case EPI_ADJ_FIRST:
        E.acc[iw] = v;
        E.u_out[iw] = E.cg * E.gbar[iw] + E.cv * v;
        break;
    case EPI_ADJ_MID:
        E.acc[iw] += v;
        E.u_out[iw] = E.cg * E.gbar[iw] + E.cv * v;
        break;
    case EPI_ADJ_LAST: E.gbar_out[iw] = E.gbar[iw] + E.acc[iw] + v; break;
    default: break;
    }
}

// ---- block reduction of NV values, fixed order --------------------------
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduces v[0..NV) over the block; thread 0 receives the totals.
template <typename T, int NV>
__device__ __forceinline__ void block_sum(T (&v)[NV]) {
    __shared__ T red[NV][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            T s = red[k][0];
            for (int w = 1; w < nw; ++w) s += red[k][w];
            v[k] = s;
        }
    }
}

// ---- per-entry coefficient evaluation -----------------------------------
template <typename T> struct EntryCoef {
    T ah, bh;   // t + de, t + da  (without |g|^2)
};

template <typename T>
__device__ __forceinline__ EntryCoef<T> entry_coef(const Tables<T> &P, T eps_d, uint32_t kq_d,
                                                   uint32_t pn, const StateRec<T> &sp) {
    const int nu = static_cast<int>(pn & 7u);
    const int q = q_linear(kq_d, sp.kq, P.nq0, P.nq1, P.nq2);
    const int64_t qi = static_cast<int64_t>(q) * P.nm + nu;
    const T w = P.hw[qi];
    const T N = P.nph[qi];
    const T de = eps_d - sp.eps;
    const T xa = de + w, xe = de - w;
    const T da = gauss_exp(xa * xa * P.mc);
    const T dem = gauss_exp(xe * xe * P.mc);
    const T t = N * (da + dem);
    EntryCoef<T> c;
    c.ah = t + dem;
    c.bh = t + da;
    return c;
}

// ---- forward, LDS-tiled --------------------------------------------------
// One workgroup per tile (a run of chunks whose destinations' partners fit an
// LDS window).  The tile's partner states {eps, f} and packed k are staged in
// LDS once; wave w then reduces chunks w, w + n_waves, ... of the tile, each
// with a fixed shuffle tree.  A destination with a single chunk is finished
// by that wave; others leave two partial sums for k_tiled_finish.  All loop
// bounds are wave-uniform scalars (chunk index, entry range), so every wave
// runs its loops in lock step with no divergent exits.
struct TileRec {
    int64_t c0, c1;
    int32_t p_lo, p_hi, lds, pad;
};

template <typename T> struct alignas(2 * sizeof(T)) Pair2 {
    T a, b;
};

template <typename T> struct TiledArgs {
    const uint32_t *__restrict__ pnu;
    const T *__restrict__ g2;
    const StateRec<T> *__restrict__ st;
    const Pair2<T> *__restrict__ hwN;   // {hw, N} of (q, mode) at hwN[q tq + mode tm]
    int64_t tq, tm;                     // (n_modes, 1): the modes of one q adjacent;
                                        // (1, table rows): one block per mode
    const int64_t *__restrict__ chunk_beg;
    const int32_t *__restrict__ chunk_dest;
    const int32_t *__restrict__ dest_chunk;
    const TileRec *__restrict__ tiles;
    int64_t n_chunks;
    int S, nm, nq0, nq1, nq2, lds_states;
    int padq;          // 1: hwN is the box table of QBox, indexed by kqp differences
    int qoff;          // box row of the q = 0 difference
    T mc, K;
    const double *__restrict__ e2tab;   // 2^(j/256), j = 0 .. 255 (FP64 kernels)
    double mc256;                       // 256 mc, the table exponential's scale
    int64_t n_tiles;
    int xcd;                            // tile ranges per XCD (tile_of_block)
    // single-copy pass only
    const int64_t *__restrict__ chunk_end;           // chunk c is [chunk_beg[c], chunk_end[c])
    unsigned long long *__restrict__ jacc;           // [S] partner-side sums, fixed point
    const unsigned long long *__restrict__ nmax_bits;  // max |N| of the packed table (double bits)
    const unsigned long long *__restrict__ gmax_bits;  // max over states of sum |g|^2 (double bits)
    // pair records (k_fwd_pairs): pnu holds partners, g2 is [n_modes][pld]
    int64_t pld;
    // occupations outside [0, 1] (the Bose plans' negated n): max |f| of the
    // call's input (double bits), or null when f lies in [0, 1]
    const unsigned long long *__restrict__ fmax_bits;
};

// ---- fixed point for the partner side of the single-copy pass -------------
// Contributions to I_p (p > d) arrive from many rows; they are rounded to
// integers on a common scale 2^s and summed with integer atomics, which are
// associative, so the sums do not depend on the order of arrival.  With
// |N| <= N_max, f in [0, 1] and the Gaussians <= 1, one entry's share is at
// most |g|^2 (2 N_max + 1), a state's column at most (2 N_max + 1) G_max with
// G_max the largest sum of |g|^2 over one state's channels; s puts that bound
// below 2^61.  With |f| <= m instead, the occupation products of a term,
// at most 1 in [0, 1], are at most (1 + 2m)^2, a factor on the bound.
__device__ __forceinline__ double occ_factor(const unsigned long long *fmax_bits) {
    if (!fmax_bits) return 1.0;
    const double m = __longlong_as_double(static_cast<long long>(*fmax_bits));
    return (1.0 + 2.0 * m) * (1.0 + 2.0 * m);
}

__device__ __forceinline__ double sym_scale(const unsigned long long *nmax_bits,
                                            const unsigned long long *gmax_bits,
                                            const unsigned long long *fmax_bits) {
    const double nmax = __longlong_as_double(static_cast<long long>(*nmax_bits));
    const double gmax = __longlong_as_double(static_cast<long long>(*gmax_bits));
    const double bound = (2.0 * nmax + 1.0) * gmax * occ_factor(fmax_bits);
    if (!(bound > 0.0) || !(bound < 1e300)) return 1.0;
    int e;
    (void)frexp(bound, &e);   // bound < 2^e
    return ldexp(1.0, 61 - e);
}

// y integral-valued with |y| < 2^62, as a two's-complement 64-bit integer
template <typename T> __device__ __forceinline__ unsigned long long to_fixed(T y) {
    const T hi = floor(y * T(2.3283064365386963e-10));   // y / 2^32, rounded down
    const T lo = fma(hi, T(-4294967296.0), y);           // y - hi 2^32, exact, in [0, 2^32)
    const uint32_t l = static_cast<uint32_t>(lo);
    const uint32_t h = static_cast<uint32_t>(static_cast<int32_t>(hi));
    return (static_cast<unsigned long long>(h) << 32) | l;
}

// max of v over the workgroup (blockDim.x <= 1024), stored by thread 0 to *dst
__device__ __forceinline__ void block_max_to(double v, double *dst) {
    __shared__ double s_m[16];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_m[0];
        for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) m = fmax(m, s_m[w]);
        *dst = m;
    }
}

// one workgroup: the max of n per-block values, as double bits
__global__ void k_max_blocks(const double *__restrict__ bm, int n, unsigned long long *out_bits) {
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, bm[i]);
    __shared__ double s_m[16];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) m = fmax(m, s_m[w]);
        m = fmax(m, s_m[0]);
        *out_bits = static_cast<unsigned long long>(__double_as_longlong(m));
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// entries of the exponential table that the FP64 streaming kernels keep in LDS
constexpr int kExpTab = 256;

template <typename T>
__global__ void k_pack_hwN(const T *__restrict__ hw, const T *__restrict__ nph,
                           Pair2<T> *__restrict__ out, int64_t n, double *bmax) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        Pair2<T> v;
        v.a = hw[i];
        v.b = nph[i];
        out[i] = v;
        m = fmax(m, fabs(static_cast<double>(v.b)));
    }
    block_max_to(m, bmax + blockIdx.x);
}

// The padded q table.  States carry k in shifted coordinates c (per axis, 0
// .. span - 1 after a per-axis origin); a pair's difference c_p - c_d lies in
// [-(span - 1), span - 1], so the row x = c_p - c_d + (span - 1) of a
// (2 span - 1)-point axis names it without a modulo, and the three axes give
// the row of one box, qp = (x0 b1 + x1) b2 + x2.  The q it stands for is
// (x - (span - 1)) mod Nq per axis.  The box holds every difference between
// two states, so every row is filled; its size follows the extent of the
// states in k, not the q grid.
struct QBox {
    int n[3];   // q grid
    int b[3];   // box axis lengths, 2 span - 1
    int h[3];   // span - 1
};

// (box rows and q points are below 2^31: 32-bit arithmetic)
__device__ __forceinline__ int box_q(int qp, const QBox &B) {
    int x[3];
    x[2] = qp % B.b[2];
    qp /= B.b[2];
    x[1] = qp % B.b[1];
    x[0] = qp / B.b[1];
    int q = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = x[a] - B.h[a];
        v += v < 0 ? B.n[a] : 0;
        q = q * B.n[a] + v;
    }
    return q;
}

// {hw, N} of the box rows `used` (the rows some entry references), every
// mode: row qp, mode nu at qp nm + nu (mode_major = 0) or nu rows + qp
// (mode_major = 1).  The table holds fewer than 2^31 entries (the plan sizes
// it under 256 MB); rows not listed keep their zeros.
template <typename T>
__global__ void k_pack_hwN_pad(const T *__restrict__ hw, const T *__restrict__ nph,
                               Pair2<T> *__restrict__ out, QBox B, int nm, int rows,
                               const int32_t *__restrict__ used, int n_used, int mode_major, double *bmax) {
    double m = 0.0;
    const int n = n_used * nm;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int nu = i % nm;
        const int qp = used[i / nm];
        const int64_t q = box_q(qp, B);
        Pair2<T> v;
        v.a = hw[q * nm + nu];
        v.b = nph[q * nm + nu];
        out[mode_major ? nu * rows + qp : qp * nm + nu] = v;
        m = fmax(m, fabs(static_cast<double>(v.b)));
    }
    block_max_to(m, bmax + blockIdx.x);
}

// exp of the Gaussian exponent x2 * (-1/(2 s^2)) for the streaming kernels
template <typename T>
__device__ __forceinline__ T stream_gauss(const TiledArgs<T> &A, T x2, const double *tab) {
    if constexpr (sizeof(T) == 8) return gauss_exp2_tab(x2 * A.mc256, tab);
    else return __builtin_amdgcn_exp2f(x2 * A.mc);
}

// Chunk reduction with a three-stage pipeline (stream loads two batches
// ahead, partner/table gathers one batch ahead of the evaluation).  The entry
// arrays are padded past their end, so stream loads are unconditional.  Only
// a chunk's last batch can hold lanes past its end (they read the padding or
// the next chunk); that batch is gathered with a mask that makes those lanes
// contribute zero, the others without one (the choice is uniform per wave).
// Offsets are 32-bit and relative to the chunk start.
template <typename T, bool LDS, bool PADQ, int U>
__device__ __forceinline__ void fwd_chunk2(const TiledArgs<T> &A, const T *__restrict__ fb,
                                           const Pair2<T> *s_ef, const uint32_t *s_kq, int p_lo,
                                           const double *s_tab, int64_t c, int b,
                                           T *__restrict__ part, const Epi<T> &E) {
    const int lane = threadIdx.x & 63;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_beg[c + 1] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const StateRec<T> sd = A.st[d];
    const uint32_t kd = PADQ ? sd.kqp : sd.kq;
    T acc_a = T(0), acc_b = T(0);
    uint32_t pn1[U];
    T gs1[U];
    T g0[U], de0[U], fp0[U];
    Pair2<T> wn0[U];
    auto load_stream = [&](int r0, uint32_t (&pn)[U], T (&gs)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pn[u] = pb[r0 + u * 64 + lane];
            gs[u] = gb[r0 + u * 64 + lane];
        }
    };
    auto gather = [&](auto masked, const uint32_t (&pn)[U], const T (&gs)[U], int r0,
                      T (&go)[U], T (&deo)[U], T (&fpo)[U], Pair2<T> (&wno)[U]) {
        constexpr bool M = decltype(masked)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool v = !M || r0 + u * 64 + lane < len;
            const int p = static_cast<int>(pn[u] >> 3);
            T ep, fp;
            uint32_t kp;
            if (LDS) {
                // a masked lane reads slot 0 (inside the allocation) and then
                // replaces what it read: partner = destination, so its table
                // index is the q = 0 entry and its operands are finite,
                // whatever the slot holds
                const int pl = v ? p - p_lo : 0;
                const Pair2<T> ef = s_ef[pl];
                ep = v ? ef.a : sd.eps;
                fp = v ? ef.b : T(0);
                kp = v ? s_kq[pl] : kd;
            } else {
                const StateRec<T> sp = A.st[p];
                ep = sp.eps;
                kp = PADQ ? sp.kqp : sp.kq;
                fp = fb[p];
            }
            const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff
                               : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.tq + static_cast<int64_t>(pn[u] & 7u) * A.tm];
            if constexpr (M) {
                // a table entry without channels may hold a non-finite N, so both
                // fields are replaced (using both keeps the {hw, N} pair one
                // 16-byte load)
                wno[u].a = v ? w.a : T(0);
                wno[u].b = v ? w.b : T(0);
                go[u] = v ? gs[u] : T(0);
            } else {
                wno[u] = w;
                go[u] = gs[u];
            }
            deo[u] = sd.eps - ep;
            fpo[u] = fp;
        }
    };
    using Masked = std::integral_constant<bool, true>;
    using Full = std::integral_constant<bool, false>;
    {
        uint32_t pn0[U];
        T gs0[U];
        load_stream(0, pn0, gs0);
        load_stream(64 * U, pn1, gs1);
        if (64 * U <= len) gather(Full{}, pn0, gs0, 0, g0, de0, fp0, wn0);
        else gather(Masked{}, pn0, gs0, 0, g0, de0, fp0, wn0);
    }
    for (int r = 0; r < len; r += 64 * U) {
        T g1[U], de1[U], fp1[U];
        Pair2<T> wn1[U];
        if (r + 128 * U <= len) gather(Full{}, pn1, gs1, r + 64 * U, g1, de1, fp1, wn1);
        else gather(Masked{}, pn1, gs1, r + 64 * U, g1, de1, fp1, wn1);
        load_stream(r + 128 * U, pn1, gs1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T xa = de0[u] + wn0[u].a, xe = de0[u] - wn0[u].a;
            const T da = stream_gauss(A, xa * xa, s_tab);
            const T dem = stream_gauss(A, xe * xe, s_tab);
            const T t = wn0[u].b * (da + dem);
            acc_a += g0[u] * (t + dem) * (T(1) - fp0[u]);
            acc_b += g0[u] * (t + da) * fp0[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            g0[u] = g1[u];
            de0[u] = de1[u];
            fp0[u] = fp1[u];
            wn0[u] = wn1[u];
        }
    }
    acc_a = wave_sum(acc_a);
    acc_b = wave_sum(acc_b);
    if (lane == 0) {
        if (A.dest_chunk[d + 1] - A.dest_chunk[d] == 1) {
            const T fd = fb[d];
            apply_epi(E, b, d, A.S, A.K * ((T(1) - fd) * acc_b - fd * acc_a));
        } else {
            T *pp = part + (static_cast<int64_t>(b) * A.n_chunks + c) * 2;
            pp[0] = acc_a;
            pp[1] = acc_b;
        }
    }
}

template <typename T, int U, int MAXT, bool PADQ>
__global__ __launch_bounds__(MAXT) void k_fwd_tiled(TiledArgs<T> A, const T *__restrict__ f,
                                                    int64_t ldf, T *__restrict__ part, Epi<T> E) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    const int b = blockIdx.y;
    const T *fb = f + static_cast<int64_t>(b) * ldf;
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(smem);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_ef + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    if (t.lds) {
        const int n = t.p_hi - t.p_lo + 1;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const StateRec<T> sr = A.st[t.p_lo + i];
            Pair2<T> ef;
            ef.a = sr.eps;
            ef.b = fb[t.p_lo + i];
            s_ef[i] = ef;
            s_kq[i] = PADQ ? sr.kqp : sr.kq;
        }
    }
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (t.lds)
            fwd_chunk2<T, true, PADQ, U>(A, fb, s_ef, s_kq, t.p_lo, s_tab, c, b, part, E);
        else
            fwd_chunk2<T, false, PADQ, U>(A, fb, s_ef, s_kq, t.p_lo, s_tab, c, b, part, E);
    }
}

// ---- forward, single copy ---------------------------------------------------
// Each channel is evaluated once, from the row of its smaller state d (the
// entries p > d of that row, the upper part of the destination-sorted layout).
// With Y = (1 - f_d) b f_p - f_d a (1 - f_p) (a, b as in the duplicated pass),
// I_d receives K Y and I_p receives -K Y: the row side is reduced in registers
// as in fwd_chunk2, the partner side is added to a fixed-point accumulator per
// partner (LDS for an LDS tile, then flushed to the global one).

// max over states of the sum of |g|^2 over the state's entries, one wave per state
template <typename T>
__global__ void k_row_gmax(const T *__restrict__ g2, const int64_t *__restrict__ chunk_beg,
                           const int32_t *__restrict__ dest_chunk, int S,
                           unsigned long long *gmax_bits) {
    const int d = static_cast<int>((blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    double sum = 0.0;
    if (d < S) {
        const int64_t b = chunk_beg[dest_chunk[d]], e = chunk_beg[dest_chunk[d + 1]];
        for (int64_t x = b + lane; x < e; x += 64) sum += fabs(static_cast<double>(g2[x]));
    }
    sum = wave_sum(sum);
    if (lane == 0 && d < S)
        atomicMax(gmax_bits, static_cast<unsigned long long>(__double_as_longlong(sum)));
}

template <typename T, bool LDS, bool PADQ, int U>
__device__ __forceinline__ void sym_chunk(const TiledArgs<T> &A, const T *__restrict__ fb,
                                          const Pair2<T> *s_ef, const uint32_t *s_kq, int p_lo,
                                          const double *s_tab, unsigned long long *s_j, T scale,
                                          int64_t c, T *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_end[c] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const StateRec<T> sd = A.st[d];
    const uint32_t kd = PADQ ? sd.kqp : sd.kq;
    const T fd = fb[d];
    const T cfd = T(1) - fd;
    T acc_a = T(0), acc_b = T(0);
    uint32_t pn1[U];
    T gs1[U];
    T g0[U], de0[U], fp0[U];
    int pl0[U];
    Pair2<T> wn0[U];
    auto load_stream = [&](int r0, uint32_t (&pn)[U], T (&gs)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pn[u] = pb[r0 + u * 64 + lane];
            gs[u] = gb[r0 + u * 64 + lane];
        }
    };
    auto gather = [&](auto masked, const uint32_t (&pn)[U], const T (&gs)[U], int r0, T (&go)[U],
                      T (&deo)[U], T (&fpo)[U], Pair2<T> (&wno)[U], int (&plo)[U]) {
        constexpr bool M = decltype(masked)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool v = !M || r0 + u * 64 + lane < len;
            const int p = static_cast<int>(pn[u] >> 3);
            T ep, fp;
            uint32_t kp;
            if (LDS) {
                // a masked lane: partner = destination (finite operands, the
                // q = 0 table entry); it adds zero to slot 0 of the window
                const int pl = v ? p - p_lo : 0;
                const Pair2<T> ef = s_ef[pl];
                ep = v ? ef.a : sd.eps;
                fp = v ? ef.b : T(0);
                kp = v ? s_kq[pl] : kd;
                plo[u] = pl;
            } else {
                const StateRec<T> sp = A.st[p];
                ep = sp.eps;
                kp = PADQ ? sp.kqp : sp.kq;
                fp = fb[p];
                plo[u] = p;
            }
            const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff
                               : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.tq + static_cast<int64_t>(pn[u] & 7u) * A.tm];
            if constexpr (M) {
                // a table entry without channels may hold a non-finite N; the
                // masked lanes then add zero to partner slot 0 (or state p)
                wno[u].a = v ? w.a : T(0);
                wno[u].b = v ? w.b : T(0);
                go[u] = v ? gs[u] : T(0);
            } else {
                wno[u] = w;
                go[u] = gs[u];
            }
            deo[u] = sd.eps - ep;
            fpo[u] = fp;
        }
    };
    using Masked = std::integral_constant<bool, true>;
    using Full = std::integral_constant<bool, false>;
    {
        uint32_t pn0[U];
        T gs0[U];
        load_stream(0, pn0, gs0);
        load_stream(64 * U, pn1, gs1);
        if (64 * U <= len) gather(Full{}, pn0, gs0, 0, g0, de0, fp0, wn0, pl0);
        else gather(Masked{}, pn0, gs0, 0, g0, de0, fp0, wn0, pl0);
    }
    for (int r = 0; r < len; r += 64 * U) {
        T g1[U], de1[U], fp1[U];
        int pl1[U];
        Pair2<T> wn1[U];
        if (r + 128 * U <= len) gather(Full{}, pn1, gs1, r + 64 * U, g1, de1, fp1, wn1, pl1);
        else gather(Masked{}, pn1, gs1, r + 64 * U, g1, de1, fp1, wn1, pl1);
        load_stream(r + 128 * U, pn1, gs1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T xa = de0[u] + wn0[u].a, xe = de0[u] - wn0[u].a;
            const T da = stream_gauss(A, xa * xa, s_tab);
            const T dem = stream_gauss(A, xe * xe, s_tab);
            const T t = wn0[u].b * (da + dem);
            const T ta = g0[u] * (t + dem) * (T(1) - fp0[u]);
            const T tb = g0[u] * (t + da) * fp0[u];
            acc_a += ta;
            acc_b += tb;
            // partner side: -Y = f_d ta - (1 - f_d) tb, on the fixed-point scale
            const unsigned long long v = to_fixed(__builtin_rint(fma(fd, ta, -cfd * tb) * scale));
            if (LDS) atomicAdd(s_j + pl0[u], v);
            else atomicAdd(A.jacc + pl0[u], v);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            g0[u] = g1[u];
            de0[u] = de1[u];
            fp0[u] = fp1[u];
            wn0[u] = wn1[u];
            pl0[u] = pl1[u];
        }
    }
    acc_a = wave_sum(acc_a);
    acc_b = wave_sum(acc_b);
    if (lane == 0) {
        part[2 * c] = acc_a;
        part[2 * c + 1] = acc_b;
    }
}

template <typename T, int U, bool PADQ>
__global__ __launch_bounds__(1024) void k_fwd_sym(TiledArgs<T> A, const T *__restrict__ f,
                                                  T *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    // LDS: partner-side sums (8 B), {eps, f}, packed k, exponential table
    unsigned long long *s_j = reinterpret_cast<unsigned long long *>(smem);
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(s_j + A.lds_states);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_ef + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    const int n = t.lds ? t.p_hi - t.p_lo + 1 : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const StateRec<T> sr = A.st[t.p_lo + i];
        Pair2<T> ef;
        ef.a = sr.eps;
        ef.b = f[t.p_lo + i];
        s_ef[i] = ef;
        s_kq[i] = PADQ ? sr.kqp : sr.kq;
        s_j[i] = 0ull;
    }
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    const T scale = static_cast<T>(sym_scale(A.nmax_bits, A.gmax_bits, A.fmax_bits));
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (t.lds)
            sym_chunk<T, true, PADQ, U>(A, f, s_ef, s_kq, t.p_lo, s_tab, s_j, scale, c, part);
        else
            sym_chunk<T, false, PADQ, U>(A, f, s_ef, s_kq, t.p_lo, s_tab, s_j, scale, c, part);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long v = s_j[i];
        if (v) atomicAdd(A.jacc + t.p_lo + i, v);
    }
}

// ---- forward, single copy over pair records ----------------------------------
// The same pass over pair records: a lane takes one pair (d, p), p > d, with
// all its modes.  The partner's {eps, f} and k are gathered once per pair, the
// {hw, N} of the modes of q = k_p - k_d are adjacent in the table, and the
// partner side of the pair (summed over its modes in a fixed order) is one
// fixed-point atomic.  A slot without a channel has |g|^2 = 0; its N is
// replaced by 0 so that a non-finite table entry of that mode (N at an
// acoustic q = 0) cannot turn the zero into a NaN.

// v where keep holds, else +0, by masking the bits: unlike a select of a
// loaded value, this cannot be turned into a load under a branch (which would
// make the wave wait for every load in flight, the next batch's stream too)
__device__ __forceinline__ double keep_or_zero(double v, bool keep) {
    const unsigned long long m = keep ? ~0ull : 0ull;
    return __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(v)) & m));
}
__device__ __forceinline__ float keep_or_zero(float v, bool keep) {
    const int m = keep ? -1 : 0;
    return __int_as_float(__float_as_int(v) & m);
}

// FP64 Gaussian of the pair pass: the table exponential (TAB) or the
// degree-12 polynomial one (no LDS reads); FP32: the hardware exponential
template <typename T, bool TAB>
__device__ __forceinline__ T pair_gauss(const TiledArgs<T> &A, T x2, const double *tab) {
    if constexpr (sizeof(T) == 8 && TAB) return gauss_exp2_tab(x2 * A.mc256, tab);
    else if constexpr (sizeof(T) == 8) return gauss_exp2(x2 * A.mc);
    else return __builtin_amdgcn_exp2f(x2 * A.mc);
}

// The pair's sums over its modes of a = |g|^2 (t + G(x - hw)) and
// b = |g|^2 (t + G(x + hw)), t = N (G(x + hw) + G(x - hw)), x = de; the
// occupation factors are the pair's.  Slots past nm, and every slot of a
// masked lane (v false), count as empty.
template <typename T, int NM, bool TAB>
__device__ __forceinline__ void pair_mode_sums(const TiledArgs<T> &A, T de, const Pair2<T> (&w)[NM],
                                               const T (&g)[NM], bool v, const double *s_tab, T &sa, T &sb) {
    const int nm = A.nm;
    sa = T(0);
    sb = T(0);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const T gm = v && m < nm ? g[m] : T(0);
        const T N = keep_or_zero(w[m].b, gm != T(0));
        const T xa = de + w[m].a, xe = de - w[m].a;
        const T da = pair_gauss<T, TAB>(A, xa * xa, s_tab);
        const T dem = pair_gauss<T, TAB>(A, xe * xe, s_tab);
        const T t = N * (da + dem);
        sa = fma(gm, t + dem, sa);
        sb = fma(gm, t + da, sb);
    }
}

template <typename T, bool LDS, bool PADQ, int NM, bool TAB>
__device__ __forceinline__ void pair_chunk(const TiledArgs<T> &A, const T *__restrict__ fb,
                                           const Pair2<T> *s_ef, const uint32_t *s_kq, int p_lo,
                                           const double *s_tab, unsigned long long *s_j, T scale,
                                           int64_t c, T *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int nm = A.nm;   // <= NM
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_end[c] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const StateRec<T> sd = A.st[d];
    const uint32_t kd = PADQ ? sd.kqp : sd.kq;
    const T fd = fb[d];
    const T cfd = T(1) - fd;
    T acc_a = T(0), acc_b = T(0);
    // the stream (partner and |g|^2 slots) runs one batch ahead of the
    // gathers and the evaluation.  The arrays are padded past their end, so
    // no stream load needs a bound.
    // Mode slots past nm (NM rounds nm up) re-read the last mode and count
    // as empty, so the mode loops carry no branch.  The stream values are
    // kept as loaded and masked where they are used: a mask applied at the
    // end of the batch would make the wave wait there for the loads it has
    // just issued.
    // Two register sets alternate (the loop is unrolled twice), so the
    // values loaded for the next batch need no copy at the end of a batch,
    // which would wait for them.
    uint32_t pn0 = pb[lane], pn1 = 0;
    T g0[NM], g1[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) g0[m] = gb[min(m, nm - 1) * A.pld + lane];
    auto batch = [&](int r, const uint32_t pn, const T (&g)[NM], uint32_t &pn_next, T (&g_next)[NM]) {
        const bool v = r + lane < len;
        const int p = static_cast<int>(pn);
        T ep, fp;
        uint32_t kp;
        int pl;
        // A masked lane takes a valid partner (the window's first state, or
        // the destination) and |g|^2 = 0, so its operands are finite and it
        // adds nothing.  The partner's values are loaded unconditionally: a
        // choice between a loaded value and another one is compiled into a
        // branch around the load, which waits for every load in flight.
        if (LDS) {
            pl = v ? p - p_lo : 0;
            const Pair2<T> ef = s_ef[pl];
            ep = ef.a;
            fp = ef.b;
            kp = s_kq[pl];
        } else {
            pl = v ? p : d;
            const StateRec<T> sp = A.st[pl];
            ep = sp.eps;
            kp = PADQ ? sp.kqp : sp.kq;
            fp = fb[pl];
        }
        const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
        const Pair2<T> *__restrict__ wq = A.hwN + static_cast<int64_t>(q) * A.tq;
        Pair2<T> w[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) w[m] = wq[min(m, nm - 1) * A.tm];
        // the next batch's stream loads are issued after this batch's table
        // gathers: loads complete in issue order for the wait counter, so
        // waiting for the gathers does not wait for the stream.  The
        // scheduling barriers keep that order and keep the compiler from
        // sinking any of these loads towards their first use, which would
        // serialise the gathers.
        __builtin_amdgcn_sched_barrier(0);
        pn_next = pb[r + 64 + lane];
#pragma unroll
        for (int m = 0; m < NM; ++m) g_next[m] = gb[min(m, nm - 1) * A.pld + r + 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
        const T ofp = T(1) - fp;
        T sa, sb;
        pair_mode_sums<T, NM, TAB>(A, sd.eps - ep, w, g, v, s_tab, sa, sb);
        const T ta = sa * ofp, tb = sb * fp;
        acc_a += ta;
        acc_b += tb;
        // partner side: -Y = f_d ta - (1 - f_d) tb
        const T y = fma(fd, ta, -cfd * tb);
        if (v) {
            const unsigned long long fx = to_fixed(__builtin_rint(y * scale));
            if (LDS) atomicAdd(s_j + pl, fx);
            else atomicAdd(A.jacc + pl, fx);
        }
    };
    for (int r = 0; r < len; r += 128) {
        batch(r, pn0, g0, pn1, g1);
        if (r + 64 >= len) break;
        batch(r + 64, pn1, g1, pn0, g0);
    }
    acc_a = wave_sum(acc_a);
    acc_b = wave_sum(acc_b);
    if (lane == 0) {
        part[2 * c] = acc_a;
        part[2 * c + 1] = acc_b;
    }
}

// The same pass over a q-ordered tile.  Its records are sorted by the table
// row of q = k_p - k_d (then destination, partner), so the lanes of a batch
// read a few rows of the {hw, N} table instead of one each.  A record's word
// holds the window offsets of its partner (high 16 bits) and destination (low
// 16 bits); the window stages both.  The destination's side of the pair, -y,
// goes to the same fixed-point accumulator as the partner's, +y, so the
// chunk's row partials are zero.
template <typename T, bool PADQ, int NM, bool TAB>
__device__ __forceinline__ void pair_chunk_q(const TiledArgs<T> &A, const Pair2<T> *s_ef, const uint32_t *s_kq,
                                             const double *s_tab, unsigned long long *s_j, T scale, int64_t c,
                                             T *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int nm = A.nm;
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_end[c] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    // stream one batch ahead, two register sets (see pair_chunk)
    uint32_t pn0 = pb[lane], pn1 = 0;
    T g0[NM], g1[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) g0[m] = gb[min(m, nm - 1) * A.pld + lane];
    auto batch = [&](int r, const uint32_t pn, const T (&g)[NM], uint32_t &pn_next, T (&g_next)[NM]) {
        const bool v = r + lane < len;
        // a masked lane takes window slot 0 as both states (q = 0) and adds nothing
        const int wd = v ? static_cast<int>(pn & 0xffffu) : 0;
        const int wp = v ? static_cast<int>(pn >> 16) : 0;
        const Pair2<T> efd = s_ef[wd], efp = s_ef[wp];
        const uint32_t kd = s_kq[wd], kp = s_kq[wp];
        const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
        const Pair2<T> *__restrict__ wq = A.hwN + static_cast<int64_t>(q) * A.tq;
        Pair2<T> w[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) w[m] = wq[min(m, nm - 1) * A.tm];
        __builtin_amdgcn_sched_barrier(0);
        pn_next = pb[r + 64 + lane];
#pragma unroll
        for (int m = 0; m < NM; ++m) g_next[m] = gb[min(m, nm - 1) * A.pld + r + 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
        T sa, sb;
        pair_mode_sums<T, NM, TAB>(A, efd.a - efp.a, w, g, v, s_tab, sa, sb);
        const T fd = efd.b, fp = efp.b;
        const T ta = sa * (T(1) - fp), tb = sb * fp;
        const T y = fma(fd, ta, -(T(1) - fd) * tb);
        if (v) {
            const unsigned long long fx = to_fixed(__builtin_rint(y * scale));
            atomicAdd(s_j + wp, fx);
            atomicAdd(s_j + wd, 0ull - fx);
        }
    };
    for (int r = 0; r < len; r += 128) {
        batch(r, pn0, g0, pn1, g1);
        if (r + 64 >= len) break;
        batch(r + 64, pn1, g1, pn0, g0);
    }
    if (lane == 0) {
        part[2 * c] = T(0);
        part[2 * c + 1] = T(0);
    }
}

template <typename T, bool PADQ, int NM, bool TAB>
__global__ __launch_bounds__(1024) void k_fwd_pairs(TiledArgs<T> A, const T *__restrict__ f,
                                                    T *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    unsigned long long *s_j = reinterpret_cast<unsigned long long *>(smem);
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(s_j + A.lds_states);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_ef + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    const int n = t.lds ? t.p_hi - t.p_lo + 1 : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const StateRec<T> sr = A.st[t.p_lo + i];
        Pair2<T> ef;
        ef.a = sr.eps;
        ef.b = f[t.p_lo + i];
        s_ef[i] = ef;
        s_kq[i] = PADQ ? sr.kqp : sr.kq;
        s_j[i] = 0ull;
    }
    if constexpr (sizeof(T) == 8 && TAB)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    const T scale = static_cast<T>(sym_scale(A.nmax_bits, A.gmax_bits, A.fmax_bits));
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (t.lds == 2)
            pair_chunk_q<T, PADQ, NM, TAB>(A, s_ef, s_kq, s_tab, s_j, scale, c, part);
        else if (t.lds)
            pair_chunk<T, true, PADQ, NM, TAB>(A, f, s_ef, s_kq, t.p_lo, s_tab, s_j, scale, c, part);
        else
            pair_chunk<T, false, PADQ, NM, TAB>(A, f, s_ef, s_kq, t.p_lo, s_tab, s_j, scale, c, part);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long v = s_j[i];
        if (v) atomicAdd(A.jacc + t.p_lo + i, v);
    }
}

// ---- reverse, single copy over pair records ----------------------------------
// Each channel (d, p, nu), d < p, of a pair record enters L = sum lam I through
// (lam_d - lam_p) X with X = K |g|^2 [(1 - f_d) bh f_p - f_d ah (1 - f_p)]
// (ah = t + G(x - hw), bh = t + G(x + hw), t = N (G(x + hw) + G(x - hw)),
// x = e_d - e_p).  Hence, with dl = lam_d - lam_p:
//   dL/df_d  += -K dl |g|^2 (ah (1 - f_p) + bh f_p)          (row side, registers)
//   dL/df_p  +=  K dl |g|^2 (bh (1 - f_d) + ah f_d)          (partner side, fixed point)
//   dL/d|g|^2 =  K dl ((1 - f_d) bh f_p - f_d ah (1 - f_p))   (one writer per channel;
//                chan0 holds the record's first channel when its slots are the
//                consecutive channels of the caller's list, else -1)
// The partner side of a pair is summed over its modes and added with one
// integer atomic, on the scale of vjp_scale.  Each channel is read once.
__device__ __forceinline__ double vjp_scale(const unsigned long long *nmax_bits,
                                            const unsigned long long *gmax_bits,
                                            const unsigned long long *lmax_bits,
                                            const unsigned long long *fmax_bits) {
    // |dl| <= 2 max |lam|: a state's column is at most 2 max|lam| (2 N_max + 1) G_max
    // (times occ_factor when f leaves [0, 1])
    const double nmax = __longlong_as_double(static_cast<long long>(*nmax_bits));
    const double gmax = __longlong_as_double(static_cast<long long>(*gmax_bits));
    const double lmax = __longlong_as_double(static_cast<long long>(*lmax_bits));
    const double bound = 2.0 * lmax * (2.0 * nmax + 1.0) * gmax * occ_factor(fmax_bits);
    if (!(bound > 0.0) || !(bound < 1e300)) return 1.0;
    int e;
    (void)frexp(bound, &e);
    return ldexp(1.0, 61 - e);
}

// threads per workgroup of the pair reverse pass: 16 waves, as the forward
// (a lane holds at most 128 registers; the pass needs about 100 with the
// modes summed per pair)
constexpr int kVjpPairThreads = 1024;

// chunks of a q-ordered pair tile: one for each wave of a 1024-thread workgroup
constexpr int kPairChunksPerTile = 16;

// The pair's sums over its modes of |g|^2 ah and |g|^2 bh, and per mode
// dL/d|g|^2 = kb bh - ka ah (gv); empty slots as in pair_mode_sums.
template <typename T, int NM, bool TAB>
__device__ __forceinline__ void vjp_mode_sums(const TiledArgs<T> &A, T x, T kb, T ka, const Pair2<T> (&w)[NM],
                                              const T (&g)[NM], bool v, const double *s_tab, T &sa, T &sb,
                                              double (&gv)[NM]) {
    const int nm = A.nm;
    sa = T(0);
    sb = T(0);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const Pair2<T> wm = w[m];
        const T gm = v && m < nm ? g[m] : T(0);
        const T N = keep_or_zero(wm.b, gm != T(0));
        const T xa = x + wm.a, xe = x - wm.a;
        const T da = pair_gauss<T, TAB>(A, xa * xa, s_tab);
        const T dem = pair_gauss<T, TAB>(A, xe * xe, s_tab);
        const T t = N * (da + dem);
        const T ah = t + dem, bh = t + da;
        sa = fma(gm, ah, sa);
        sb = fma(gm, bh, sb);
        gv[m] = static_cast<double>(fma(kb, bh, -ka * ah));
    }
}

// Writes (gg2_mode 1) or adds (2) the record's dL/d|g|^2 to its channels:
// c0 >= 0 when they are the consecutive channels c0, c0 + 1, ..; else each
// slot's channel is cb[m pld] (-1: no channel)
template <int NM>
__device__ __forceinline__ void write_gg2(double *__restrict__ gg2, int gg2_mode, int32_t c0,
                                          const int32_t *__restrict__ cb, int64_t pld, int nm,
                                          const double (&gv)[NM]) {
    // The overwriting stores do not share instructions with the accumulating
    // ones: a store of either a loaded value or another would wait for every
    // load in flight, the next batch's stream too.
    if (c0 >= 0 && NM == nm && (NM & 1) == 0 && (c0 & 1) == 0) {
        // 16-byte aligned: the lane writes them as whole pairs
        double2 *dst = reinterpret_cast<double2 *>(gg2 + c0);
        if (gg2_mode == 2) {
#pragma unroll
            for (int k = 0; k < NM / 2; ++k) {
                double2 o = dst[k];
                o.x += gv[2 * k];
                o.y += gv[2 * k + 1];
                dst[k] = o;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NM / 2; ++k) dst[k] = make_double2(gv[2 * k], gv[2 * k + 1]);
        }
    } else if (c0 >= 0 && gg2_mode != 2) {
#pragma unroll
        for (int m = 0; m < NM; ++m)
            if (m < nm) gg2[c0 + m] = gv[m];
    } else {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if (m >= nm) break;
            const int32_t ch = c0 >= 0 ? c0 + m : cb[m * pld];
            if (ch >= 0) gg2[ch] = gg2_mode == 2 ? gg2[ch] + gv[m] : gv[m];
        }
    }
}

template <typename T, bool LDS, bool PADQ, int NM, bool TAB>
__device__ __forceinline__ void vjp_pair_chunk(const TiledArgs<T> &A, const T *__restrict__ fb,
                                               const T *__restrict__ lb, const Pair2<T> *s_ef,
                                               const uint32_t *s_kq, const T *s_l, int p_lo,
                                               const double *s_tab, unsigned long long *s_j, T scale,
                                               int64_t c, T *__restrict__ part, bool want_f,
                                               const int32_t *__restrict__ chan,
                                               const int32_t *__restrict__ chan0, double *__restrict__ gg2,
                                               int gg2_mode) {
    const int lane = threadIdx.x & 63;
    const int nm = A.nm;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_end[c] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const int32_t *__restrict__ cb = chan + beg;
    const int32_t *__restrict__ cb0 = chan0 + beg;
    const StateRec<T> sd = A.st[d];
    const uint32_t kd = PADQ ? sd.kqp : sd.kq;
    const T fd = fb[d];
    const T cfd = T(1) - fd;
    const T ld = lb[d];
    T acc = T(0);
    uint32_t pn = pb[lane];
    for (int r = 0; r < len; r += 64) {
        const bool v = r + lane < len;
        const uint32_t pn_next = pb[r + 64 + lane];
        // mode slots past nm re-read the last mode and count as empty; the
        // values are masked where they are used (see pair_chunk)
        T g[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) g[m] = gb[min(m, nm - 1) * A.pld + r + lane];
        const int32_t c0 = gg2_mode ? cb0[r + lane] : -1;
        const int p = static_cast<int>(pn);
        T ep, fp, lp;
        uint32_t kp;
        int pl;
        // a masked lane takes a valid partner and |g|^2 = 0 (see pair_chunk)
        if (LDS) {
            pl = v ? p - p_lo : 0;
            const Pair2<T> ef = s_ef[pl];
            ep = ef.a;
            fp = ef.b;
            lp = s_l[pl];
            kp = s_kq[pl];
        } else {
            pl = v ? p : d;
            const StateRec<T> sp = A.st[pl];
            ep = sp.eps;
            kp = PADQ ? sp.kqp : sp.kq;
            fp = fb[pl];
            lp = lb[pl];
        }
        const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
        const Pair2<T> *__restrict__ wq = A.hwN + static_cast<int64_t>(q) * A.tq;
        Pair2<T> w[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) w[m] = wq[min(m, nm - 1) * A.tm];
        // all table gathers are in flight before the first is waited for
        __builtin_amdgcn_sched_barrier(0);
        const T x = sd.eps - ep;
        const T ofp = T(1) - fp;
        const T dl = ld - lp;
        // per mode dL/d|g|^2 = kb bh - ka ah; the pair's sums of |g|^2 ah and
        // |g|^2 bh serve both occupation sides
        const T kb = A.K * dl * cfd * fp, ka = A.K * dl * fd * ofp;
        T sa, sb;
        double gv[NM];
        vjp_mode_sums<T, NM, TAB>(A, x, kb, ka, w, g, v, s_tab, sa, sb, gv);
        acc += dl * fma(sa, ofp, sb * fp);
        const T y = dl * fma(sb, cfd, sa * fd);
        // consecutive records of a row write consecutive memory when their
        // channels are consecutive in the caller's order
        if (gg2_mode && v) write_gg2<NM>(gg2, gg2_mode, c0, cb + r + lane, A.pld, nm, gv);
        if (want_f && v) {
            const unsigned long long fx = to_fixed(__builtin_rint(y * scale));
            if (LDS) atomicAdd(s_j + pl, fx);
            else atomicAdd(A.jacc + pl, fx);
        }
        pn = pn_next;
    }
    if (!want_f) return;
    acc = wave_sum(acc);
    if (lane == 0) part[c] = acc;
}

// The reverse pass over a q-ordered tile (see pair_chunk_q): both sides of a
// pair go to the fixed-point accumulator, -K dl (ah (1 - f_p) + bh f_p) |g|^2
// summed over modes to the destination and the partner's side as in
// vjp_pair_chunk; the chunk's row partial is zero.
template <typename T, bool PADQ, int NM, bool TAB>
__device__ __forceinline__ void vjp_pair_chunk_q(const TiledArgs<T> &A, const Pair2<T> *s_ef,
                                                 const uint32_t *s_kq, const T *s_l, const double *s_tab,
                                                 unsigned long long *s_j, T scale, int64_t c, T *__restrict__ part,
                                                 bool want_f, const int32_t *__restrict__ chan,
                                                 const int32_t *__restrict__ chan0, double *__restrict__ gg2,
                                                 int gg2_mode) {
    const int lane = threadIdx.x & 63;
    const int nm = A.nm;
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_end[c] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const int32_t *__restrict__ cb = chan + beg;
    const int32_t *__restrict__ cb0 = chan0 + beg;
    // stream one batch ahead, two register sets (see pair_chunk)
    uint32_t pn0 = pb[lane], pn1 = 0;
    int32_t h0 = gg2_mode ? cb0[lane] : -1, h1 = -1;
    T g0[NM], g1[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) g0[m] = gb[min(m, nm - 1) * A.pld + lane];
    auto batch = [&](int r, const uint32_t pn, const T (&g)[NM], const int32_t c0, uint32_t &pn_next,
                     T (&g_next)[NM], int32_t &c0_next) {
        const bool v = r + lane < len;
        // a masked lane takes window slot 0 as both states and adds nothing
        const int wd = v ? static_cast<int>(pn & 0xffffu) : 0;
        const int wp = v ? static_cast<int>(pn >> 16) : 0;
        const Pair2<T> efd = s_ef[wd], efp = s_ef[wp];
        const T ld = s_l[wd], lp = s_l[wp];
        const uint32_t kd = s_kq[wd], kp = s_kq[wp];
        const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
        const Pair2<T> *__restrict__ wq = A.hwN + static_cast<int64_t>(q) * A.tq;
        Pair2<T> w[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) w[m] = wq[min(m, nm - 1) * A.tm];
        __builtin_amdgcn_sched_barrier(0);
        pn_next = pb[r + 64 + lane];
#pragma unroll
        for (int m = 0; m < NM; ++m) g_next[m] = gb[min(m, nm - 1) * A.pld + r + 64 + lane];
        c0_next = gg2_mode ? cb0[r + 64 + lane] : -1;
        __builtin_amdgcn_sched_barrier(0);
        const T fd = efd.b, cfd = T(1) - fd, fp = efp.b, ofp = T(1) - fp;
        const T dl = ld - lp;
        const T kb = A.K * dl * cfd * fp, ka = A.K * dl * fd * ofp;
        T sa, sb;
        double gv[NM];
        vjp_mode_sums<T, NM, TAB>(A, efd.a - efp.a, kb, ka, w, g, v, s_tab, sa, sb, gv);
        if (gg2_mode && v) write_gg2<NM>(gg2, gg2_mode, c0, cb + r + lane, A.pld, nm, gv);
        if (want_f && v) {
            const T rd = dl * fma(sa, ofp, sb * fp);
            const T y = dl * fma(sb, cfd, sa * fd);
            atomicAdd(s_j + wp, to_fixed(__builtin_rint(y * scale)));
            atomicAdd(s_j + wd, to_fixed(__builtin_rint(-rd * scale)));
        }
    };
    for (int r = 0; r < len; r += 128) {
        batch(r, pn0, g0, h0, pn1, g1, h1);
        if (r + 64 >= len) break;
        batch(r + 64, pn1, g1, h1, pn0, g0, h0);
    }
    if (want_f && lane == 0) part[c] = T(0);
}

template <typename T, bool PADQ, int NM, bool TAB>
__global__ __launch_bounds__(kVjpPairThreads) void k_vjp_pairs(TiledArgs<T> A, const T *__restrict__ f,
                                                    const T *__restrict__ lam, T *__restrict__ part, int want_f,
                                                    const unsigned long long *__restrict__ lmax_bits,
                                                    const int32_t *__restrict__ chan,
                                                    const int32_t *__restrict__ chan0, double *__restrict__ gg2,
                                                    int gg2_mode) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    unsigned long long *s_j = reinterpret_cast<unsigned long long *>(smem);
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(s_j + A.lds_states);
    T *s_l = reinterpret_cast<T *>(s_ef + A.lds_states);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_l + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    const int n = t.lds ? t.p_hi - t.p_lo + 1 : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const StateRec<T> sr = A.st[t.p_lo + i];
        Pair2<T> ef;
        ef.a = sr.eps;
        ef.b = f[t.p_lo + i];
        s_ef[i] = ef;
        s_l[i] = lam[t.p_lo + i];
        s_kq[i] = PADQ ? sr.kqp : sr.kq;
        s_j[i] = 0ull;
    }
    if constexpr (sizeof(T) == 8 && TAB)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    const T scale = static_cast<T>(vjp_scale(A.nmax_bits, A.gmax_bits, lmax_bits, A.fmax_bits));
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (t.lds == 2)
            vjp_pair_chunk_q<T, PADQ, NM, TAB>(A, s_ef, s_kq, s_l, s_tab, s_j, scale, c, part, want_f != 0, chan,
                                               chan0, gg2, gg2_mode);
        else if (t.lds)
            vjp_pair_chunk<T, true, PADQ, NM, TAB>(A, f, lam, s_ef, s_kq, s_l, t.p_lo, s_tab, s_j, scale, c, part,
                                                   want_f != 0, chan, chan0, gg2, gg2_mode);
        else
            vjp_pair_chunk<T, false, PADQ, NM, TAB>(A, f, lam, s_ef, s_kq, s_l, t.p_lo, s_tab, s_j, scale, c,
                                                    part, want_f != 0, chan, chan0, gg2, gg2_mode);
    }
    if (!want_f) return;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long v = s_j[i];
        if (v) atomicAdd(A.jacc + t.p_lo + i, v);
    }
}

// dL/df_d = K [-(row partials, chunk order) + partner side], then the
// epilogue; the partner-side accumulator of d is cleared for the next call.
template <typename T>
__global__ void k_vjp_pairs_finish(TiledArgs<T> A, const T *__restrict__ part,
                                   const unsigned long long *__restrict__ lmax_bits, Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    T a = T(0);
    for (int c = A.dest_chunk[d]; c < A.dest_chunk[d + 1]; ++c) a += part[c];
    const double inv = 1.0 / vjp_scale(A.nmax_bits, A.gmax_bits, lmax_bits, A.fmax_bits);
    const long long j = static_cast<long long>(A.jacc[d]);
    A.jacc[d] = 0ull;
    const T jside = static_cast<T>(static_cast<double>(j) * inv);
    apply_epi(E, 0, d, A.S, A.K * (jside - a));
}

// I_d = K [(1 - f_d) sum b - f_d sum a] from the row side (chunk partials in
// chunk order) plus the partner side, then the epilogue; the partner-side
// accumulator of d is cleared for the next call.
template <typename T>
__global__ void k_sym_finish(TiledArgs<T> A, const T *__restrict__ f, const T *__restrict__ part,
                             Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    T a = T(0), b = T(0);
    for (int c = A.dest_chunk[d]; c < A.dest_chunk[d + 1]; ++c) {
        a += part[2 * c];
        b += part[2 * c + 1];
    }
    const double inv = 1.0 / sym_scale(A.nmax_bits, A.gmax_bits, A.fmax_bits);
    const long long j = static_cast<long long>(A.jacc[d]);
    A.jacc[d] = 0ull;
    const T fd = f[d];
    const T jside = static_cast<T>(static_cast<double>(j) * inv);
    apply_epi(E, 0, d, A.S, A.K * ((T(1) - fd) * b - fd * a + jside));
}

// destinations with several chunks: sum their partials in chunk order
template <typename T>
__global__ void k_tiled_finish(TiledArgs<T> A, const T *__restrict__ f, int64_t ldf,
                               const T *__restrict__ part, Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    const int c0 = A.dest_chunk[d], c1 = A.dest_chunk[d + 1];
    if (c1 - c0 == 1) return;
    const int b = blockIdx.y;
    const T *pb = part + static_cast<int64_t>(b) * A.n_chunks * 2;
    T a = T(0), bb = T(0);
    for (int c = c0; c < c1; ++c) {
        a += pb[2 * c];
        bb += pb[2 * c + 1];
    }
    const T fd = f[static_cast<int64_t>(b) * ldf + d];
    apply_epi(E, b, d, A.S, A.K * ((T(1) - fd) * bb - fd * a));
}

// ---- reverse, LDS-tiled ---------------------------------------------------
// Same tiles, chunks and stream pipeline as the forward pass.  Per entry:
//   dL/df_d  += -K (lam_d - lam_p) (a (1 - f_p) + b f_p)
//   dL/dg2_c  =  K (lam_d - lam_p) (bh f_p (1 - f_d) - ah f_d (1 - f_p))   (p > d only)
// The partner's {eps, f} and k come from LDS, lam_p from global memory.
template <typename T, bool LDS, bool PADQ, int U>
__device__ __forceinline__ void vjp_chunk2(const TiledArgs<T> &A, const T *__restrict__ fb,
                                           const T *__restrict__ lb, const Pair2<T> *s_ef,
                                           const uint32_t *s_kq, int p_lo, const double *s_tab,
                                           int64_t c, T *__restrict__ part, const Epi<T> &E,
                                           const int32_t *__restrict__ ent_chan,
                                           double *__restrict__ gg2, int gg2_mode) {
    const int lane = threadIdx.x & 63;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_beg[c + 1] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ gb = A.g2 + beg;
    const int32_t *__restrict__ cb = ent_chan + beg;
    const StateRec<T> sd = A.st[d];
    const uint32_t kd = PADQ ? sd.kqp : sd.kq;
    const T fd = fb[d];
    const T ld = lb[d];
    T acc = T(0);
    // one batch of gathered operands: coupling, energy difference, partner
    // occupation, lam_d - lam_p, {hw, N}, and the dL/d|g|^2 slot this entry
    // writes (-1: none) with its previous value when accumulating
    struct Gath {
        T g[U], de[U], fp[U], dl[U];
        Pair2<T> wn[U];
        int32_t ch[U];
        double old[U];
    };
    uint32_t pn1[U];
    T gs1[U];
    Gath G0;
    auto load_stream = [&](int r0, uint32_t (&pn)[U], T (&gs)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pn[u] = pb[r0 + u * 64 + lane];
            gs[u] = gb[r0 + u * 64 + lane];
        }
    };
    auto gather = [&](auto masked, const uint32_t (&pn)[U], const T (&gs)[U], int r0, Gath &o) {
        constexpr bool M = decltype(masked)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int rel = r0 + u * 64 + lane;
            const bool v = !M || rel < len;
            const int p = static_cast<int>(pn[u] >> 3);
            T ep, fp;
            uint32_t kp;
            if (LDS) {
                // a masked lane reads slot 0 (inside the allocation) and then
                // replaces what it read: partner = destination, so its table
                // index is the q = 0 entry and its operands are finite,
                // whatever the slot holds
                const int pl = v ? p - p_lo : 0;
                const Pair2<T> ef = s_ef[pl];
                ep = v ? ef.a : sd.eps;
                fp = v ? ef.b : T(0);
                kp = v ? s_kq[pl] : kd;
            } else {
                const StateRec<T> sp = A.st[p];
                ep = sp.eps;
                kp = PADQ ? sp.kqp : sp.kq;
                fp = fb[p];
            }
            const T lp = lb[p];
            const int q = PADQ ? static_cast<int>(kp - kd) + A.qoff
                               : q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.tq + static_cast<int64_t>(pn[u] & 7u) * A.tm];
            if constexpr (M) {
                // a table entry without channels may hold a non-finite N
                o.wn[u].a = v ? w.a : T(0);
                o.wn[u].b = v ? w.b : T(0);
                o.g[u] = v ? gs[u] : T(0);
            } else {
                o.wn[u] = w;
                o.g[u] = gs[u];
            }
            o.de[u] = sd.eps - ep;
            o.fp[u] = fp;
            o.dl[u] = ld - lp;
            const bool wr = gg2_mode && v && p > d;
            o.ch[u] = wr ? cb[rel] : -1;
            o.old[u] = (wr && gg2_mode == 2) ? gg2[o.ch[u]] : 0.0;
        }
    };
    using Masked = std::integral_constant<bool, true>;
    using Full = std::integral_constant<bool, false>;
    {
        uint32_t pn0[U];
        T gs0[U];
        load_stream(0, pn0, gs0);
        load_stream(64 * U, pn1, gs1);
        if (64 * U <= len) gather(Full{}, pn0, gs0, 0, G0);
        else gather(Masked{}, pn0, gs0, 0, G0);
    }
    for (int r = 0; r < len; r += 64 * U) {
        Gath G1;
        if (r + 128 * U <= len) gather(Full{}, pn1, gs1, r + 64 * U, G1);
        else gather(Masked{}, pn1, gs1, r + 64 * U, G1);
        load_stream(r + 128 * U, pn1, gs1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T xa = G0.de[u] + G0.wn[u].a, xe = G0.de[u] - G0.wn[u].a;
            const T da = stream_gauss(A, xa * xa, s_tab);
            const T dem = stream_gauss(A, xe * xe, s_tab);
            const T t = G0.wn[u].b * (da + dem);
            const T ah = t + dem, bh = t + da;
            const T fp = G0.fp[u], dl = G0.dl[u];
            acc += dl * G0.g[u] * (ah * (T(1) - fp) + bh * fp);
            if (G0.ch[u] >= 0)
                gg2[G0.ch[u]] = G0.old[u] + static_cast<double>(
                                                A.K * dl * (bh * fp * (T(1) - fd) - ah * fd * (T(1) - fp)));
        }
        G0 = G1;
    }
    if (E.mode < 0) return;
    acc = wave_sum(acc);
    if (lane == 0) {
        if (A.dest_chunk[d + 1] - A.dest_chunk[d] == 1)
            apply_epi(E, 0, d, A.S, -A.K * acc);
        else
            part[c] = acc;
    }
}

template <typename T, int U, bool PADQ>
__global__ __launch_bounds__(512) void k_vjp_tiled(TiledArgs<T> A, const T *__restrict__ f,
                                                   const T *__restrict__ lam, T *__restrict__ part,
                                                   Epi<T> E, const int32_t *__restrict__ ent_chan,
                                                   double *__restrict__ gg2, int gg2_mode) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(smem);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_ef + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    if (t.lds) {
        const int n = t.p_hi - t.p_lo + 1;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const StateRec<T> sr = A.st[t.p_lo + i];
            Pair2<T> ef;
            ef.a = sr.eps;
            ef.b = f[t.p_lo + i];
            s_ef[i] = ef;
            s_kq[i] = PADQ ? sr.kqp : sr.kq;
        }
    }
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (t.lds)
            vjp_chunk2<T, true, PADQ, U>(A, f, lam, s_ef, s_kq, t.p_lo, s_tab, c, part, E,
                                         ent_chan, gg2, gg2_mode);
        else
            vjp_chunk2<T, false, PADQ, U>(A, f, lam, s_ef, s_kq, t.p_lo, s_tab, c, part, E,
                                          ent_chan, gg2, gg2_mode);
    }
}

template <typename T>
__global__ void k_vjp_tiled_finish(TiledArgs<T> A, const T *__restrict__ part, Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    const int c0 = A.dest_chunk[d], c1 = A.dest_chunk[d + 1];
    if (c1 - c0 == 1) return;
    T a = T(0);
    for (int c = c0; c < c1; ++c) a += part[c];
    apply_epi(E, 0, d, A.S, -A.K * a);
}

// ---- transport iteration, LDS-tiled -------------------------------------
// x_new_d = tau_d (rhs_d + sum_entries W_e x_p) for the three field
// directions.  The partner window of x is staged in LDS (3 values per state)
// when the plan's LDS budget allows it, else x_p is gathered from global memory.
template <typename T, bool LDS>
__device__ __forceinline__ void tr_chunk(const TiledArgs<T> &A, const T *__restrict__ W,
                                         const Vec4<T> *__restrict__ x, const T *s_x, int p_lo,
                                         int64_t c, const Vec4<T> *__restrict__ rhs,
                                         const T *__restrict__ tau, Vec4<T> *__restrict__ part,
                                         Vec4<T> *__restrict__ x_new) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c];
    const int len = static_cast<int>(A.chunk_beg[c + 1] - beg);
    const uint32_t *__restrict__ pb = A.pnu + beg;
    const T *__restrict__ wb = W + beg;
    T a0 = T(0), a1 = T(0), a2 = T(0);
    auto load = [&](int r0, uint32_t (&pn)[U], T (&w)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pn[u] = pb[r0 + u * 64 + lane];
            w[u] = wb[r0 + u * 64 + lane];
        }
    };
    auto body = [&](auto masked, int r, const uint32_t (&pn)[U], const T (&w)[U]) {
        constexpr bool M = decltype(masked)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool v = !M || r + u * 64 + lane < len;
            const int p = static_cast<int>(pn[u] >> 3);
            T x0, x1, x2;
            if (LDS) {
                // a masked lane reads slot 0 and discards it (its weight is 0,
                // and 0 times a stale non-finite value would not be)
                const int pl = v ? p - p_lo : 0;
                x0 = v ? s_x[3 * pl] : T(0);
                x1 = v ? s_x[3 * pl + 1] : T(0);
                x2 = v ? s_x[3 * pl + 2] : T(0);
            } else {
                const Vec4<T> xp = x[p];
                x0 = xp.x;
                x1 = xp.y;
                x2 = xp.z;
            }
            const T ww = M ? (v ? w[u] : T(0)) : w[u];
            a0 += ww * x0;
            a1 += ww * x1;
            a2 += ww * x2;
        }
    };
    // the next batch's stream loads are in flight while this batch is
    // reduced; the arrays are padded, so they need no bound
    uint32_t pn0[U];
    T w0[U];
    load(0, pn0, w0);
    for (int r = 0; r < len; r += 64 * U) {
        uint32_t pn1[U];
        T w1[U];
        load(r + 64 * U, pn1, w1);
        if (r + 64 * U <= len) body(std::integral_constant<bool, false>{}, r, pn0, w0);
        else body(std::integral_constant<bool, true>{}, r, pn0, w0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pn0[u] = pn1[u];
            w0[u] = w1[u];
        }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
        if (A.dest_chunk[d + 1] - A.dest_chunk[d] == 1) {
            const Vec4<T> rr = rhs[d];
            const T t = tau[d];
            Vec4<T> o;
            o.x = t * (rr.x + a0);
            o.y = t * (rr.y + a1);
            o.z = t * (rr.z + a2);
            o.w = T(0);
            x_new[d] = o;
        } else {
            Vec4<T> o;
            o.x = a0;
            o.y = a1;
            o.z = a2;
            o.w = T(0);
            part[c] = o;
        }
    }
}

// W must be padded past its end like the entry arrays.
template <typename T>
__global__ __launch_bounds__(512) void k_tr_tiled(TiledArgs<T> A, int use_lds, const T *__restrict__ W,
                                                  const Vec4<T> *__restrict__ x,
                                                  const Vec4<T> *__restrict__ rhs,
                                                  const T *__restrict__ tau, Vec4<T> *__restrict__ part,
                                                  Vec4<T> *__restrict__ x_new) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    T *s_x = reinterpret_cast<T *>(smem);
    const bool lds = use_lds && t.lds;
    if (lds) {
        const int n = t.p_hi - t.p_lo + 1;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const Vec4<T> v = x[t.p_lo + i];
            s_x[3 * i] = v.x;
            s_x[3 * i + 1] = v.y;
            s_x[3 * i + 2] = v.z;
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        if (lds)
            tr_chunk<T, true>(A, W, x, s_x, t.p_lo, c, rhs, tau, part, x_new);
        else
            tr_chunk<T, false>(A, W, x, s_x, t.p_lo, c, rhs, tau, part, x_new);
    }
}

template <typename T>
__global__ void k_tr_tiled_finish(TiledArgs<T> A, const Vec4<T> *__restrict__ part,
                                  const Vec4<T> *__restrict__ rhs, const T *__restrict__ tau,
                                  Vec4<T> *__restrict__ x_new) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    const int c0 = A.dest_chunk[d], c1 = A.dest_chunk[d + 1];
    if (c1 - c0 == 1) return;
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int c = c0; c < c1; ++c) {
        a0 += part[c].x;
        a1 += part[c].y;
        a2 += part[c].z;
    }
    const Vec4<T> rr = rhs[d];
    const T t = tau[d];
    Vec4<T> o;
    o.x = t * (rr.x + a0);
    o.y = t * (rr.y + a1);
    o.z = t * (rr.z + a2);
    o.w = T(0);
    x_new[d] = o;
}

// ---- forward, batched (B vectors in one pass) -----------------------------
// Workgroup = batch tile: up to DPW destinations per wave, consecutive
// destinations sharing a partner window.  The window is walked in sub-tiles
// of PT partners; for each, f[p][0:64] (64 vectors, transposed, padded) and
// the partners' {eps, k} are staged in LDS.  For each of its destinations a
// wave then computes the coefficients of the entries whose partner lies in
// the sub-tile (lane = entry), merges entries with the same partner by a
// segmented shuffle reduction, and applies every merged coefficient pair to
// the 64 vectors (lane = vector):
//   acc_a[b] += a_p (1 - f_{p,b}),  acc_b[b] += b_p f_{p,b}.
// Each entry's coefficients are evaluated once per pass, not once per vector.
struct BTileRec {
    int32_t d0, d1;        // destinations [d0, d1)
    int32_t p_lo, n_sub;   // window start and number of sub-tiles
    int64_t off_base;      // sub_off index of destination d0
};

template <typename T> struct BArgs {
    const uint32_t *__restrict__ pnu;
    const T *__restrict__ g2;
    const StateRec<T> *__restrict__ st;
    const Pair2<T> *__restrict__ hwN;
    int64_t tq, tm;                          // as in TiledArgs
    const BTileRec *__restrict__ btiles;
    const int64_t *__restrict__ sub_off;   // per destination: n_sub + 1 entry offsets
    int S, nm, nq0, nq1, nq2, pt;
    int padq, qoff;                          // as in TiledArgs
    T mc, K;
    int64_t n_btiles;
    int xcd;                                 // as in TiledArgs
};

// Sub-tile entry offsets of the batch tiles: one workgroup per tile, one
// thread per (destination, slot); slot k is the first entry of the
// destination whose partner is >= p_lo + k pt (a lower bound on the sorted
// partner << 3 | mode keys; the row end if there is none).  A destination's
// entries are [chunk_beg[dest_chunk[x]], chunk_beg[dest_chunk[x + 1]]).
__global__ void k_sub_offsets(const BTileRec *__restrict__ tiles, const uint32_t *__restrict__ pnu,
                              const int64_t *__restrict__ chunk_beg,
                              const int32_t *__restrict__ dest_chunk, int S, int pt,
                              int64_t *__restrict__ sub_off) {
    const BTileRec t = tiles[blockIdx.x];
    const int per = t.n_sub + 1;
    const int n = (t.d1 - t.d0) * per;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int x = t.d0 + i / per;
        const int k = i % per;
        int64_t lo = chunk_beg[dest_chunk[x]], hi = chunk_beg[dest_chunk[x + 1]];
        const int64_t p = static_cast<int64_t>(t.p_lo) + static_cast<int64_t>(k) * pt;
        const uint32_t key = p >= S ? UINT32_MAX : static_cast<uint32_t>(p) << 3;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (pnu[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        sub_off[t.off_base + i] = lo;
    }
}

// Entries of one (destination, partner) pair: one per mode, at most 8 modes,
// no duplicates (both checked at plan build).
constexpr int kMaxRun = 8;

template <typename T> __device__ __forceinline__ T lane_bcast(T v, int src);
template <> __device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<long long>(lo) & 0xffffffffLL));
}
template <> __device__ __forceinline__ float lane_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Fourth word of a raw buffer resource on gfx9-family parts (32-bit data
// format; no swizzle, no index stride)
constexpr int kBufferDword3 = 0x00020000;

template <typename T> __device__ __forceinline__ T buffer_load_value(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ double buffer_load_value(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float buffer_load_value(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// RUN = 0: one phonon table for all vectors.  RUN > 0: a bath per vector
// (RUN bounds the entries of one pair, the mode count rounded up): N comes
// from nvec, [row][mode][64] for the launch's 64 vectors (nvec_ld values; row
// = the q index of the shared table), and an entry's coefficients split into
// the part without
// N, summed over the pair's modes as before, and |g|^2 (G(x + hw) +
// G(x - hw)), applied per vector with that vector's N.
template <typename T, int DPW, int RUN>
__global__ __launch_bounds__(512) void k_fwd_batched(BArgs<T> A, const T *__restrict__ f,
                                                     int64_t ldf, int B, Epi<T> E,
                                                     const T *__restrict__ nvec, int64_t nvec_ld) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int PT = A.pt;
    T *s_F = reinterpret_cast<T *>(smem);                                   // [PT][65]
    StateRec<T> *s_ek = reinterpret_cast<StateRec<T> *>(s_F + PT * 65);    // [PT]
    const int64_t ti = tile_of_block(A.n_btiles, A.xcd);
    if (ti < 0) return;
    const BTileRec t = A.btiles[ti];
    const int b0 = blockIdx.y * 64;
    const int nb = min(64, B - b0);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    const int nd = t.d1 - t.d0;
    T acc_a[DPW], acc_b[DPW];
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
        acc_a[j] = T(0);
        acc_b[j] = T(0);
    }
    for (int k = 0; k < t.n_sub; ++k) {
        const int pa = t.p_lo + k * PT;
        const int pc = min(PT, A.S - pa);
        __syncthreads();
        for (int i = threadIdx.x; i < pc * nb; i += blockDim.x) {
            const int bb = i / pc, pl = i - bb * pc;
            s_F[pl * 65 + bb] = f[static_cast<int64_t>(b0 + bb) * ldf + pa + pl];
        }
        for (int i = threadIdx.x; i < pc; i += blockDim.x) s_ek[i] = A.st[pa + i];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < DPW; ++j) {
            const int dl = wave + j * nw;
            if (dl < nd) {
                const int d = t.d0 + dl;
                const int64_t *so = A.sub_off + t.off_base + static_cast<int64_t>(dl) * (t.n_sub + 1);
                const int64_t e_lo = so[k], e_hi = so[k + 1];
                const StateRec<T> sd = A.st[d];
                // the sub-tile's terms are summed on their own, then added to
                // the running sums (two levels: each sum has at most PT terms
                // plus one per sub-tile, instead of one per partner)
                T sa = T(0), sb = T(0);
                for (int64_t e0 = e_lo; e0 < e_hi; e0 += 64) {
                    const int64_t e = e0 + lane;
                    const bool valid = e < e_hi;
                    int pl = -1 - lane;     // distinct for invalid lanes: never merged
                    T ca = T(0), cb = T(0), c1 = T(0);
                    int ti = 0;
                    if (valid) {
                        const uint32_t pn = A.pnu[e];
                        const T g = A.g2[e];
                        pl = static_cast<int>(pn >> 3) - pa;
                        const StateRec<T> sp = s_ek[pl];
                        const int q = A.padq ? static_cast<int>(sp.kqp - sd.kqp) + A.qoff
                                             : q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
                        const Pair2<T> wn = A.hwN[static_cast<int64_t>(q) * A.tq + static_cast<int64_t>(pn & 7u) * A.tm];
                        const T de = sd.eps - sp.eps;
                        const T xa = de + wn.a, xe = de - wn.a;
                        const T da = gauss_exp(xa * xa * A.mc);
                        const T dem = gauss_exp(xe * xe * A.mc);
                        if constexpr (RUN > 0) {
                            ca = g * dem;
                            cb = g * da;
                            c1 = g * (da + dem);
                            ti = q * A.nm + static_cast<int>(pn & 7u);
                        } else {
                            const T tt = wn.b * (da + dem);
                            ca = g * (tt + dem);
                            cb = g * (tt + da);
                        }
                    }
                    // sum each run of equal partners into its first lane (a run is
                    // one pair over its modes, at most kMaxRun lanes)
#pragma unroll
                    for (int off = 1; off < kMaxRun; off <<= 1) {
                        const T oa = __shfl_down(ca, off, 64);
                        const T ob = __shfl_down(cb, off, 64);
                        const int op = __shfl_down(pl, off, 64);
                        if (lane + off < 64 && op == pl) {
                            ca += oa;
                            cb += ob;
                        }
                    }
                    const int prev = __shfl_up(pl, 1, 64);
                    const bool head = valid && (lane == 0 || prev != pl);
                    unsigned long long m = __ballot(head);
                    if constexpr (RUN > 0) {
                        // the run of a head ends at the next head or at the
                        // last valid lane; each of its entries adds
                        // c1 N_b(q, mode) for this lane's vector b
                        const int nvalid = static_cast<int>(min<int64_t>(64, e_hi - e0));
                        // buffer loads: the row offset is a scalar operand and
                        // the lane offset a fixed register, so a load needs no
                        // address registers (whose reuse would make the wave
                        // wait for loads in flight); reads past the table
                        // return 0
                        const __amdgpu_buffer_rsrc_t nvr = __builtin_amdgcn_make_buffer_rsrc(
                            const_cast<T *>(nvec), 0, static_cast<int>(nvec_ld * sizeof(T)), kBufferDword3);
                        const int lane_off = lane * static_cast<int>(sizeof(T));
                        // entries past a run re-read its last one, weighted 0
                        auto load_run = [&](int src, int end, T (&buf)[RUN]) {
#pragma unroll
                            for (int r = 0; r < RUN; ++r) {
                                const int j = min(src + r, end - 1);
                                const int row = __builtin_amdgcn_readlane(ti, j) * 64 * static_cast<int>(sizeof(T));
                                buf[r] = buffer_load_value<T>(nvr, lane_off, row);
                            }
                        };
                        auto apply_run = [&](int src, int end, const T (&buf)[RUN]) {
                            T nsum = T(0);
#pragma unroll
                            for (int r = 0; r < RUN; ++r) {
                                const int j = min(src + r, end - 1);
                                const T w = src + r < end ? lane_bcast(c1, j) : T(0);
                                nsum += w * buf[r];
                            }
                            const T a = lane_bcast(ca, src) + nsum;
                            const T bq = lane_bcast(cb, src) + nsum;
                            const int pls = __builtin_amdgcn_readlane(pl, src);
                            const T fpb = s_F[pls * 65 + lane];
                            sa += a * (T(1) - fpb);
                            sb += bq * fpb;
                        };
                        // two runs in flight: the next run's N loads are
                        // issued before this run's are waited for (two
                        // register sets, so nothing is copied between them).
                        // Past the last run the loads repeat the current
                        // one, so every step issues the same number of loads
                        // and the wait for a run never covers the next.
                        if (m) {
                            T b0[RUN], b1[RUN];
                            int s0 = __builtin_ctzll(m), s1, t1;
                            m &= m - 1;
                            int t0 = m ? __builtin_ctzll(m) : nvalid;
                            load_run(s0, t0, b0);
                            while (true) {
                                const bool h1 = m != 0;
                                s1 = h1 ? __builtin_ctzll(m) : s0;
                                m &= m - 1;
                                t1 = h1 ? (m ? __builtin_ctzll(m) : nvalid) : t0;
                                load_run(s1, t1, b1);
                                apply_run(s0, t0, b0);
                                if (!h1) break;
                                const bool h0 = m != 0;
                                s0 = h0 ? __builtin_ctzll(m) : s1;
                                m &= m - 1;
                                t0 = h0 ? (m ? __builtin_ctzll(m) : nvalid) : t1;
                                load_run(s0, t0, b0);
                                apply_run(s1, t1, b1);
                                if (!h0) break;
                            }
                        }
                    } else {
                        while (m) {
                            const int src = __builtin_ctzll(m);
                            m &= m - 1;
                            const T a = lane_bcast(ca, src);
                            const T bq = lane_bcast(cb, src);
                            const int pls = __builtin_amdgcn_readlane(pl, src);
                            const T fpb = s_F[pls * 65 + lane];
                            sa += a * (T(1) - fpb);
                            sb += bq * fpb;
                        }
                    }
                }
                acc_a[j] += sa;
                acc_b[j] += sb;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
        const int dl = wave + j * nw;
        if (dl < nd && lane < nb) {
            const int d = t.d0 + dl;
            const int b = b0 + lane;
            const T fd = f[static_cast<int64_t>(b) * ldf + d];
            apply_epi(E, b, d, A.S, A.K * ((T(1) - fd) * acc_b[j] - fd * acc_a[j]));
        }
    }
}

// Moves v from the lane the DPP control selects (rows of 16 lanes; ROWS masks
// the rows that receive, the others and lanes without a source get 0).
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Sum over the 64 lanes of a wave, returned to every lane, without LDS:
// shifts by 1, 2, 4 and 8 lanes inside each row of 16 leave the row's sum in
// its lane 15; broadcasting lane 15 into the next row (rows 1 and 3) and then
// lane 31 into rows 2 and 3 leaves the total in lane 63.  Fixed order.
template <typename T> __device__ __forceinline__ T wave_total(T v) {
    v += dpp_mov<0x111, 0xf>(v);   // row_shr:1
    v += dpp_mov<0x112, 0xf>(v);   // row_shr:2
    v += dpp_mov<0x114, 0xf>(v);   // row_shr:4
    v += dpp_mov<0x118, 0xf>(v);   // row_shr:8
    v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31
    return lane_bcast(v, 63);
}

// Reverse mode of Eq. 2 for up to 64 vectors sharing one phonon table
// (vectors b0 .. b0 + nb - 1; lane = vector).  Tiles and sub-tiles as in
// k_fwd_batched; the LDS tile holds {f_p, lam_p} per (partner, vector).
//   dL/df_d = -K sum_e (lam_d - lam_p) u_e,  u_e = a_e (1 - f_p) + b_e f_p,
// summed per lane as lam_d sum u - sum lam_p u.  The |g|^2 gradient of a
// channel, written by its entry with p > d, is
//   K [bh sum_b (lam_d - lam_p) f_p (1 - f_d) - ah sum_b (lam_d - lam_p) f_d (1 - f_p)],
// where the two sums over the vectors depend only on the pair (d, p): they are
// reduced across the wave once per run of equal partners and serve every mode
// of the run.  gg2_mode: 0 none, 1 overwrite, 2 add.  Every slot is written by
// one lane of one launch: deterministic.
// RUN > 0: a bath per vector, N from nvec as in k_fwd_batched (the 64
// vectors of this launch).  With c = G(x + hw) + G(x - hw) the coefficients
// split into the N-free parts and c N_b; a channel's |g|^2 gradient is
//   K [G(x + hw) p2 - G(x - hw) p1 + c sum_b N_b (P2_b - P1_b)],
// P1_b = (lam_d - lam_p) f_d (1 - f_p), P2_b = (lam_d - lam_p) f_p (1 - f_d),
// p1 and p2 their sums over the vectors: one more sum over the wave per
// channel.
template <typename T, int DPW, int RUN>
__global__ __launch_bounds__(512) void k_vjp_batched(BArgs<T> A, const T *__restrict__ f, int64_t ldf,
                                                     const T *__restrict__ lam, int64_t ldl, int b0,
                                                     int nb, T *__restrict__ gf, int64_t ldgf,
                                                     const int32_t *__restrict__ ent_chan,
                                                     double *__restrict__ gg2, int gg2_mode,
                                                     const T *__restrict__ nvec, int64_t nvec_ld) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int PT = A.pt;
    Pair2<T> *s_FL = reinterpret_cast<Pair2<T> *>(smem);                   // [PT][65]
    StateRec<T> *s_ek = reinterpret_cast<StateRec<T> *>(s_FL + PT * 65);  // [PT]
    const int64_t ti = tile_of_block(A.n_btiles, A.xcd);
    if (ti < 0) return;
    const BTileRec t = A.btiles[ti];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    const int nd = t.d1 - t.d0;
    const bool lv = lane < nb;
    T fd[DPW], ld[DPW], acc_u[DPW], acc_l[DPW];
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
        const int dl = wave + j * nw;
        const bool ok = dl < nd && lv;
        const int64_t row = static_cast<int64_t>(b0 + lane);
        fd[j] = ok ? f[row * ldf + t.d0 + dl] : T(0);
        ld[j] = ok ? lam[row * ldl + t.d0 + dl] : T(0);
        acc_u[j] = T(0);
        acc_l[j] = T(0);
    }
    for (int k = 0; k < t.n_sub; ++k) {
        const int pa = t.p_lo + k * PT;
        const int pc = min(PT, A.S - pa);
        __syncthreads();
        // vectors past nb hold f = lam = 0: their terms vanish in every sum
        for (int i = threadIdx.x; i < pc * 64; i += blockDim.x) {
            const int bb = i / pc, pl = i - bb * pc;
            Pair2<T> v;
            v.a = T(0);
            v.b = T(0);
            if (bb < nb) {
                const int64_t row = static_cast<int64_t>(b0 + bb);
                v.a = f[row * ldf + pa + pl];
                v.b = lam[row * ldl + pa + pl];
            }
            s_FL[pl * 65 + bb] = v;
        }
        for (int i = threadIdx.x; i < pc; i += blockDim.x) s_ek[i] = A.st[pa + i];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < DPW; ++j) {
            const int dl = wave + j * nw;
            if (dl < nd) {
                const int d = t.d0 + dl;
                const int64_t *so = A.sub_off + t.off_base + static_cast<int64_t>(dl) * (t.n_sub + 1);
                const int64_t e_lo = so[k], e_hi = so[k + 1];
                const StateRec<T> sd = A.st[d];
                // the pairs of this sub-tile with p > d carry the |g|^2 gradients
                const bool g_any = gg2_mode != 0 && pa + pc - 1 > d;
                T su = T(0), sl = T(0);   // this sub-tile's sums (two-level, as in the forward)
                for (int64_t e0 = e_lo; e0 < e_hi; e0 += 64) {
                    const int64_t e = e0 + lane;
                    const bool valid = e < e_hi;
                    int pl = -1 - lane;     // distinct for invalid lanes: never merged
                    T ca = T(0), cb = T(0), ah = T(0), bh = T(0), c1 = T(0);
                    int32_t ch = -1;
                    int ti = 0;
                    if (valid) {
                        const uint32_t pn = A.pnu[e];
                        const T g = A.g2[e];
                        pl = static_cast<int>(pn >> 3) - pa;
                        const StateRec<T> sp = s_ek[pl];
                        const int q = A.padq ? static_cast<int>(sp.kqp - sd.kqp) + A.qoff
                                             : q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
                        const Pair2<T> wn = A.hwN[static_cast<int64_t>(q) * A.tq + static_cast<int64_t>(pn & 7u) * A.tm];
                        const T de = sd.eps - sp.eps;
                        const T xa = de + wn.a, xe = de - wn.a;
                        const T da = gauss_exp(xa * xa * A.mc);
                        const T dem = gauss_exp(xe * xe * A.mc);
                        if constexpr (RUN > 0) {
                            // ah, bh keep the N-free parts; c1 the N coefficient
                            ah = dem;
                            bh = da;
                            ca = g * dem;
                            cb = g * da;
                            c1 = g * (da + dem);
                            ti = q * A.nm + static_cast<int>(pn & 7u);
                        } else {
                            const T tt = wn.b * (da + dem);
                            ah = tt + dem;
                            bh = tt + da;
                            ca = g * ah;
                            cb = g * bh;
                        }
                        if (g_any && pa + pl > d) ch = ent_chan[e];
                    }
                    // sum each run of equal partners into its first lane (a run is
                    // one pair over its modes, at most kMaxRun lanes)
#pragma unroll
                    for (int off = 1; off < kMaxRun; off <<= 1) {
                        const T oa = __shfl_down(ca, off, 64);
                        const T ob = __shfl_down(cb, off, 64);
                        const int op = __shfl_down(pl, off, 64);
                        if (lane + off < 64 && op == pl) {
                            ca += oa;
                            cb += ob;
                        }
                    }
                    const int prev = __shfl_up(pl, 1, 64);
                    const bool head = valid && (lane == 0 || prev != pl);
                    unsigned long long m = __ballot(head);
                    if constexpr (RUN > 0) {
                        // a run of entries (one pair over its modes) ends at
                        // the next head or the last valid lane; its N per
                        // vector through a buffer resource (reads past the
                        // table return 0)
                        const int nvalid = static_cast<int>(min<int64_t>(64, e_hi - e0));
                        const __amdgpu_buffer_rsrc_t nvr = __builtin_amdgcn_make_buffer_rsrc(
                            const_cast<T *>(nvec), 0, static_cast<int>(nvec_ld * sizeof(T)), kBufferDword3);
                        const int lane_off = lane * static_cast<int>(sizeof(T));
                        while (m) {
                            const int src = __builtin_ctzll(m);
                            m &= m - 1;
                            const int end = m ? __builtin_ctzll(m) : nvalid;
                            T nv[RUN];
#pragma unroll
                            for (int r = 0; r < RUN; ++r) {
                                const int jj = min(src + r, end - 1);
                                const int row = __builtin_amdgcn_readlane(ti, jj) * 64 * static_cast<int>(sizeof(T));
                                nv[r] = buffer_load_value<T>(nvr, lane_off, row);
                            }
                            T nsum = T(0);
#pragma unroll
                            for (int r = 0; r < RUN; ++r) {
                                const int jj = min(src + r, end - 1);
                                const T w = src + r < end ? lane_bcast(c1, jj) : T(0);
                                nsum += w * nv[r];
                            }
                            const T a = lane_bcast(ca, src) + nsum;
                            const T bq = lane_bcast(cb, src) + nsum;
                            const int pls = __builtin_amdgcn_readlane(pl, src);
                            const Pair2<T> fl = s_FL[pls * 65 + lane];
                            const T u = a + (bq - a) * fl.a;
                            su += u;
                            sl += fl.b * u;
                            if (g_any && pa + pls > d) {
                                const T dlm = ld[j] - fl.b;
                                const T q1 = dlm * fd[j] * (T(1) - fl.a);
                                const T q2 = dlm * fl.a * (T(1) - fd[j]);
                                const T p1 = wave_total(q1);
                                const T p2 = wave_total(q2);
#pragma unroll
                                for (int r = 0; r < RUN; ++r) {
                                    if (src + r >= end) break;
                                    const T rn = wave_total(nv[r] * (q2 - q1));
                                    if (lane == src + r && ch >= 0) {
                                        const double v = static_cast<double>(A.K * (bh * p2 - ah * p1 + (ah + bh) * rn));
                                        gg2[ch] = gg2_mode == 2 ? gg2[ch] + v : v;
                                    }
                                }
                            }
                        }
                    } else {
                        while (m) {
                            const int src = __builtin_ctzll(m);
                            m &= m - 1;
                            const T a = lane_bcast(ca, src);
                            const T bq = lane_bcast(cb, src);
                            const int pls = __builtin_amdgcn_readlane(pl, src);
                            const Pair2<T> fl = s_FL[pls * 65 + lane];
                            const T u = a + (bq - a) * fl.a;
                            su += u;
                            sl += fl.b * u;
                            if (g_any && pa + pls > d) {
                                const T dlm = ld[j] - fl.b;
                                const T p1 = wave_total(dlm * fd[j] * (T(1) - fl.a));
                                const T p2 = wave_total(dlm * fl.a * (T(1) - fd[j]));
                                if (pl == pls && ch >= 0) {
                                    const double v = static_cast<double>(A.K * (bh * p2 - ah * p1));
                                    gg2[ch] = gg2_mode == 2 ? gg2[ch] + v : v;
                                }
                            }
                        }
                    }
                }
                acc_u[j] += su;
                acc_l[j] += sl;
            }
        }
    }
    if (!gf) return;
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
        const int dl = wave + j * nw;
        if (dl < nd && lv)
            gf[static_cast<int64_t>(b0 + lane) * ldgf + t.d0 + dl] = -A.K * (ld[j] * acc_u[j] - acc_l[j]);
    }
}

// ---- phonon side of the same processes (coupled e-ph dynamics) ----------
// A channel (i, j, nu) carries the processes that exchange phonon (nu, q),
// q = k_j - k_i (i -> j absorbing it, j -> i emitting it, delta
// G(e_i - e_j + hw)), and those that exchange (nu, -q) (delta
// G(e_i - e_j - hw)).  The channels are grouped by the unordered pair
// {qc, -qc} into pair records (a, b) with k_b - k_a = qc and one |g|^2 slot
// per mode (zero where the pair has no channel of that mode), bucketed by qc
// and cut into chunks of at most kPhChunk records.  One wave reduces one
// chunk: with P1 = f_b (1 - f_a), P2 = f_a (1 - f_b), a record adds
//   |g|^2 G(e_a - e_b + hw(qc)) (P1 + N(qc) (P1 - P2))    to bin (qc, nu),
//   |g|^2 G(e_a - e_b - hw(-qc)) (P2 - N(-qc) (P1 - P2))  to bin (-qc, nu),
// (net emission: (N+1) x gain - N x loss), in registers, in record order;
// the two sums per mode go to the chunk's partials, and k_phonon_bins_finish
// adds the partials of each bin in chunk order.  No atomics.
constexpr int kPhChunk = 512;

template <typename T> struct PhArgs {
    const uint32_t *__restrict__ pa;
    const uint32_t *__restrict__ pb;
    const T *__restrict__ g2;          // [n_modes][ld]
    int64_t ld;
    const StateRec<T> *__restrict__ st;
    const T *__restrict__ hw;          // [Nq][n_modes]
    const int64_t *__restrict__ chunk_beg;    // [n_chunks + 1] record ranges
    const int32_t *__restrict__ chunk_bucket; // [n_chunks]
    const int32_t *__restrict__ bucket_chunk; // [n_buckets + 1]
    const int32_t *__restrict__ bucket_q;     // [n_buckets] qc
    const int32_t *__restrict__ bucket_qm;    // [n_buckets] -qc
    const uint32_t *__restrict__ bucket_modes;
    const int32_t *__restrict__ q_bucket;     // [Nq] 2 bucket + side, -1: none
    int64_t n_chunks;
    int64_t nq;
    int nm;
    T mc;                    // Gaussian exponent scale, base 2
    double mc256;            // 256 mc (FP64 table exponential)
    const double *__restrict__ e2tab;
    double Kp;               // 2 pi / (hbar N_k) / (sigma sqrt(2 pi))
    uint32_t elastic;        // bit nu: mode nu is elastic (no phonon side)
    const int32_t *__restrict__ chan;   // [n_modes][ld] caller channel of each slot, -1: none
};

template <typename T>
__device__ __forceinline__ T ph_gauss(const PhArgs<T> &A, T x, const double *tab) {
    if constexpr (sizeof(T) == 8) return gauss_exp2_tab(x * x * A.mc256, tab);
    else return __builtin_amdgcn_exp2f(x * x * A.mc);
}

// The mode loop is unrolled to NM >= nm slots (1, 2, 3, 4, 6 or 8).  The
// record stream (a, b and the |g|^2 slots) runs one batch ahead of the state
// gathers and the evaluation, with two register sets, as in the pair pass;
// a lane past the chunk's end re-reads the chunk's last record and adds
// nothing.
template <typename T, int NM>
__global__ __launch_bounds__(256) void k_phonon_bins(PhArgs<T> A, const T *__restrict__ f,
                                                     const T *__restrict__ nph, T *__restrict__ part) {
    __shared__ double s_tab[kExpTab];
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) +
                      __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    if (c >= A.n_chunks) return;
    const int nm = A.nm;
    const int bk = A.chunk_bucket[c];
    const int64_t qc = A.bucket_q[bk], qm = A.bucket_qm[bk];
    const uint32_t modes = A.bucket_modes[bk] & ~A.elastic;
    T w1[NM], n1[NM], w2[NM], n2[NM], acc1[NM], acc2[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const bool on = m < nm && ((modes >> m) & 1u);
        const int mm = min(m, nm - 1);
        w1[m] = on ? A.hw[qc * nm + mm] : T(0);
        n1[m] = on ? nph[qc * nm + mm] : T(0);
        w2[m] = on ? A.hw[qm * nm + mm] : T(0);
        n2[m] = on ? nph[qm * nm + mm] : T(0);
        acc1[m] = T(0);
        acc2[m] = T(0);
    }
    const int64_t beg = A.chunk_beg[c];
    const int n = static_cast<int>(A.chunk_beg[c + 1] - beg);
    auto rec = [&](int r) { return beg + min(r + lane, n - 1); };
    uint32_t a0 = A.pa[rec(0)], b0 = A.pb[rec(0)], a1 = 0, b1 = 0;
    T g0[NM], g1[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) g0[m] = A.g2[min(m, nm - 1) * A.ld + rec(0)];
    auto batch = [&](int r, const uint32_t a, const uint32_t b, const T (&g)[NM], uint32_t &an, uint32_t &bn,
                     T (&gn)[NM]) {
        const bool v = r + lane < n;
        const T fa = f[a], fb = f[b];
        const T d = A.st[a].eps - A.st[b].eps;
        __builtin_amdgcn_sched_barrier(0);
        const int64_t x = rec(r + 64);
        an = A.pa[x];
        bn = A.pb[x];
#pragma unroll
        for (int m = 0; m < NM; ++m) gn[m] = A.g2[min(m, nm - 1) * A.ld + x];
        __builtin_amdgcn_sched_barrier(0);
        const T p1 = fb * (T(1) - fa), p2 = fa * (T(1) - fb);
        const T dp = p1 - p2;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            // modes outside the bucket (and elastic ones) add nothing
            const T gm = keep_or_zero(g[m], v && m < nm && ((modes >> m) & 1u));
            const T ga = ph_gauss(A, d + w1[m], s_tab);
            const T ge = ph_gauss(A, d - w2[m], s_tab);
            acc1[m] = fma(gm * ga, fma(n1[m], dp, p1), acc1[m]);
            acc2[m] = fma(gm * ge, fma(-n2[m], dp, p2), acc2[m]);
        }
    };
    for (int r = 0; r < n; r += 128) {
        batch(r, a0, b0, g0, a1, b1, g1);
        if (r + 64 >= n) break;
        batch(r + 64, a1, b1, g1, a0, b0, g0);
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        acc1[m] = wave_sum(acc1[m]);
        acc2[m] = wave_sum(acc2[m]);
    }
    if (lane == 0) {
        T *pc = part + c * 2 * nm;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if (m >= nm) break;
            pc[m] = acc1[m];
            pc[nm + m] = acc2[m];
        }
    }
}

// Reverse mode over the same records at a stage (u, N) of the coupled step,
// given lam = dL/dI and mu = dL/d(dN/dt) per bin.  Per record and mode, with
// x = e_a - e_b, G1 = G(x + hw(qc)), E1 = G(x - hw(qc)), G2 = G(x + hw(-qc)),
// E2 = G(x - hw(-qc)) (two exponentials when hw(-qc) = hw(qc)):
//   bin (qc, nu):  |g|^2 (f_b - f_a) [Ke lam_a (G1 + E1) + Kp mu(qc) G1]
//   bin (-qc, nu): |g|^2 (f_a - f_b) [Ke lam_b (G2 + E2) + Kp mu(-qc) E2]
// (dL/dN: the collision integral is affine in N, the phonon-side rate too);
// and, for phonon modes, dL/d|g|^2 of the record's channel gains
//   Kp [mu(qc) G1 (P1 + N(qc) (P1 - P2)) + mu(-qc) E2 (P2 - N(-qc) (P1 - P2))]
// (its only writer: every channel has one slot).  Elastic modes have no
// phonon side: only their lam terms.  lam or mu may be null (taken as 0).
// The mode loop is unrolled to NM >= nm slots and the record stream (a, b,
// |g|^2 slots and, with gg2, the slots' channels) runs one batch ahead, as in
// k_phonon_bins.  With gg2, the old values of a batch's channels are loaded
// before the next batch's stream is issued, so that waiting for them does
// not wait for the stream; each channel has one slot, so nothing else writes
// it in between.  A lane past the chunk's end, or a slot without a channel,
// loads a valid address and stores nothing.
template <typename T, int NM>
__global__ __launch_bounds__(256) void k_phonon_bins_adj(PhArgs<T> A, const T *__restrict__ f,
                                                         const T *__restrict__ nph, const T *__restrict__ lam,
                                                         const T *__restrict__ mu, T *__restrict__ part,
                                                         double *__restrict__ gg2, double Ke) {
    __shared__ double s_tab[kExpTab];
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) +
                      __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    if (c >= A.n_chunks) return;
    const int nm = A.nm;
    const int bk = A.chunk_bucket[c];
    const int64_t qc = A.bucket_q[bk], qm = A.bucket_qm[bk];
    const uint32_t modes = A.bucket_modes[bk];
    const uint32_t phon = mu ? modes & ~A.elastic : 0u;
    const bool want_g = gg2 != nullptr && phon != 0u;
    const T ke = static_cast<T>(Ke), kp = static_cast<T>(A.Kp);
    T w1[NM], n1[NM], w2[NM], n2[NM], m1[NM], m2[NM], acc1[NM], acc2[NM];
    bool same = true;   // hw(-qc) = hw(qc) for every mode of the bucket
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const int mm = min(m, nm - 1);
        const bool on = m < nm && ((modes >> m) & 1u);
        const bool ph = m < nm && ((phon >> m) & 1u);
        w1[m] = on ? A.hw[qc * nm + mm] : T(0);
        w2[m] = on ? A.hw[qm * nm + mm] : T(0);
        n1[m] = ph ? nph[qc * nm + mm] : T(0);
        n2[m] = ph ? nph[qm * nm + mm] : T(0);
        m1[m] = ph ? mu[qc * nm + mm] : T(0);
        m2[m] = ph ? mu[qm * nm + mm] : T(0);
        same = same && w2[m] == w1[m];
        acc1[m] = T(0);
        acc2[m] = T(0);
    }
    const int64_t beg = A.chunk_beg[c];
    const int n = static_cast<int>(A.chunk_beg[c + 1] - beg);
    auto rec = [&](int r) { return beg + min(r + lane, n - 1); };
    uint32_t a0 = A.pa[rec(0)], b0 = A.pb[rec(0)], a1 = 0, b1 = 0;
    T g0[NM], g1[NM];
    int32_t h0[NM], h1[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        g0[m] = A.g2[min(m, nm - 1) * A.ld + rec(0)];
        h0[m] = want_g ? A.chan[min(m, nm - 1) * A.ld + rec(0)] : -1;
    }
    auto batch = [&](int r, const uint32_t a, const uint32_t b, const T (&g)[NM], const int32_t (&h)[NM],
                     uint32_t &an, uint32_t &bn, T (&gn)[NM], int32_t (&hn)[NM]) {
        const bool v = r + lane < n;
        const T fa = f[a], fb = f[b];
        const T la = lam ? lam[a] : T(0), lb = lam ? lam[b] : T(0);
        const T x = A.st[a].eps - A.st[b].eps;
        double old[NM];
        if (want_g) {
#pragma unroll
            for (int m = 0; m < NM; ++m) old[m] = gg2[h[m] >= 0 ? h[m] : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        const int64_t xi = rec(r + 64);
        an = A.pa[xi];
        bn = A.pb[xi];
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            gn[m] = A.g2[min(m, nm - 1) * A.ld + xi];
            hn[m] = want_g ? A.chan[min(m, nm - 1) * A.ld + xi] : -1;
        }
        __builtin_amdgcn_sched_barrier(0);
        const T p1 = fb * (T(1) - fa), p2 = fa * (T(1) - fb);
        const T dp = p1 - p2;   // = f_b - f_a
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const bool on = v && m < nm && ((modes >> m) & 1u);
            const T gm = keep_or_zero(g[m], on);
            const T gq1 = ph_gauss(A, x + w1[m], s_tab);
            const T e1 = ph_gauss(A, x - w1[m], s_tab);
            T gq2 = gq1, e2 = e1;
            if (!same) {
                gq2 = ph_gauss(A, x + w2[m], s_tab);
                e2 = ph_gauss(A, x - w2[m], s_tab);
            }
            acc1[m] += gm * dp * (ke * la * (gq1 + e1) + kp * m1[m] * gq1);
            acc2[m] -= gm * dp * (ke * lb * (gq2 + e2) + kp * m2[m] * e2);
            if (want_g && on && ((phon >> m) & 1u) && h[m] >= 0)
                gg2[h[m]] = old[m] + static_cast<double>(kp * (m1[m] * gq1 * (p1 + n1[m] * dp) +
                                                                m2[m] * e2 * (p2 - n2[m] * dp)));
        }
    };
    for (int r = 0; r < n; r += 128) {
        batch(r, a0, b0, g0, h0, a1, b1, g1, h1);
        if (r + 64 >= n) break;
        batch(r + 64, a1, b1, g1, h1, a0, b0, g0, h0);
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        acc1[m] = wave_sum(acc1[m]);
        acc2[m] = wave_sum(acc2[m]);
    }
    if (lane == 0) {
        T *pc = part + c * 2 * nm;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if (m >= nm) break;
            pc[m] = acc1[m];
            pc[nm + m] = acc2[m];
        }
    }
}

// Per-vector baths of the batched pass, 64 vectors: entry (row nm + nu) 64 + j
// holds N of vector j (0 past the last of the B vectors) at table row `row`
// and mode nu, for the box rows in `used` (pad != 0; other rows keep their
// zeros) or every q (pad = 0, n_rows = Nq).  nph holds B tables of [Nq][nm].
template <typename T>
__global__ void k_pack_nvec(const T *__restrict__ nph, T *__restrict__ out, int pad, QBox Bx, int nm,
                            const int32_t *__restrict__ used, int n_rows, int B) {
    const int64_t tab = static_cast<int64_t>(Bx.n[0]) * Bx.n[1] * Bx.n[2] * nm;
    const int64_t n = static_cast<int64_t>(n_rows) * nm * 64;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int j = static_cast<int>(i & 63);
        const int64_t r = i >> 6;
        const int nu = static_cast<int>(r % nm);
        const int u = static_cast<int>(r / nm);
        const int row = pad ? used[u] : u;
        const int64_t q = pad ? box_q(row, Bx) : row;
        out[(static_cast<int64_t>(row) * nm + nu) * 64 + j] = j < B ? nph[static_cast<int64_t>(j) * tab + q * nm + nu] : T(0);
    }
}

// {hw, N, mu} per (q, mode) for the reverse of the phonon-side rate: the
// box of k_pack_hwN_pad with the modes of one row adjacent (pad != 0), or the
// plain table.
template <typename T>
__global__ void k_pack_hwNmu(const T *__restrict__ hw, const T *__restrict__ nph, const T *__restrict__ mu,
                             Vec4<T> *__restrict__ out, int pad, QBox B, int nm, const int32_t *__restrict__ used,
                             int64_t n) {
    // pad != 0: n = (rows in used) nm, other box rows keep their zeros
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        int64_t src = i, dst = i;
        if (pad) {
            const int row = used[i / nm];
            src = static_cast<int64_t>(box_q(row, B)) * nm + i % nm;
            dst = static_cast<int64_t>(row) * nm + i % nm;
        }
        Vec4<T> v;
        v.x = hw[src];
        v.y = nph[src];
        v.z = mu[src];
        v.w = T(0);
        out[dst] = v;
    }
}

// Electron side of the reverse of the phonon-side rate: for every entry
// (d, p, nu) with q = k_p - k_d (x = e_d - e_p),
//   dL/df_d += Kp |g|^2 [mu(-q) G(x - hw(-q)) (N(-q) + 1 - f_p) - mu(q) G(x + hw(q)) (N(q) + f_p)]
// (the entry's channel feeds bin q through G(x + hw(q)) and bin -q through
// G(x - hw(-q)); the same form holds from either end of the channel).  One
// workgroup per chunk of the destination layout; a destination with one
// chunk adds its sum to out, others leave a partial for k_vjp_phonon_f_finish.
// The entry stream (partner word, |g|^2) runs one batch ahead of the state
// and table gathers, with two register sets, as in the pair pass; the
// entry arrays are padded past their end, so the prefetch needs no bound, and
// a thread past the row's end (or on an elastic mode) adds nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_vjp_phonon_f(TiledArgs<T> A, const Vec4<T> *__restrict__ tab,
                                                      const T *__restrict__ f, uint32_t elastic,
                                                      double Kp, T *__restrict__ out, T *__restrict__ part) {
    __shared__ double s_tab[kExpTab];
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    __syncthreads();
    const int64_t c = blockIdx.x;
    if (c >= A.n_chunks) return;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c], end = A.chunk_beg[c + 1];
    const StateRec<T> sd = A.st[d];
    const int64_t stride = blockDim.x;
    T acc[1] = {T(0)};
    int64_t e = beg + threadIdx.x;
    uint32_t pn0 = A.pnu[e], pn1 = 0;
    T g0 = A.g2[e], g1 = T(0);
    auto step = [&](int64_t x, const uint32_t pn, const T g, uint32_t &pn_next, T &g_next) {
        const int mode = static_cast<int>(pn & 7u);
        const int p = static_cast<int>(pn >> 3);
        const StateRec<T> sp = A.st[p];
        const T fp = f[p];
        int64_t iq, im;
        if (A.padq) {
            iq = static_cast<int64_t>(static_cast<int>(sp.kqp - sd.kqp) + A.qoff);
            im = 2 * static_cast<int64_t>(A.qoff) - iq;
        } else {
            iq = q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
            im = q_linear(sp.kq, sd.kq, A.nq0, A.nq1, A.nq2);
        }
        const Vec4<T> t1 = tab[iq * A.nm + mode], t2 = tab[im * A.nm + mode];
        __builtin_amdgcn_sched_barrier(0);
        pn_next = A.pnu[x + stride];
        g_next = A.g2[x + stride];
        __builtin_amdgcn_sched_barrier(0);
        const T gm = keep_or_zero(g, x < end && !((elastic >> mode) & 1u));
        const T xe = sd.eps - sp.eps;
        const T ga = stream_gauss(A, (xe + t1.x) * (xe + t1.x), s_tab);
        const T ge = stream_gauss(A, (xe - t2.x) * (xe - t2.x), s_tab);
        acc[0] += gm * (t2.z * ge * (t2.y + T(1) - fp) - t1.z * ga * (t1.y + fp));
    };
    for (; e < end; e += 2 * stride) {
        step(e, pn0, g0, pn1, g1);
        if (e + stride >= end) break;
        step(e + stride, pn1, g1, pn0, g0);
    }
    block_sum<T, 1>(acc);
    if (threadIdx.x == 0) {
        const T v = static_cast<T>(Kp) * acc[0];
        if (A.dest_chunk[d + 1] - A.dest_chunk[d] == 1) out[d] += v;
        else part[c] = v;
    }
}

template <typename T>
__global__ void k_vjp_phonon_f_finish(TiledArgs<T> A, const T *__restrict__ part, T *__restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    const int c0 = A.dest_chunk[d], c1 = A.dest_chunk[d + 1];
    if (c1 - c0 == 1) return;
    T a = T(0);
    for (int c = c0; c < c1; ++c) a += part[c];
    out[d] += a;
}

// The same over pair records when every tile of the pair pass is q-ordered.
// A lane takes one pair (d, p) with all its modes; seen from p, q and -q swap
// roles and x = e_d - e_p changes sign, so the channel's two Gaussians
// ga = G(x + hw(q)) and ge = G(x - hw(-q)) serve both states:
//   dL/df_d += Kp |g|^2 [mu(-q) ge (N(-q) + 1 - f_p) - mu(q) ga (N(q) + f_p)]
//   dL/df_p += Kp |g|^2 [mu(q) ga (N(q) + 1 - f_d) - mu(-q) ge (N(-q) + f_d)]
// Each channel is read once and the lanes of a batch share the table rows of
// their q.  Both sides are fixed-point LDS sums on the scale of vjp_scale
// (max |mu| in place of max |lambda|), flushed to the global accumulator;
// k_vjp_phonon_pairs_finish adds them to out.  A slot without a channel (or
// of an elastic mode) is masked after its product, since its N may be
// infinite (acoustic modes at q = 0).
template <typename T, bool PADQ, int NM>
__global__ __launch_bounds__(1024) void k_vjp_phonon_pairs(TiledArgs<T> A, const Vec4<T> *__restrict__ tab,
                                                          const T *__restrict__ f, uint32_t elastic,
                                                          const unsigned long long *__restrict__ mmax_bits) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t ti = tile_of_block(A.n_tiles, A.xcd);
    if (ti < 0) return;
    const TileRec t = A.tiles[ti];
    unsigned long long *s_j = reinterpret_cast<unsigned long long *>(smem);
    Pair2<T> *s_ef = reinterpret_cast<Pair2<T> *>(s_j + A.lds_states);
    uint32_t *s_kq = reinterpret_cast<uint32_t *>(s_ef + A.lds_states);
    double *s_tab = reinterpret_cast<double *>(s_kq + A.lds_states);
    const int n = t.p_hi - t.p_lo + 1;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const StateRec<T> sr = A.st[t.p_lo + i];
        Pair2<T> ef;
        ef.a = sr.eps;
        ef.b = f[t.p_lo + i];
        s_ef[i] = ef;
        s_kq[i] = PADQ ? sr.kqp : sr.kq;
        s_j[i] = 0ull;
    }
    if constexpr (sizeof(T) == 8)
        for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_tab[i] = A.e2tab[i];
    const T scale = static_cast<T>(vjp_scale(A.nmax_bits, A.gmax_bits, mmax_bits, A.fmax_bits));
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nw = static_cast<int>(blockDim.x >> 6);
    const int nm = A.nm;
    for (int64_t c = t.c0 + wave; c < t.c1; c += nw) {
        const int64_t beg = A.chunk_beg[c];
        const int len = static_cast<int>(A.chunk_end[c] - beg);
        const uint32_t *__restrict__ pb = A.pnu + beg;
        const T *__restrict__ gb = A.g2 + beg;
        for (int r = 0; r < len; r += 64) {
            const bool v = r + lane < len;
            const uint32_t pn = pb[r + lane];
            // a masked lane takes window slot 0 as both states and adds nothing
            const int wd = v ? static_cast<int>(pn & 0xffffu) : 0;
            const int wp = v ? static_cast<int>(pn >> 16) : 0;
            const Pair2<T> efd = s_ef[wd], efp = s_ef[wp];
            const uint32_t kd = s_kq[wd], kp = s_kq[wp];
            int64_t iq, im;
            if (PADQ) {
                iq = static_cast<int64_t>(static_cast<int>(kp - kd) + A.qoff);
                im = 2 * static_cast<int64_t>(A.qoff) - iq;
            } else {
                iq = q_linear(kd, kp, A.nq0, A.nq1, A.nq2);
                im = q_linear(kp, kd, A.nq0, A.nq1, A.nq2);
            }
            const T x = efd.a - efp.a, fd = efd.b, fp = efp.b;
            T sd = T(0), sp = T(0);
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                const int mm = min(m, nm - 1);
                const Vec4<T> t1 = tab[iq * nm + mm], t2 = tab[im * nm + mm];
                const T g = gb[mm * A.pld + r + lane];
                const bool on = v && m < nm && !((elastic >> m) & 1u) && g != T(0);
                const T ga = stream_gauss(A, (x + t1.x) * (x + t1.x), s_tab);
                const T ge = stream_gauss(A, (x - t2.x) * (x - t2.x), s_tab);
                const T a1 = t1.z * ga, a2 = t2.z * ge;
                sd += keep_or_zero(g * (a2 * (t2.y + T(1) - fp) - a1 * (t1.y + fp)), on);
                sp += keep_or_zero(g * (a1 * (t1.y + T(1) - fd) - a2 * (t2.y + fd)), on);
            }
            if (v) {
                atomicAdd(s_j + wd, to_fixed(__builtin_rint(sd * scale)));
                atomicAdd(s_j + wp, to_fixed(__builtin_rint(sp * scale)));
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long u = s_j[i];
        if (u) atomicAdd(A.jacc + t.p_lo + i, u);
    }
}

// out[d] += Kp (the fixed-point sum of d) / scale; the accumulator of d is
// cleared for the next call
template <typename T>
__global__ void k_vjp_phonon_pairs_finish(TiledArgs<T> A, const unsigned long long *__restrict__ mmax_bits,
                                          double Kp, T *__restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.S) return;
    const double inv = 1.0 / vjp_scale(A.nmax_bits, A.gmax_bits, mmax_bits, A.fmax_bits);
    const long long j = static_cast<long long>(A.jacc[d]);
    A.jacc[d] = 0ull;
    out[d] += static_cast<T>(Kp * static_cast<double>(j) * inv);
}

// out = x (mode 0) or out = (x(q) + x(-q)) / 2 per (q, mode) (mode 1): the
// even part in q, which is its own transpose
template <typename T>
__global__ void k_even_q(const T *__restrict__ x, T *__restrict__ out, int n0, int n1, int n2, int nm) {
    const int64_t n = static_cast<int64_t>(n0) * n1 * n2 * nm;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t q = i / nm;
        const int nu = static_cast<int>(i - q * nm);
        const int a2 = static_cast<int>(q % n2), a1 = static_cast<int>((q / n2) % n1),
                  a0 = static_cast<int>(q / (static_cast<int64_t>(n1) * n2));
        const int64_t qm = (static_cast<int64_t>((n0 - a0) % n0) * n1 + (n1 - a1) % n1) * n2 + (n2 - a2) % n2;
        out[i] = T(0.5) * (x[i] + x[qm * nm + nu]);
    }
}

// out = a x + b y (y may be null: out = a x)
template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *__restrict__ x, T b, const T *__restrict__ y, T *__restrict__ out) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// dst[b][d] = -src[b][d] for B rows of S values (row strides lds, ldd; dst may
// be src)
template <typename T>
__global__ void k_neg_rows(const T *src, int64_t lds, T *dst, int64_t ldd, int B, int S) {
    const int64_t n = static_cast<int64_t>(B) * S;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t b = i / S, d = i - b * S;
        dst[b * ldd + d] = -src[b * lds + d];
    }
}

// |g|^2 slots of the pair records from the caller's list (update_g2)
template <typename T>
__global__ void k_ph_gather_g2(const int32_t *__restrict__ chan, const double *__restrict__ g2,
                               T *__restrict__ out, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t c = chan[i];
        out[i] = c >= 0 ? static_cast<T>(g2[c]) : T(0);
    }
}

// dN(q, nu) = Kp (sum over the chunks of q's bucket of q's side, in chunk
// order; both sides when q = -q), 0 for bins without channels.
template <typename T>
__global__ void k_phonon_bins_finish(PhArgs<T> A, const T *__restrict__ part, T *__restrict__ out) {
    const int64_t n = A.nq * A.nm;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t q = i / A.nm;
        const int m = static_cast<int>(i - q * A.nm);
        const int qb = A.q_bucket[q];
        T sum = T(0);
        if (qb >= 0) {
            const int bk = qb >> 1, side = qb & 1;
            const int c0 = A.bucket_chunk[bk], c1 = A.bucket_chunk[bk + 1];
            for (int c = c0; c < c1; ++c) sum += part[(static_cast<int64_t>(c) * 2 + side) * A.nm + m];
            if (A.bucket_q[bk] == A.bucket_qm[bk])
                for (int c = c0; c < c1; ++c) sum += part[(static_cast<int64_t>(c) * 2 + 1) * A.nm + m];
        }
        out[i] = static_cast<T>(A.Kp * static_cast<double>(sum));
    }
}

// max |x| over x[0..n) as the bits of a non-negative double (integer order of
// such bits is their numeric order, so the atomic max is order-independent)
template <typename T>
__global__ __launch_bounds__(256) void k_abs_max_bits(const T *__restrict__ x, int64_t n,
                                                      unsigned long long *out) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(static_cast<double>(x[i])));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(m)));
}

// Pair records in a new order: slot m of position i takes slot m of position
// idx[i] (|g|^2 and channel), and so does the first-channel array; positions
// np .. ld - 1 get the padding values (|g|^2 0, channel -1).  idx[i] < np.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_pairs(const uint32_t *__restrict__ idx, int64_t np, int64_t ld,
                                                       int nm, const T *__restrict__ g_in, T *__restrict__ g_out,
                                                       const int32_t *__restrict__ c_in, int32_t *__restrict__ c_out,
                                                       const int32_t *__restrict__ c0_in,
                                                       int32_t *__restrict__ c0_out) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < ld;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool in = i < np;
        const int64_t j = in ? static_cast<int64_t>(idx[i]) : 0;
        for (int m = 0; m < nm; ++m) {
            g_out[m * ld + i] = in ? g_in[m * ld + j] : T(0);
            c_out[m * ld + i] = in ? c_in[m * ld + j] : -1;
        }
        c0_out[i] = in ? c0_in[j] : -1;
    }
}

// ---- transport ----------------------------------------------------------
// Linearisation at f0: per entry W_dp = K g2 [da (N + 1 - f0_d) + de (N + f0_d)]
// is stored; 1/tau_d = K sum g2 [da (N + f0_p) + de (N + 1 - f0_p)].
template <typename T, bool FUSED>
__global__ __launch_bounds__(512) void k_transport_setup(Tables<T> P, const T *__restrict__ f0,
                                                         T *__restrict__ W, T *__restrict__ part,
                                                         T *__restrict__ tau_inv) {
    const int64_t c = chunk_of_block(P.n_chunks, P.xcd_m);
    if (c >= P.n_chunks) return;
    const int d = P.chunk_dest[c];
    const int64_t beg = P.chunk_beg[c], end = P.chunk_beg[c + 1];
    const StateRec<T> sd = P.st[d];
    const T fd = f0[d];
    T acc[1] = {T(0)};
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const uint32_t pn = P.pnu[e];
        const T g = P.g2[e];
        const int p = static_cast<int>(pn >> 3);
        const StateRec<T> sp = P.st[p];
        const T fp = f0[p];
        EntryCoef<T> k = entry_coef(P, sd.eps, sd.kq, pn, sp);
        // ah = N(da+de) + de, bh = N(da+de) + da
        // W  = g [ (N(da+de) + da) - f0_d (da - de) ]  = g [bh - f0_d (da - de)]
        // out= g [ (N(da+de) + de) + f0_p (da - de) ]  = g [ah + f0_p (da - de)]
        const T dd = k.bh - k.ah;   // da - de
        W[e] = P.K * g * (k.bh - fd * dd);
        acc[0] += g * (k.ah + fp * dd);
    }
    block_sum<T, 1>(acc);
    if (threadIdx.x == 0) {
        if (FUSED) tau_inv[d] = P.K * acc[0];
        else part[c] = acc[0];
    }
}

template <typename T>
__global__ void k_transport_setup_finish(Tables<T> P, const T *__restrict__ part,
                                         T *__restrict__ tau_inv) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= P.S) return;
    T a = T(0);
    for (int c = P.dest_chunk[d]; c < P.dest_chunk[d + 1]; ++c) a += part[c];
    tau_inv[d] = P.K * a;
}

}  // namespace ephbte
