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
// kqp: the same k as a linear index on a grid padded to (2 Nq0, 2 Nq1, 2 Nq2),
//      so that kqp_p - kqp_d + offset is the padded index of q = k_p - k_d
//      (each axis difference + Nq lies in [1, 2 Nq), so no borrow crosses axes)
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
    const Pair2<T> *__restrict__ hwN;   // [Nq * n_modes] {hw, N}
    const int64_t *__restrict__ chunk_beg;
    const int32_t *__restrict__ chunk_dest;
    const int32_t *__restrict__ dest_chunk;
    const TileRec *__restrict__ tiles;
    int64_t n_chunks;
    int S, nm, nq0, nq1, nq2, lds_states;
    int padq;          // 1: hwN is the padded table indexed by kqp differences
    int qoff;          // padded index of q = 0 difference
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
};

// ---- fixed point for the partner side of the single-copy pass -------------
// Contributions to I_p (p > d) arrive from many rows; they are rounded to
// integers on a common scale 2^s and summed with integer atomics, which are
// associative, so the sums do not depend on the order of arrival.  With
// |N| <= N_max, f in [0, 1] and the Gaussians <= 1, one entry's share is at
// most |g|^2 (2 N_max + 1), a state's column at most (2 N_max + 1) G_max with
// G_max the largest sum of |g|^2 over one state's channels; s puts that bound
// below 2^61.
__device__ __forceinline__ double sym_scale(const unsigned long long *nmax_bits,
                                            const unsigned long long *gmax_bits) {
    const double nmax = __longlong_as_double(static_cast<long long>(*nmax_bits));
    const double gmax = __longlong_as_double(static_cast<long long>(*gmax_bits));
    const double bound = (2.0 * nmax + 1.0) * gmax;
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

// Padded table: entry (qp, nu) holds {hw, N} of q = (c - Nq) mod Nq per axis,
// where c are the axis coordinates of qp on the (2 Nq0, 2 Nq1, 2 Nq2) grid.
// The modes of one q are contiguous, so partners at neighbouring k (consecutive
// q along the last axis) read neighbouring table bytes.
template <typename T>
__global__ void k_pack_hwN_pad(const T *__restrict__ hw, const T *__restrict__ nph,
                               Pair2<T> *__restrict__ out, int n0, int n1, int n2, int nm,
                               int64_t n, double *bmax) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int nu = static_cast<int>(i % nm);
        int64_t qp = i / nm;
        const int c2 = static_cast<int>(qp % (2 * n2));
        qp /= 2 * n2;
        const int c1 = static_cast<int>(qp % (2 * n1));
        const int c0 = static_cast<int>(qp / (2 * n1));
        int a0 = c0 - n0, a1 = c1 - n1, a2 = c2 - n2;
        a0 += a0 < 0 ? n0 : 0;
        a1 += a1 < 0 ? n1 : 0;
        a2 += a2 < 0 ? n2 : 0;
        const int64_t q = (static_cast<int64_t>(a0) * n1 + a1) * n2 + a2;
        Pair2<T> v;
        v.a = hw[q * nm + nu];
        v.b = nph[q * nm + nu];
        out[i] = v;
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
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.nm + (pn[u] & 7u)];
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
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.nm + (pn[u] & 7u)];
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
    const T scale = static_cast<T>(sym_scale(A.nmax_bits, A.gmax_bits));
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
    const double inv = 1.0 / sym_scale(A.nmax_bits, A.gmax_bits);
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
            const Pair2<T> w = A.hwN[static_cast<int64_t>(q) * A.nm + (pn[u] & 7u)];
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

template <typename T, int DPW>
__global__ __launch_bounds__(512) void k_fwd_batched(BArgs<T> A, const T *__restrict__ f,
                                                     int64_t ldf, int B, Epi<T> E) {
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
                for (int64_t e0 = e_lo; e0 < e_hi; e0 += 64) {
                    const int64_t e = e0 + lane;
                    const bool valid = e < e_hi;
                    int pl = -1 - lane;     // distinct for invalid lanes: never merged
                    T ca = T(0), cb = T(0);
                    if (valid) {
                        const uint32_t pn = A.pnu[e];
                        const T g = A.g2[e];
                        pl = static_cast<int>(pn >> 3) - pa;
                        const StateRec<T> sp = s_ek[pl];
                        const int q = A.padq ? static_cast<int>(sp.kqp - sd.kqp) + A.qoff
                                             : q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
                        const Pair2<T> wn = A.hwN[static_cast<int64_t>(q) * A.nm + (pn & 7u)];
                        const T de = sd.eps - sp.eps;
                        const T xa = de + wn.a, xe = de - wn.a;
                        const T da = gauss_exp(xa * xa * A.mc);
                        const T dem = gauss_exp(xe * xe * A.mc);
                        const T tt = wn.b * (da + dem);
                        ca = g * (tt + dem);
                        cb = g * (tt + da);
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
                    while (m) {
                        const int src = __builtin_ctzll(m);
                        m &= m - 1;
                        const T a = lane_bcast(ca, src);
                        const T bq = lane_bcast(cb, src);
                        const int pls = __builtin_amdgcn_readlane(pl, src);
                        const T fpb = s_F[pls * 65 + lane];
                        acc_a[j] += a * (T(1) - fpb);
                        acc_b[j] += bq * fpb;
                    }
                }
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
template <typename T, int DPW>
__global__ __launch_bounds__(512) void k_vjp_batched(BArgs<T> A, const T *__restrict__ f, int64_t ldf,
                                                     const T *__restrict__ lam, int64_t ldl, int b0,
                                                     int nb, T *__restrict__ gf, int64_t ldgf,
                                                     const int32_t *__restrict__ ent_chan,
                                                     double *__restrict__ gg2, int gg2_mode) {
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
                for (int64_t e0 = e_lo; e0 < e_hi; e0 += 64) {
                    const int64_t e = e0 + lane;
                    const bool valid = e < e_hi;
                    int pl = -1 - lane;     // distinct for invalid lanes: never merged
                    T ca = T(0), cb = T(0), ah = T(0), bh = T(0);
                    int32_t ch = -1;
                    if (valid) {
                        const uint32_t pn = A.pnu[e];
                        const T g = A.g2[e];
                        pl = static_cast<int>(pn >> 3) - pa;
                        const StateRec<T> sp = s_ek[pl];
                        const int q = A.padq ? static_cast<int>(sp.kqp - sd.kqp) + A.qoff
                                             : q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
                        const Pair2<T> wn = A.hwN[static_cast<int64_t>(q) * A.nm + (pn & 7u)];
                        const T de = sd.eps - sp.eps;
                        const T xa = de + wn.a, xe = de - wn.a;
                        const T da = gauss_exp(xa * xa * A.mc);
                        const T dem = gauss_exp(xe * xe * A.mc);
                        const T tt = wn.b * (da + dem);
                        ah = tt + dem;
                        bh = tt + da;
                        ca = g * ah;
                        cb = g * bh;
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
                    while (m) {
                        const int src = __builtin_ctzll(m);
                        m &= m - 1;
                        const T a = lane_bcast(ca, src);
                        const T bq = lane_bcast(cb, src);
                        const int pls = __builtin_amdgcn_readlane(pl, src);
                        const Pair2<T> fl = s_FL[pls * 65 + lane];
                        const T u = a + (bq - a) * fl.a;
                        acc_u[j] += u;
                        acc_l[j] += fl.b * u;
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
// Each entry (d, p, nu) carries the processes that create or destroy phonon
// (nu, q = k_p - k_d): d -> p absorbing it and p -> d emitting it, both with
// the delta G(e_d - e_p + hw).  Its net emission, |g|^2 Ga [(N+1) f_p (1 - f_d)
// - N f_d (1 - f_p)], is rounded to fixed point on the scale of sym_scale with
// the bound phb (largest entry count of a bin times max |g|^2) and added to the
// bin with an integer atomic, so each bin's sum does not depend on the order.
// Entries of elastic mechanisms (bit nu of elastic) have no phonon: skipped.
template <typename T>
__global__ __launch_bounds__(256) void k_phonon_rate(TiledArgs<T> A, const T *__restrict__ f,
                                                     uint32_t elastic,
                                                     const unsigned long long *__restrict__ phb_bits,
                                                     unsigned long long *__restrict__ bins) {
    const int64_t c = blockIdx.x;
    if (c >= A.n_chunks) return;
    const int d = A.chunk_dest[c];
    const int64_t beg = A.chunk_beg[c], end = A.chunk_beg[c + 1];
    const StateRec<T> sd = A.st[d];
    const T fd = f[d];
    const T scale = static_cast<T>(sym_scale(A.nmax_bits, phb_bits));
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const uint32_t pn = A.pnu[e];
        const int mode = static_cast<int>(pn & 7u);
        if ((elastic >> mode) & 1u) continue;
        const int p = static_cast<int>(pn >> 3);
        const StateRec<T> sp = A.st[p];
        const int ql = q_linear(sd.kq, sp.kq, A.nq0, A.nq1, A.nq2);
        const int qi = A.padq ? static_cast<int>(sp.kqp - sd.kqp) + A.qoff : ql;
        const Pair2<T> wn = A.hwN[static_cast<int64_t>(qi) * A.nm + mode];
        const T xa = (sd.eps - sp.eps) + wn.a;
        const T da = gauss_exp(xa * xa * A.mc);
        const T fp = f[p];
        const T y = A.g2[e] * da * ((wn.b + T(1)) * fp * (T(1) - fd) - wn.b * fd * (T(1) - fp));
        const unsigned long long v = to_fixed(__builtin_rint(y * scale));
        atomicAdd(bins + static_cast<int64_t>(ql) * A.nm + mode, v);
    }
}

// dN = Kp sum of the bin (Kp = 2 pi / (hbar N_k) / (sigma sqrt(2 pi))); clears the bins.
template <typename T>
__global__ void k_phonon_finish(unsigned long long *__restrict__ bins, int64_t n,
                                const unsigned long long *__restrict__ nmax_bits,
                                const unsigned long long *__restrict__ phb_bits, double Kp,
                                T *__restrict__ out) {
    const double inv = 1.0 / sym_scale(nmax_bits, phb_bits);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const long long v = static_cast<long long>(bins[i]);
        bins[i] = 0ull;
        out[i] = static_cast<T>(Kp * (static_cast<double>(v) * inv));
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

// phb = count * max |g|^2 (the per-bin bound of the phonon-side sums)
__global__ void k_phonon_bound(const unsigned long long *__restrict__ gmax_bits, double count,
                               unsigned long long *__restrict__ phb_bits) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double g = __longlong_as_double(static_cast<long long>(*gmax_bits));
        *phb_bits = static_cast<unsigned long long>(__double_as_longlong(count * g));
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
