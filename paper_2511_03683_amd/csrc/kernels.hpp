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
// shuffle tree and waves through LDS in fixed order.  No atomics anywhere.
//
// Entry algebra (Eq. 2 with the golden-rule occupation factors).  With
// da = exp(-(e_d - e_p + hw)^2 / 2 s^2), de = exp(-(e_d - e_p - hw)^2 / 2 s^2),
// t = N (da + de):
//   a = g2 (t + de)  (weight of the out-scattering product f_d (1 - f_p))
//   b = g2 (t + da)  (weight of the in-scattering product  f_p (1 - f_d))
// and I_d = K [ (1 - f_d) sum b f_p  -  f_d sum a (1 - f_p) ] with
// K = 2 pi / (hbar N_q) / (s sqrt(2 pi)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ephbte {

template <typename T> struct StateRec;
template <> struct alignas(16) StateRec<double> {
    double eps;
    uint32_t kq;
    uint32_t pad;
};
template <> struct alignas(8) StateRec<float> {
    float eps;
    uint32_t kq;
};

// exp of the (pre-scaled) Gaussian exponent: FP64 uses the accurate libm
// exp; FP32 uses the hardware base-2 exponential with the log2(e) factor
// folded into the exponent scale on the host.
__device__ __forceinline__ double gauss_exp(double a) { return exp(a); }
__device__ __forceinline__ float gauss_exp(float a) { return __builtin_amdgcn_exp2f(a); }

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
    T mc;   // Gaussian exponent scale (FP64: -1/(2 s^2); FP32: -log2(e)/(2 s^2))
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
};

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

// ---- forward: I[f] -------------------------------------------------------
// FUSED: one chunk per destination, the workgroup applies the epilogue.
// Otherwise the two sums of each chunk go to part[b][chunk][2].
template <typename T, bool FUSED>
__global__ __launch_bounds__(512) void k_collision(Tables<T> P, const T *__restrict__ f,
                                                   int64_t ldf, T *__restrict__ part, Epi<T> E) {
    const int64_t c = chunk_of_block(P.n_chunks, P.xcd_m);
    if (c >= P.n_chunks) return;
    const int b = blockIdx.y;
    const T *fb = f + static_cast<int64_t>(b) * ldf;
    const int d = P.chunk_dest[c];
    const int64_t beg = P.chunk_beg[c], end = P.chunk_beg[c + 1];
    const StateRec<T> sd = P.st[d];
    T acc[2] = {T(0), T(0)};   // sum a (1 - f_p), sum b f_p
    const int stride = blockDim.x;
    int64_t e = beg + threadIdx.x;
    for (; e + 3 * stride < end; e += 4 * stride) {
        uint32_t pn[4];
        T g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pn[u] = P.pnu[e + u * stride];
            g[u] = P.g2[e + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = static_cast<int>(pn[u] >> 3);
            const StateRec<T> sp = P.st[p];
            const T fp = fb[p];
            EntryCoef<T> k = entry_coef(P, sd.eps, sd.kq, pn[u], sp);
            acc[0] += g[u] * k.ah * (T(1) - fp);
            acc[1] += g[u] * k.bh * fp;
        }
    }
    for (; e < end; e += stride) {
        const uint32_t pn = P.pnu[e];
        const T g = P.g2[e];
        const int p = static_cast<int>(pn >> 3);
        const StateRec<T> sp = P.st[p];
        const T fp = fb[p];
        EntryCoef<T> k = entry_coef(P, sd.eps, sd.kq, pn, sp);
        acc[0] += g * k.ah * (T(1) - fp);
        acc[1] += g * k.bh * fp;
    }
    block_sum<T, 2>(acc);
    if (threadIdx.x == 0) {
        if (FUSED) {
            const T fd = fb[d];
            apply_epi(E, b, d, P.S, P.K * ((T(1) - fd) * acc[1] - fd * acc[0]));
        } else {
            T *pp = part + (static_cast<int64_t>(b) * P.n_chunks + c) * 2;
            pp[0] = acc[0];
            pp[1] = acc[1];
        }
    }
}

template <typename T>
__global__ void k_collision_finish(Tables<T> P, const T *__restrict__ f, int64_t ldf,
                                   const T *__restrict__ part, Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= P.S) return;
    const int b = blockIdx.y;
    T a = T(0), bb = T(0);
    const T *pb = part + static_cast<int64_t>(b) * P.n_chunks * 2;
    for (int c = P.dest_chunk[d]; c < P.dest_chunk[d + 1]; ++c) {
        a += pb[2 * c];
        bb += pb[2 * c + 1];
    }
    const T fd = f[static_cast<int64_t>(b) * ldf + d];
    apply_epi(E, b, d, P.S, P.K * ((T(1) - fd) * bb - fd * a));
}

// ---- reverse: dL/df and dL/d|g|^2 ---------------------------------------
// dL/df_d = -K sum_entries (lam_d - lam_p) (a (1 - f_p) + b f_p)
// dL/dg2_c = K (lam_d - lam_p) (bh f_p (1 - f_d) - ah f_d (1 - f_p)), written by
// the entry with p > d (each channel has exactly one such entry).
template <typename T, bool FUSED>
__global__ __launch_bounds__(512) void k_collision_vjp(Tables<T> P, const T *__restrict__ f,
                                                       int64_t ldf, const T *__restrict__ lam,
                                                       int64_t ldl, T *__restrict__ part, Epi<T> E,
                                                       double *__restrict__ gg2, int gg2_mode) {
    const int64_t c = chunk_of_block(P.n_chunks, P.xcd_m);
    if (c >= P.n_chunks) return;
    const int b = blockIdx.y;
    const T *fb = f + static_cast<int64_t>(b) * ldf;
    const T *lb = lam + static_cast<int64_t>(b) * ldl;
    const int d = P.chunk_dest[c];
    const int64_t beg = P.chunk_beg[c], end = P.chunk_beg[c + 1];
    const StateRec<T> sd = P.st[d];
    const T fd = fb[d];
    const T ld = lb[d];
    T acc[1] = {T(0)};
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const uint32_t pn = P.pnu[e];
        const T g = P.g2[e];
        const int p = static_cast<int>(pn >> 3);
        const StateRec<T> sp = P.st[p];
        const T fp = fb[p];
        const T dl = ld - lb[p];
        EntryCoef<T> k = entry_coef(P, sd.eps, sd.kq, pn, sp);
        acc[0] += dl * g * (k.ah * (T(1) - fp) + k.bh * fp);
        if (gg2_mode && p > d) {
            const double v = static_cast<double>(P.K * dl * (k.bh * fp * (T(1) - fd) - k.ah * fd * (T(1) - fp)));
            double *o = gg2 + P.ent_chan[e];
            *o = (gg2_mode == 2) ? (*o + v) : v;
        }
    }
    if (E.mode < 0) return;   // |g|^2 gradient only
    block_sum<T, 1>(acc);
    if (threadIdx.x == 0) {
        if (FUSED) {
            apply_epi(E, b, d, P.S, -P.K * acc[0]);
        } else {
            part[static_cast<int64_t>(b) * P.n_chunks + c] = acc[0];
        }
    }
}

template <typename T>
__global__ void k_vjp_finish(Tables<T> P, const T *__restrict__ part, Epi<T> E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= P.S) return;
    const int b = blockIdx.y;
    T a = T(0);
    const T *pb = part + static_cast<int64_t>(b) * P.n_chunks;
    for (int c = P.dest_chunk[d]; c < P.dest_chunk[d + 1]; ++c) a += pb[c];
    apply_epi(E, b, d, P.S, -P.K * a);
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

template <typename T> struct alignas(4 * sizeof(T)) Vec4 {
    T x, y, z, w;
};

// x_new_d = tau_d (b_d + sum W_dp x_p), three field directions at once.
template <typename T, bool FUSED>
__global__ __launch_bounds__(512) void k_transport_iter(Tables<T> P, const T *__restrict__ W,
                                                        const Vec4<T> *__restrict__ x,
                                                        const Vec4<T> *__restrict__ rhs,
                                                        const T *__restrict__ tau,
                                                        Vec4<T> *__restrict__ part,
                                                        Vec4<T> *__restrict__ x_new) {
    const int64_t c = chunk_of_block(P.n_chunks, P.xcd_m);
    if (c >= P.n_chunks) return;
    const int d = P.chunk_dest[c];
    const int64_t beg = P.chunk_beg[c], end = P.chunk_beg[c + 1];
    T acc[3] = {T(0), T(0), T(0)};
    for (int64_t e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const int p = static_cast<int>(P.pnu[e] >> 3);
        const T w = W[e];
        const Vec4<T> xp = x[p];
        acc[0] += w * xp.x;
        acc[1] += w * xp.y;
        acc[2] += w * xp.z;
    }
    block_sum<T, 3>(acc);
    if (threadIdx.x == 0) {
        if (FUSED) {
            const Vec4<T> r = rhs[d];
            const T t = tau[d];
            Vec4<T> o;
            o.x = t * (r.x + acc[0]);
            o.y = t * (r.y + acc[1]);
            o.z = t * (r.z + acc[2]);
            o.w = T(0);
            x_new[d] = o;
        } else {
            Vec4<T> o;
            o.x = acc[0];
            o.y = acc[1];
            o.z = acc[2];
            o.w = T(0);
            part[c] = o;
        }
    }
}

template <typename T>
__global__ void k_transport_iter_finish(Tables<T> P, const Vec4<T> *__restrict__ part,
                                        const Vec4<T> *__restrict__ rhs, const T *__restrict__ tau,
                                        Vec4<T> *__restrict__ x_new) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= P.S) return;
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int c = P.dest_chunk[d]; c < P.dest_chunk[d + 1]; ++c) {
        a0 += part[c].x;
        a1 += part[c].y;
        a2 += part[c].z;
    }
    const Vec4<T> r = rhs[d];
    const T t = tau[d];
    Vec4<T> o;
    o.x = t * (r.x + a0);
    o.y = t * (r.y + a1);
    o.z = t * (r.z + a2);
    o.w = T(0);
    x_new[d] = o;
}

}  // namespace ephbte
