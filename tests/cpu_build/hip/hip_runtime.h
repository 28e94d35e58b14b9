// A CPU stand-in for the HIP runtime and device built-ins, so that the
// library's kernels and host code compile with g++ and run under
// AddressSanitizer (test infrastructure; never part of the library).
//
// Kernels run one workgroup at a time.  Each work-item is a fiber on one OS
// thread (x86-64 register switch, announced to ASan as a fiber switch); a
// fiber runs until it reaches __syncthreads, a cross-lane exchange
// (shuffle, ballot, readlane, DPP) or its end.  An exchange completes when
// every live lane of the wave has reached it, a barrier when every live
// work-item of the block has.  Device memory is host memory from
// aligned_alloc, so every out-of-range access of a kernel is an ASan report;
// dynamic LDS is one 160 KB buffer whose part beyond the launch's size is
// poisoned, and it starts each block filled with 0xFF bytes (LDS is not
// cleared on the GPU either).  Only what the library uses is provided.
#pragma once
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <functional>
#include <numeric>
#include <memory>
#include <mutex>
#include <sys/mman.h>
#include <tuple>
#include <vector>
#include <sanitizer/asan_interface.h>

struct alignas(16) double2 {
    double x, y;
};
inline double2 make_double2(double a, double b) { return double2{a, b}; }

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {
struct Wave {
    uint64_t buf[64];
    bool alive[64];
    int n;
};
struct Ctx {
    dim3 tid, bid, bdim, gdim;
    Wave *wave = nullptr;
    int lane = 0;
};
inline Ctx ctx;
constexpr size_t kLds = 160 * 1024;
alignas(256) inline unsigned char lds[kLds];
inline unsigned char *dyn_smem() { return lds; }
inline long long n_launch = 0, n_blocks = 0;
inline bool verbose = false;
// fibers of one block; a fiber runs until it reaches a barrier or exits
enum { RUN = 0, AT_BLOCK = 1, AT_WAVE = 2, DONE = 3 };
struct Fiber { void *sp; int state; };
struct Block {
    int nt = 0, cur = 0;
    std::vector<Fiber> f;
    void *sched_sp = nullptr;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
};
inline Block blk;
extern "C" void emu_switch(void **save_sp, void *to_sp);
// saves the callee-saved registers on the current stack, stores its pointer
// in *save_sp, continues on to_sp (a stack saved the same way)
asm(R"(
    .text
    .globl emu_switch
    .type emu_switch, @function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_switch, .-emu_switch
)");
inline void wait_at(int st) {
    Fiber &me = blk.f[blk.cur];
    me.state = st;
    void *fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, blk.sched_bottom, blk.sched_size);
    emu_switch(&me.sp, blk.sched_sp);
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}
template <class T> T xchg(T v, int src) {
    Wave &w = *ctx.wave;
    const int lane = ctx.lane;
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    w.buf[lane] = bits;
    wait_at(AT_WAVE);
    if (src < 0 || src >= w.n) { fprintf(stderr, "cpu build: shuffle source lane %d of %d\n", src, w.n); abort(); }
    const uint64_t r = w.buf[src];
    wait_at(AT_WAVE);
    T out;
    std::memcpy(&out, &r, sizeof(T));
    return out;
}
}  // namespace emu

#define threadIdx (emu::ctx.tid)
#define blockIdx (emu::ctx.bid)
#define blockDim (emu::ctx.bdim)
#define gridDim (emu::ctx.gdim)
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) alignas(n)
#define __shared__ static

inline void __syncthreads() { emu::wait_at(emu::AT_BLOCK); }
template <class T> T __shfl_xor(T v, int m, int w = 64) { (void)w; return emu::xchg(v, emu::ctx.lane ^ m); }
template <class T> T __shfl_down(T v, unsigned d, int w = 64) {
    (void)w; int s = emu::ctx.lane + int(d); if (s >= emu::ctx.wave->n) s = emu::ctx.lane; return emu::xchg(v, s);
}
template <class T> T __shfl_up(T v, unsigned d, int w = 64) {
    (void)w; int s = emu::ctx.lane - int(d); if (s < 0) s = emu::ctx.lane; return emu::xchg(v, s);
}
template <class T> T __shfl(T v, int src, int w = 64) { (void)w; return emu::xchg(v, src); }
inline unsigned long long __ballot(int p) {
    emu::Wave &w = *emu::ctx.wave;
    w.buf[emu::ctx.lane] = p ? 1 : 0;
    emu::wait_at(emu::AT_WAVE);
    unsigned long long m = 0;
    for (int l = 0; l < w.n; ++l) if (w.alive[l] && w.buf[l]) m |= 1ull << l;
    emu::wait_at(emu::AT_WAVE);
    return m;
}
#define __builtin_amdgcn_readfirstlane(x) (x)
inline int __builtin_amdgcn_readlane(int v, int src) { return emu::xchg(v, src); }
inline float __builtin_amdgcn_exp2f(float x) { return exp2f(x); }
inline void __builtin_amdgcn_sched_barrier(int) {}
// raw buffer resources: base, size in bytes; loads past the size return 0
struct __amdgpu_buffer_rsrc_t {
    const unsigned char *base;
    int num;
};
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void *p, short, int num, int) {
    return {static_cast<const unsigned char *>(p), num};
}
inline unsigned long long __builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t r, int voff, int soff, int) {
    const long long o = static_cast<long long>(voff) + soff;
    unsigned long long v = 0;
    if (o >= 0 && o + 8 <= r.num) std::memcpy(&v, r.base + o, 8);
    return v;
}
inline unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int voff, int soff, int) {
    const long long o = static_cast<long long>(voff) + soff;
    unsigned v = 0;
    if (o >= 0 && o + 4 <= r.num) std::memcpy(&v, r.base + o, 4);
    return v;
}
// DPP moves with the controls the library uses: row_shr:1..15 within rows
// of 16 lanes, row_bcast:15 (lane 15 of each row to the next row) and
// row_bcast:31 (lane 31 to rows 2 and 3).  Rows outside row_mask, and lanes
// whose source is outside the row or the wave, keep `old` (0 with bound_ctrl).
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound) {
    emu::Wave &w = *emu::ctx.wave;
    const int lane = emu::ctx.lane, row = lane >> 4;
    if (bank_mask != 0xf) { fprintf(stderr, "cpu build: DPP bank mask %x\n", bank_mask); abort(); }
    w.buf[lane] = static_cast<uint32_t>(src);
    emu::wait_at(emu::AT_WAVE);
    int res = old;
    if ((row_mask >> row) & 1) {
        int s = -1;
        if (ctrl >= 0x111 && ctrl <= 0x11f) {
            const int n = ctrl - 0x110;
            if ((lane & 15) >= n) s = lane - n;
        } else if (ctrl == 0x142) {
            if (row > 0) s = 16 * row - 1;
        } else if (ctrl == 0x143) {
            if (row >= 2) s = 31;
        } else {
            fprintf(stderr, "cpu build: DPP control %x\n", ctrl);
            abort();
        }
        if (s >= 0 && s < w.n && w.alive[s]) res = static_cast<int>(static_cast<uint32_t>(w.buf[s]));
        else if (bound) res = 0;
    }
    emu::wait_at(emu::AT_WAVE);
    return res;
}
inline double __longlong_as_double(long long x) { double d; std::memcpy(&d, &x, 8); return d; }
inline long long __double_as_longlong(double x) { long long d; std::memcpy(&d, &x, 8); return d; }
inline float __int_as_float(int x) { float d; std::memcpy(&d, &x, 4); return d; }
inline int __float_as_int(float x) { int d; std::memcpy(&d, &x, 4); return d; }

inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline int atomicAdd(int *p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline unsigned atomicAdd(unsigned *p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
template <class F> inline F atomic_add_fp(F *p, F v) {
    F o, n;
    __atomic_load(p, &o, __ATOMIC_RELAXED);
    do { n = o + v; } while (!__atomic_compare_exchange(p, &o, &n, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
    return o;
}
inline double atomicAdd(double *p, double v) { return atomic_add_fp(p, v); }
inline float atomicAdd(float *p, float v) { return atomic_add_fp(p, v); }
template <class T> inline T min(T a, T b) { return b < a ? b : a; }
template <class T> inline T max(T a, T b) { return a < b ? b : a; }
inline unsigned long long atomicMax(unsigned long long *p, unsigned long long v) {
    unsigned long long o = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (o < v && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {}
    return o;
}

// ---------------------------------------------------------------- runtime
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101, hipErrorInvalidSymbol = 701 };
typedef struct emu_stream *hipStream_t;
typedef struct emu_event *hipEvent_t;
struct emu_graph { std::vector<std::function<void()>> ops; };
typedef emu_graph *hipGraph_t;
typedef emu_graph *hipGraphExec_t;
typedef int hipStreamCaptureStatus;
enum { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
enum { hipStreamCaptureModeThreadLocal = 0 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost, hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeMaxSharedMemoryPerBlock };
struct hipDeviceProp_t { char gcnArchName[256]; char name[256]; int multiProcessorCount; };

namespace emu {
inline emu_graph *capture = nullptr;
inline int n_cu = 256;
inline long long n_malloc = 0;   // hipMalloc calls so far (allocation-free checks)
}
// Fill of fresh device memory and of LDS at the start of each workgroup:
// CPU_BUILD_FILL = pattern (default: 0xA5 for device memory, 0xFF for LDS) or
// random:<seed> (bytes from a counter-based generator), so that a read of
// memory nothing wrote sees values that differ from run to run.
inline void fill_unwritten(void *p, size_t n, unsigned char pattern) {
    static const char *mode = getenv("CPU_BUILD_FILL");
    if (!mode || strncmp(mode, "random:", 7) != 0) {
        std::memset(p, pattern, n);
        return;
    }
    static unsigned long long ctr = strtoull(mode + 7, nullptr, 10) * 0x9E3779B97F4A7C15ull;
    unsigned char *b = static_cast<unsigned char *>(p);
    for (size_t i = 0; i < n; i += 8) {
        unsigned long long z = (ctr += 0x9E3779B97F4A7C15ull);   // splitmix64
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        std::memcpy(b + i, &z, std::min<size_t>(8, n - i));
    }
}
inline hipError_t hipMalloc(void **p, size_t n) {
    ++emu::n_malloc;
    *p = aligned_alloc(256, (n + 255) / 256 * 256);
    if (!*p) return 1;
    fill_unwritten(*p, n, 0xA5);
    __asan_poison_memory_region((char *)*p + n, (n + 255) / 256 * 256 - n);
    return hipSuccess;
}
inline hipError_t hipFree(void *p) { free(p); return hipSuccess; }
// a file-scope device array is a host global here
#define HIP_SYMBOL(x) reinterpret_cast<const void *>(&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { if (n) std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    if (emu::capture) { emu::capture->ops.push_back([=] { if (n) std::memmove(d, s, n); }); return hipSuccess; }
    return hipMemcpy(d, s, n, k);
}
inline hipError_t hipMemset(void *p, int v, size_t n) { std::memset(p, v, n); return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emu error"; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeMultiprocessorCount ? emu::n_cu : 163840; return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) { std::strcpy(p->gcnArchName, "gfx950-emu"); std::strcpy(p->name, "emu"); p->multiProcessorCount = emu::n_cu; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)new char; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete (char *)e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t)new char; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete (char *)s; return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *st) { *st = emu::capture ? 1 : 0; return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { emu::capture = new emu_graph; return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = emu::capture; emu::capture = nullptr; return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, void *, size_t) { *x = new emu_graph(*g); return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { for (auto &f : x->ops) f(); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }

namespace emu {
constexpr size_t kStack = 256 * 1024;
inline unsigned char *stacks() {
    static unsigned char *p = (unsigned char *)mmap(nullptr, kStack * 1024, PROT_READ | PROT_WRITE,
                                                    MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    return p;
}
inline std::function<void(int)> *g_job;
[[noreturn]] inline void fiber_entry() {
    __sanitizer_finish_switch_fiber(nullptr, &blk.sched_bottom, &blk.sched_size);
    const int t = blk.cur;
    (*g_job)(t);
    blk.f[t].state = DONE;
    void *dead;
    __sanitizer_start_switch_fiber(nullptr, blk.sched_bottom, blk.sched_size);
    emu_switch(&dead, blk.sched_sp);
    abort();
}
// a fresh stack whose first switch-in enters fiber_entry with the stack
// aligned as after a call
inline void *fresh_stack(unsigned char *base) {
    uintptr_t top = reinterpret_cast<uintptr_t>(base + kStack) & ~uintptr_t(15);
    void **sp = reinterpret_cast<void **>(top);
    *--sp = nullptr;                                          // return address slot of fiber_entry
    *--sp = reinterpret_cast<void *>(&fiber_entry);           // popped by ret
    for (int r = 0; r < 6; ++r) *--sp = nullptr;              // rbp rbx r12 r13 r14 r15
    return sp;
}
// Order in which workgroups, and the work-items of a workgroup, are run:
// CPU_BUILD_ORDER = forward (default), reverse, or shuffle:<seed>.  Results
// that do not depend on scheduling must not change with it.
inline std::vector<int> run_order(int n, unsigned long long salt) {
    std::vector<int> o(static_cast<size_t>(n));
    std::iota(o.begin(), o.end(), 0);
    static const char *mode = getenv("CPU_BUILD_ORDER");
    if (!mode || !strcmp(mode, "forward")) return o;
    if (!strcmp(mode, "reverse")) {
        std::reverse(o.begin(), o.end());
        return o;
    }
    if (strncmp(mode, "shuffle:", 8) != 0) { fprintf(stderr, "cpu build: CPU_BUILD_ORDER=%s\n", mode); abort(); }
    unsigned long long x = (strtoull(mode + 8, nullptr, 10) + 1) * 0x9E3779B97F4A7C15ull ^ (salt * 0xBF58476D1CE4E5B9ull);
    for (int i = n - 1; i > 0; --i) {   // Fisher-Yates with xorshift64*
        x ^= x >> 12;
        x ^= x << 25;
        x ^= x >> 27;
        const int j = static_cast<int>((x * 2685821657736338717ull) % static_cast<unsigned long long>(i + 1));
        std::swap(o[static_cast<size_t>(i)], o[static_cast<size_t>(j)]);
    }
    return o;
}
template <class... KP, class Tup>
void run(void (*k)(KP...), dim3 g, dim3 b, size_t shm, Tup args) {
    ++n_launch;
    const int nt = int(b.x * b.y * b.z);
    if (nt < 1 || nt > 1024) { fprintf(stderr, "cpu build: block of %d threads\n", nt); abort(); }
    if (shm > kLds) { fprintf(stderr, "cpu build: %zu B of dynamic LDS\n", shm); abort(); }
    if (verbose) fprintf(stderr, "EMU launch %lld grid %u,%u,%u block %d shm %zu\n", n_launch, g.x, g.y, g.z, nt, shm);
    const int nw = (nt + 63) / 64;
    std::vector<Wave> waves(nw);
    const int nb = static_cast<int>(g.x * g.y * g.z);
    const std::vector<int> blocks = run_order(nb, static_cast<unsigned long long>(n_launch));
    for (int bi : blocks) {
                const unsigned bx = static_cast<unsigned>(bi) % g.x, by = (static_cast<unsigned>(bi) / g.x) % g.y,
                               bz = static_cast<unsigned>(bi) / (g.x * g.y);
                const std::vector<int> lanes = run_order(nt, static_cast<unsigned long long>(n_blocks) * 7919u + 1u);
                ++n_blocks;
                __asan_unpoison_memory_region(lds, kLds);
                fill_unwritten(lds, kLds, 0xFF);
                __asan_poison_memory_region(lds + shm, kLds - shm);
                for (int w = 0; w < nw; ++w) {
                    waves[w].n = std::min(64, nt - 64 * w);
                    for (int l = 0; l < 64; ++l) waves[w].alive[l] = l < waves[w].n;
                }
                std::function<void(int)> job = [&](int t) {
                    Tup a = args;
                    std::apply(k, a);
                    waves[t / 64].alive[t % 64] = false;
                };
                g_job = &job;
                blk.nt = nt;
                blk.f.assign(nt, Fiber{});
                for (int t = 0; t < nt; ++t) {
                    blk.f[t].sp = fresh_stack(stacks() + kStack * t);
                    blk.f[t].state = RUN;
                }
                for (;;) {
                    for (int t : lanes) {
                        if (blk.f[t].state != RUN) continue;
                        blk.cur = t;
                        ctx.tid = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
                        ctx.bid = dim3(bx, by, bz);
                        ctx.bdim = b;
                        ctx.gdim = g;
                        ctx.wave = &waves[t / 64];
                        ctx.lane = t % 64;
                        void *fake = nullptr;
                        __sanitizer_start_switch_fiber(&fake, stacks() + kStack * t, kStack);
                        emu_switch(&blk.sched_sp, blk.f[t].sp);
                        __sanitizer_finish_switch_fiber(fake, &blk.sched_bottom, &blk.sched_size);
                    }
                    bool released = false, all_done = true, all_block = true;
                    for (int w = 0; w < nw; ++w) {
                        bool any = false, all_wave = true;
                        for (int l = 0; l < waves[w].n; ++l) {
                            const int st = blk.f[64 * w + l].state;
                            if (st == DONE) continue;
                            any = true;
                            all_done = false;
                            if (st != AT_WAVE) all_wave = false;
                            if (st != AT_BLOCK) all_block = false;
                        }
                        if (any && all_wave) {
                            for (int l = 0; l < waves[w].n; ++l)
                                if (blk.f[64 * w + l].state == AT_WAVE) blk.f[64 * w + l].state = RUN;
                            released = true;
                        }
                    }
                    if (all_done) break;
                    if (!released && all_block) {
                        for (int t = 0; t < nt; ++t)
                            if (blk.f[t].state == AT_BLOCK) blk.f[t].state = RUN;
                        released = true;
                    }
                    if (!released) { fprintf(stderr, "cpu build: lanes of one wave wait at different barriers\n"); abort(); }
                }
            }
    __asan_unpoison_memory_region(lds, kLds);
}
template <class... KP, class... A>
void launch(void (*k)(KP...), dim3 g, dim3 b, size_t shm, hipStream_t, A &&...a) {
    std::tuple<std::decay_t<KP>...> args(static_cast<KP>(a)...);
    if (capture) { capture->ops.push_back([=] { run(k, g, b, shm, args); }); return; }
    run(k, g, b, shm, args);
}
}  // namespace emu
#define hipLaunchKernelGGL(K, G, B, SHM, S, ...) emu::launch(K, dim3(G), dim3(B), SHM, S, ##__VA_ARGS__)
