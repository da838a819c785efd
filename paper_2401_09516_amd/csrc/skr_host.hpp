// Host-side internals of libskr shared by the C ABI (skr_api.hip) and the serving runtime
// (skr_serve.hip): the context, error reporting and the per-system solve.
#pragma once
#include <map>
#include <mutex>
#include <string>

#include "skr_internal.hpp"

namespace skr {
struct Server;
struct ChainSet;

// Sub-allocator over a caller-owned device buffer (the arena of skr_ctx_create): first fit over the
// free blocks in address order, every block a multiple of 256 bytes at a 256-byte offset, freed
// blocks merged with free neighbours. Thread-safe (serving workers allocate concurrently).
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::mutex mu;
    std::map<size_t, size_t> free_blocks;   // offset -> length
    std::map<size_t, size_t> live;          // offset -> length
    size_t in_use = 0;
    Arena(void* b, size_t n);
    void* alloc(size_t bytes);              // nullptr when no free block is large enough
    void release(void* p);
    bool can_fit(const size_t* sizes, int count);   // would these allocations succeed, in order?
};
constexpr int PROF_PERIOD = 16;   // one Arnoldi step in PROF_PERIOD is timed
constexpr int PROF_MAXSAMP = (MMAX + PROF_PERIOD - 1) / PROF_PERIOD + 1;
}  // namespace skr

struct skr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    skr::Arena* arena = nullptr;        // caller's arena (shared with the serving chains' contexts)
    bool owns_arena = false;            // this context created the Arena record (not the memory)
    skr::Work w;
    skr::CtrlHost* hctrl = nullptr;     // pinned
    hipEvent_t ev_ctrl = nullptr;       // recorded after the read of a cycle end's control block
    int* hkeff = nullptr;          // pinned
    // sort scratch
    double* sortD = nullptr;
    size_t sortD_cap = 0;
    double* sortP = nullptr;       // slice partials of the distance pass
    size_t sortP_cap = 0;
    long long* order_d = nullptr;
    double* dist_d = nullptr;
    size_t sortN_cap = 0;
    // FP32 copy of the operator's values (CSR values or stencil faces) for the mixed mode's
    // Arnoldi products, grown on demand
    float* op32 = nullptr;
    size_t op32_cap = 0;
    // profiling
    hipEvent_t ev[skr::PROF_MAXSAMP * 6] = {};
    bool ev_ok = false;
    int64_t step_counter = 0;
    skr_profile prof = {};
    // steps the first cycle of the previous system on this context ran when it stopped early (0: it
    // ran the full cycle); predicts the launch length of the next system's first cycle
    int pred_first = 0;
    // recycle space carried in w.U after the last solve on this context (or skr_recycle_set): its
    // column count and the (n, m, k, mixed) it belongs to; valid only while the workspace keeps it
    bool carry_valid = false;
    int carry_k = 0, carry_n = 0, carry_m = 0, carry_kmax = 0, carry_mixed = 0;
    // serving (skr_serve_start .. skr_serve_stop)
    skr::Server* server = nullptr;
    // the chain contexts and tables of skr_solve_chains, kept for the next call on this context
    skr::ChainSet* chains = nullptr;
};

namespace skr {
// Records the message of an error for skr_last_error() in the calling thread; returns code.
int fail(int code, const char* fmt, ...);
// The calling thread's last error message.
const std::string& last_error();
// Per-system solve and its set-up (skr_api.hip).
int check_opts(const skr_opts* opts);
int prepare_solve(skr_ctx* ctx, int n, const skr_opts& opts);
int solve_system(skr_ctx* ctx, const skr_op& op, const double* b, double* x, const skr_opts& opts, int& kin,
                 skr_result& res);
int to_devop(const skr_op& o, DevOp& d, int64_t& nvals);
// Internal context with its own stream (serving chains), allocating from `arena` when given;
// freed with skr_ctx_destroy.
int ctx_make(int device, hipStream_t stream, skr_ctx** out, Arena* arena = nullptr);
// Device bytes of the workspace ensure_work allocates for (n, m, k): one block.
size_t work_bytes(int n, int m, int k);
// Device memory of a context: from its arena when it has one, else hipMalloc.
hipError_t dev_alloc(skr_ctx* ctx, void** p, size_t bytes);
void dev_free(skr_ctx* ctx, void* p);
inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }
// Serving state of a context (skr_serve.hip).
void serve_free(skr_ctx* ctx);
// Algorithmic bytes of the kernels of Arnoldi step j (passes A, B, C; c = 0 with two kernels).
void step_bytes(const DevOp& op, int64_t nvals, int kc, int j, bool mixed, bool merged, double& a, double& b,
                double& c);
// Releases the chain contexts and tables skr_solve_chains keeps on ctx.
void chains_free(skr_ctx* ctx);
}  // namespace skr

#define HIPCHK(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return skr::fail(SKR_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define HIPLAUNCHCHK()                                                                          \
    do {                                                                                        \
        hipError_t e_ = hipGetLastError();                                                      \
        if (e_ != hipSuccess) return skr::fail(SKR_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)
