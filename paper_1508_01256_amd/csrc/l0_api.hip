// Host side of the l0decode C-ABI: argument checks, workspace layout and
// kernel launches.  Every check happens before anything is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "l0_internal.h"

struct l0_matrix_s {
    l0::MatrixView view;
    void* base;
    int device;
};

namespace l0 {

MatrixBuffers matrix_layout(int64_t n, int32_t m, int32_t d) {
    MatrixBuffers b{};
    const int64_t ntiles = (n + kTile - 1) / kTile;
    b.soa = align256(static_cast<size_t>(ntiles) * d * kTile * (rows16(m) ? 2 : 4));
    b.row_off = align256((static_cast<size_t>(m) + 1) * sizeof(int32_t));
    b.deg = align256(static_cast<size_t>(m) * sizeof(int32_t));
    b.flag = 256;
    b.partial = repack_lds_hist(m, d) ? 0
                                      : align256(static_cast<size_t>(deg_slices(n, d)) * m * sizeof(int32_t));
    b.blk = b.partial ? align256(static_cast<size_t>(deg_blocks(m)) * sizeof(int32_t)) : 0;
    b.total = b.soa + b.row_off + b.deg + b.flag + b.partial + b.blk;
    return b;
}

SolveBuffers solve_layout(int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    SolveBuffers b{};
    b.ctrl = align256(sizeof(Ctrl));
    b.counters = align256(2 * (static_cast<size_t>(max_iter) + 2) * sizeof(int32_t));
    b.r = align256(static_cast<size_t>(m) * sizeof(double));
    b.rword = align256(static_cast<size_t>(m) * sizeof(uint32_t));
    b.slot_cnt = b.slot_sorted = b.aff_flag = align256(static_cast<size_t>(m) * sizeof(int32_t));
    b.aff_list = align256(2 * static_cast<size_t>(m) * sizeof(int32_t));
    b.member = align256(static_cast<size_t>((n + 31) / 32) * sizeof(uint32_t));
    b.slots = align256(static_cast<size_t>(n) * d * sizeof(int32_t));
    b.total = b.ctrl + b.counters + b.r + b.rword + 3 * b.slot_cnt + b.aff_list + b.member + b.slots;
    return b;
}

}  // namespace l0

namespace {

constexpr int32_t kMaxIterCap = 1 << 20;

bool sizes_ok(int64_t n, int32_t m, int32_t d) {
    if (n < 1 || m < 1 || d < l0::kDMin || d > l0::kDMax || d > m) return false;
    if (n > INT32_MAX) return false;                  // column ids are stored as int32
    if (n * static_cast<int64_t>(d) >= INT32_MAX) return false;  // row capacities are int32
    return true;
}

bool solve_args_ok(double alpha, int32_t d, int32_t max_iter, double tol) {
    if (!(alpha > 1.0) || !(alpha <= static_cast<double>(d))) return false;
    if (max_iter < 0 || max_iter > kMaxIterCap) return false;
    if (!(tol >= 0.0) || !std::isfinite(tol)) return false;
    return true;
}

bool opts_ok(const l0_opts* o) {
    if (!o) return true;
    if ((o->rule < L0_RULE_L0DEC || o->rule > L0_RULE_SHIFTED_MODE)) return false;
    if (o->tol_mode != L0_TOL_RELATIVE && o->tol_mode != L0_TOL_ABSOLUTE) return false;
    return o->reserved0 == 0 && o->reserved1 == 0;
}

// A device-accessible buffer of at least `bytes` starting at p.  Plain host
// memory is rejected; when the runtime knows the allocation's extent, the
// buffer must lie inside it.
bool buffer_ok(const void* p, size_t bytes) {
    if (bytes == 0) return true;
    if (!p) return false;
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof(at));
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged &&
        !(at.type == hipMemoryTypeHost && at.devicePointer != nullptr))
        return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
        const uintptr_t lo = reinterpret_cast<uintptr_t>(base), hi = lo + size;
        const uintptr_t a = reinterpret_cast<uintptr_t>(p);
        if (a < lo || a + bytes > hi) return false;
    } else {
        (void)hipGetLastError();
    }
    return true;
}

l0_status from_hip(hipError_t e) {
    if (e == hipSuccess) return L0_OK;
    if (e == hipErrorOutOfMemory) return L0_ERR_OOM;
    return L0_ERR_HIP;
}

l0::MatrixView carve_matrix(char* base, int64_t n, int32_t m, int32_t d) {
    const l0::MatrixBuffers b = l0::matrix_layout(n, m, d);
    l0::MatrixView v{};
    v.n = n;
    v.m = m;
    v.d = d;
    v.ntiles = (n + l0::kTile - 1) / l0::kTile;
    char* p = base;
    v.rows16 = l0::rows16(m) ? 1 : 0;
    v.soa = p;                                    p += b.soa;
    v.row_off = reinterpret_cast<int32_t*>(p);   p += b.row_off;
    v.deg = reinterpret_cast<int32_t*>(p);       p += b.deg;
    v.bad_input = reinterpret_cast<int32_t*>(p); p += b.flag;
    v.partial = b.partial ? reinterpret_cast<int32_t*>(p) : nullptr;  p += b.partial;
    v.blk = b.blk ? reinterpret_cast<int32_t*>(p) : nullptr;
    v.slices = b.partial ? l0::deg_slices(n, d) : 0;
    return v;
}

void carve_solve(l0::SolveParams& q, char* base, int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    const l0::SolveBuffers b = l0::solve_layout(n, m, d, max_iter);
    char* p = base;
    q.ctrl = reinterpret_cast<l0::Ctrl*>(p);            p += b.ctrl;
    q.tcount = reinterpret_cast<int32_t*>(p);
    q.affc = q.tcount + (max_iter + 2);                  p += b.counters;
    q.r = reinterpret_cast<double*>(p);                  p += b.r;
    q.rword = p;                                         p += b.rword;
    q.slot_cnt = reinterpret_cast<int32_t*>(p);          p += b.slot_cnt;
    q.slot_sorted = reinterpret_cast<int32_t*>(p);       p += b.slot_sorted;
    q.aff_flag = reinterpret_cast<int32_t*>(p);          p += b.aff_flag;
    q.aff_list = reinterpret_cast<int32_t*>(p);          p += b.aff_list;
    q.member = reinterpret_cast<uint32_t*>(p);           p += b.member;
    q.slots = reinterpret_cast<int32_t*>(p);
}

// The control-block run that a one-shot decode's preparation clears for the
// solve whose workspace starts at ws (none when the solve must fill it).
l0::ZeroSpan one_shot_clear(char* ws, int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    l0::SolveParams q{};
    q.max_iter = max_iter;
    carve_solve(q, ws, n, m, d, max_iter);
    return l0::solve_control_span(q);
}

l0_status run_solve(const l0::MatrixView& A, const double* y, double alpha, int32_t max_iter,
                    double tol, double* x_out, const l0_opts* opts, l0_result* res,
                    int32_t* iters_out, char* ws, hipStream_t stream, bool ctrl_cleared = false) {
    l0::SolveParams q{};
    q.n = A.n;
    q.m = A.m;
    q.d = A.d;
    q.ntiles = A.ntiles;
    q.wmode = l0::word_mode(A.m);
    q.soa = A.soa;
    q.row_off = A.row_off;
    q.bad_input = A.bad_input;
    q.y = y;
    q.tol = tol;
    q.a = static_cast<int32_t>(std::ceil(alpha));
    q.max_iter = max_iter;
    q.rule = opts ? opts->rule : L0_RULE_L0DEC;
    q.tol_mode = opts ? opts->tol_mode : L0_TOL_RELATIVE;
    q.x_init = opts ? opts->x_init : nullptr;
    q.w = opts ? opts->weights : nullptr;
    q.x = x_out;
    q.trace = opts ? opts->trace : nullptr;
    q.tsize = opts ? opts->tsize : nullptr;
    q.timeline = opts ? opts->timeline : nullptr;
    q.res = res;
    q.iters_out = iters_out;
    carve_solve(q, ws, A.n, A.m, A.d, max_iter);
    q.ctrl_cleared = ctrl_cleared ? 1 : 0;
    return from_hip(l0::launch_solve(q, stream));
}

bool common_buffers_ok(int64_t n, int32_t m, int32_t max_iter, const double* y, double* x_out,
                       const l0_opts* opts) {
    if (!buffer_ok(y, static_cast<size_t>(m) * sizeof(double))) return false;
    if (!buffer_ok(x_out, static_cast<size_t>(n) * sizeof(double))) return false;
    if (opts) {
        if (opts->x_init && !buffer_ok(opts->x_init, static_cast<size_t>(n) * sizeof(double))) return false;
        if (opts->weights && !buffer_ok(opts->weights, static_cast<size_t>(n) * sizeof(double))) return false;
        if (opts->trace && !buffer_ok(opts->trace, (static_cast<size_t>(max_iter) + 1) * sizeof(int32_t)))
            return false;
        if (opts->tsize && max_iter > 0 &&
            !buffer_ok(opts->tsize, static_cast<size_t>(max_iter) * sizeof(int64_t)))
            return false;
        if (opts->timeline &&
            !buffer_ok(opts->timeline, (6 * static_cast<size_t>(max_iter) + 16) * sizeof(int64_t)))
            return false;
    }
    return true;
}

}  // namespace

namespace l0 {

bool device_buffer_ok(const void* p, size_t bytes) { return buffer_ok(p, bytes); }

}  // namespace l0

extern "C" {

const char* l0_version(void) { return "l0decode 0.1 (gfx950)"; }

l0_status l0_set_solve_admission(int32_t max_members, int32_t window_us) {
    l0::set_solve_admission(max_members, window_us);
    return L0_OK;
}

const char* l0_status_string(int32_t code) {
    switch (code) {
        case 0: return "L0_OK / L0_CONVERGED";
        case 1: return "L0_ERR_ARG / L0_STALLED";
        case 2: return "L0_ERR_OOM / L0_MAX_ITER";
        case 3: return "L0_ERR_HIP";
        case 4: return "L0_ERR_WORKSPACE";
        case L0_DEV_BAD_INDEX: return "L0_DEV_BAD_INDEX";
        case L0_DEV_NONFINITE_Y: return "L0_DEV_NONFINITE_Y";
        case L0_DEV_ABORTED: return "L0_DEV_ABORTED";
        case L0_DEV_BAD_WEIGHT: return "L0_DEV_BAD_WEIGHT";
        case L0_DEV_REPEATED_ROW: return "L0_DEV_REPEATED_ROW";
        default: return "unknown";
    }
}

size_t l0_workspace_bytes(int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    if (!sizes_ok(n, m, d) || max_iter < 0 || max_iter > kMaxIterCap) return 0;
    return l0::matrix_layout(n, m, d).total + l0::solve_layout(n, m, d, max_iter).total;
}

l0_status l0_decode_ex(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                       double alpha, int32_t max_iter, double tol, double* x_out,
                       const l0_opts* opts, l0_result* res_out, void* workspace,
                       size_t ws_bytes, hipStream_t stream) {
    if (!sizes_ok(n, m, d) || !solve_args_ok(alpha, d, max_iter, tol) || !opts_ok(opts)) return L0_ERR_ARG;
    if (!buffer_ok(col_idx, static_cast<size_t>(n) * d * sizeof(int32_t))) return L0_ERR_ARG;
    if (!common_buffers_ok(n, m, max_iter, y, x_out, opts)) return L0_ERR_ARG;
    if (!buffer_ok(res_out, sizeof(l0_result))) return L0_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return L0_ERR_ARG;
    const size_t need = l0_workspace_bytes(n, m, d, max_iter);
    if (ws_bytes < need) return L0_ERR_WORKSPACE;
    if (!buffer_ok(workspace, need)) return L0_ERR_ARG;
    char* base = static_cast<char*>(workspace);
    const l0::MatrixView A = carve_matrix(base, n, m, d);
    char* const sws = base + l0::matrix_layout(n, m, d).total;
    const l0::ZeroSpan clear = one_shot_clear(sws, n, m, d, max_iter);
    l0_status st = from_hip(l0::launch_prepare(col_idx, A, 1, stream, clear));
    if (st != L0_OK) return st;
    return run_solve(A, y, alpha, max_iter, tol, x_out, opts, res_out, nullptr, sws, stream, clear.p != nullptr);
}

}  // extern "C"

namespace {

// Host checks of l0_decode's arguments (and of its allocation-free variant).
bool plain_args_ok(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y, double alpha,
                   int32_t max_iter, double tol, double* x_out, int32_t* iters_out) {
    if (!sizes_ok(n, m, d) || !solve_args_ok(alpha, d, max_iter, tol)) return false;
    if (!buffer_ok(col_idx, static_cast<size_t>(n) * d * sizeof(int32_t))) return false;
    if (!common_buffers_ok(n, m, max_iter, y, x_out, nullptr)) return false;
    return buffer_ok(iters_out, sizeof(int32_t));
}

// Workspace of one plain decode: matrix, solve, then the device result.
size_t plain_workspace_bytes(int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    return l0::matrix_layout(n, m, d).total + l0::solve_layout(n, m, d, max_iter).total +
           l0::align256(sizeof(l0_result));
}

// Enqueue a plain decode in the workspace at base (need bytes, laid out as
// plain_workspace_bytes says); nothing in it needs to be initialised.
l0_status plain_decode_in(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y, double alpha,
                          int32_t max_iter, double tol, double* x_out, int32_t* iters_out, char* base, size_t need,
                          hipStream_t stream) {
    const size_t mat = l0::matrix_layout(n, m, d).total;
    const l0::MatrixView A = carve_matrix(base, n, m, d);
    l0_result* res = reinterpret_cast<l0_result*>(base + need - l0::align256(sizeof(l0_result)));
    const l0::ZeroSpan clear = one_shot_clear(base + mat, n, m, d, max_iter);
    l0_status st = from_hip(l0::launch_prepare(col_idx, A, 1, stream, clear));
    if (st == L0_OK)
        st = run_solve(A, y, alpha, max_iter, tol, x_out, nullptr, res, iters_out, base + mat, stream,
                       clear.p != nullptr);
    return st;
}

}  // namespace

extern "C" {

l0_status l0_decode(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                    double alpha, int32_t max_iter, double tol, double* x_out,
                    int32_t* iters_out, hipStream_t stream) {
    if (!plain_args_ok(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out)) return L0_ERR_ARG;
    const size_t need = plain_workspace_bytes(n, m, d, max_iter);
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, need, stream);
    if (e != hipSuccess) return from_hip(e);
    l0_status st = plain_decode_in(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out,
                                   static_cast<char*>(ws), need, stream);
    e = hipFreeAsync(ws, stream);
    if (st == L0_OK && e != hipSuccess) st = from_hip(e);
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plain decode without any allocation: the workspace is a fixed device array
// ---------------------------------------------------------------------------

namespace {

// The array the allocation-free decode works in, one copy per device (each
// device holds its own until the process ends).  Its name is a host-side
// stand-in: host code uses only the device address taken below.
constexpr size_t kScratchBytes = size_t(128) << 20;
static_assert(kScratchBytes == L0_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, taken once per
// device (with that device current); nullptr if it cannot be had.
char* scratch_on_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace

extern "C" {

l0_status l0_decode_noalloc(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, const double* y,
                            double alpha, int32_t max_iter, double tol, double* x_out, int32_t* iters_out,
                            hipStream_t stream) {
    if (!plain_args_ok(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out)) return L0_ERR_ARG;
    const size_t need = plain_workspace_bytes(n, m, d, max_iter);
    if (need > kScratchBytes) return L0_ERR_WORKSPACE;
    char* base = scratch_on_current_device();
    if (!base) return L0_ERR_HIP;
    // every part of the workspace that must start at zero is cleared by the
    // decode's own fill kernels (no memset)
    return plain_decode_in(col_idx, n, m, d, y, alpha, max_iter, tol, x_out, iters_out, base, need, stream);
}

size_t l0_noalloc_workspace_bytes(int64_t n, int32_t m, int32_t d, int32_t max_iter) {
    if (!sizes_ok(n, m, d) || max_iter < 0 || max_iter > kMaxIterCap) return 0;
    return plain_workspace_bytes(n, m, d, max_iter);
}

l0_status l0_matrix_create(const int32_t* col_idx, int64_t n, int32_t m, int32_t d, l0_matrix* out,
                           hipStream_t stream) {
    if (!out) return L0_ERR_ARG;
    *out = nullptr;
    if (!sizes_ok(n, m, d)) return L0_ERR_ARG;
    if (!buffer_ok(col_idx, static_cast<size_t>(n) * d * sizeof(int32_t))) return L0_ERR_ARG;
    l0_matrix h = new (std::nothrow) l0_matrix_s;
    if (!h) return L0_ERR_OOM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return L0_ERR_HIP;
    }
    hipError_t e = hipMalloc(&h->base, l0::matrix_layout(n, m, d).total);
    if (e != hipSuccess) {
        delete h;
        return from_hip(e);
    }
    h->view = carve_matrix(static_cast<char*>(h->base), n, m, d);
    l0_status st = from_hip(l0::launch_prepare(col_idx, h->view, 1, stream));
    if (st != L0_OK) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(h->base);
        delete h;
        return st;
    }
    *out = h;
    return L0_OK;
}

l0_status l0_matrix_destroy(l0_matrix A) {
    if (!A) return L0_OK;
    hipError_t e = hipDeviceSynchronize();
    hipError_t f = hipFree(A->base);
    delete A;
    return from_hip(e != hipSuccess ? e : f);
}

size_t l0_solve_workspace_bytes(l0_matrix A, int32_t max_iter) {
    if (!A || max_iter < 0 || max_iter > kMaxIterCap) return 0;
    return l0::solve_layout(A->view.n, A->view.m, A->view.d, max_iter).total;
}

l0_status l0_solve(l0_matrix A, const double* y, double alpha, int32_t max_iter, double tol,
                   double* x_out, const l0_opts* opts, l0_result* res_out, void* workspace,
                   size_t ws_bytes, hipStream_t stream) {
    if (!A || !solve_args_ok(alpha, A->view.d, max_iter, tol) || !opts_ok(opts)) return L0_ERR_ARG;
    const int64_t n = A->view.n;
    const int32_t m = A->view.m;
    if (!common_buffers_ok(n, m, max_iter, y, x_out, opts)) return L0_ERR_ARG;
    if (!buffer_ok(res_out, sizeof(l0_result))) return L0_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return L0_ERR_ARG;
    const size_t need = l0_solve_workspace_bytes(A, max_iter);
    if (ws_bytes < need) return L0_ERR_WORKSPACE;
    if (!buffer_ok(workspace, need)) return L0_ERR_ARG;
    return run_solve(A->view, y, alpha, max_iter, tol, x_out, opts, res_out, nullptr,
                     static_cast<char*>(workspace), stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched decoding
// ---------------------------------------------------------------------------

#include <algorithm>
#include <numeric>
#include <vector>

#include "l0_batch.h"

namespace {

// Instances of one degree range (l0::kBatchRanges): they run in one
// persistent launch of that range's kernel.
struct Group {
    int range = 0;
    int d = 0;                         // largest degree in the group
    int32_t inst_start = 0, inst_count = 0;  // range of the instance order
    int32_t item_start = 0, item_count = 0;  // range of the work items
    int32_t max_m = 0;
    int words_cap = 0;
    size_t lds = 0;
    int grid = 0;
};

struct BatchPlan {
    int block_threads = 256;
    int words_cap = 8192;
    std::vector<int32_t> order;     // instances: by degree range, then largest n*d first
    std::vector<Group> groups;
    std::vector<int32_t> items;     // work items of every group, in claim order
    std::vector<int32_t> team;      // team size per instance
    std::vector<int64_t> inst_off;  // scratch offset per instance
    size_t table = 0, items_bytes = 0, team_bytes = 0, off_bytes = 0, counters = 0, ctl = 0, scratch = 0,
           total = 0;
};

constexpr size_t kLdsLimit = 160 * 1024 - 1024;  // dynamic LDS bound (static use is < 1 KiB)
constexpr int64_t kTeamUnit = int64_t(1) << 19;     // estimated cost per team member (large batches)
constexpr int64_t kMinTeamUnit = int64_t(1) << 15;  // least cost per team member (small batches)

bool batch_opts_ok(const l0_batch_opts* o) {
    if (!o) return true;
    if ((o->rule < L0_RULE_L0DEC || o->rule > L0_RULE_SHIFTED_MODE)) return false;
    if (o->tol_mode != L0_TOL_RELATIVE && o->tol_mode != L0_TOL_ABSOLUTE) return false;
    if (o->block_threads != 0 && o->block_threads != 256 && o->block_threads != 512) return false;
    return o->words_cap == 0 || (o->words_cap >= 64 && o->words_cap <= 32768);
}

// Validate every instance (sizes and scalars always; buffers when asked),
// order them, group them by degree range and lay out their scratch.
bool problems_ok(const l0_problem* probs, int32_t count, BatchPlan& pl, bool buffers) {
    if (!probs || count < 1 || count >= (1 << l0::kItemInstBits)) return false;
    for (int32_t i = 0; i < count; ++i) {
        const l0_problem& P = probs[i];
        if (!sizes_ok(P.n, P.m, P.d) || !solve_args_ok(P.alpha, P.d, P.max_iter, P.tol) || P.reserved != 0)
            return false;
        if (buffers) {
            if (!buffer_ok(P.col_idx, static_cast<size_t>(P.n) * P.d * sizeof(int32_t))) return false;
            if (!buffer_ok(P.y, static_cast<size_t>(P.m) * sizeof(double))) return false;
            if (!buffer_ok(P.x_out, static_cast<size_t>(P.n) * sizeof(double))) return false;
            if (P.weights && !buffer_ok(P.weights, static_cast<size_t>(P.n) * sizeof(double))) return false;
        }
    }
    pl.order.resize(count);
    std::iota(pl.order.begin(), pl.order.end(), 0);
    std::stable_sort(pl.order.begin(), pl.order.end(), [&](int32_t a, int32_t b) {
        const int ra = l0::batch_range_of(probs[a].d), rb = l0::batch_range_of(probs[b].d);
        if (ra != rb) return ra < rb;
        return probs[a].n * probs[a].d > probs[b].n * probs[b].d;
    });
    pl.groups.clear();
    for (int32_t q = 0; q < count; ++q) {
        const l0_problem& P = probs[pl.order[q]];
        const int range = l0::batch_range_of(P.d);
        if (pl.groups.empty() || pl.groups.back().range != range) {
            Group g;
            g.range = range;
            g.inst_start = q;
            pl.groups.push_back(g);
        }
        Group& g = pl.groups.back();
        ++g.inst_count;
        g.d = std::max(g.d, static_cast<int>(P.d));
        g.max_m = std::max(g.max_m, P.m);
    }
    pl.inst_off.resize(count);
    size_t off = 0;
    for (int32_t i = 0; i < count; ++i) {
        pl.inst_off[i] = static_cast<int64_t>(off);
        off += l0::inst_layout(probs[i].n, probs[i].m, probs[i].d).total;
    }
    pl.scratch = off;
    return true;
}

// Resident workgroups, LDS, team sizes and work items of every group for
// one schedule (block size, bucket-word capacity); false if infeasible.
// share: the number of batches that may run on the device at once (each is
// planned within an equal share of the resident workgroups, so that all of
// them can be resident together and no team waits for members that cannot be
// scheduled).
bool plan_batch(const l0_problem* probs, int32_t count, int block_threads, int words_cap, BatchPlan& pl,
                int share = 1) {
    pl.block_threads = block_threads;
    pl.words_cap = words_cap;
    const int cus = l0::device_cus();
    pl.items.clear();
    pl.team.assign(count, 1);
    for (Group& g : pl.groups) {
        // no more LDS words than the group's largest m needs
        const int64_t need = (static_cast<int64_t>(g.max_m) + 63) / 64 * 64;
        g.words_cap = static_cast<int>(std::min<int64_t>(words_cap, need));
        g.lds = l0::batch_lds_bytes(block_threads, g.words_cap, g.d);
        if (g.lds > kLdsLimit) return false;
        const void* fn = l0::batch_kernel_fn(block_threads, g.range);
        if (!fn) return false;
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(g.lds)) !=
            hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block_threads, g.lds) != hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            return false;
        }
        const int64_t resident =
            std::max<int64_t>(1, static_cast<int64_t>(per_cu) * (cus > 0 ? cus : 1) / std::max(1, share));
        // Estimated cost of an instance: its column indices, three times over
        // when its bucket words do not fit in LDS even folded to 16 bits (the
        // vote then gathers them from global memory, about three times
        // slower).  An instance gets one team member per unit of cost (at
        // most kMaxTeam, never more than the resident workgroups: members
        // wait for each other).
        auto cost = [&](int32_t i) {
            const int64_t nd = probs[i].n * probs[i].d;
            return probs[i].m <= 2 * static_cast<int64_t>(g.words_cap) ? nd : 3 * nd;
        };
        const int64_t tmax = std::min<int64_t>(l0::kMaxTeam, resident);
        // A batch too small to fill the resident workgroups at kTeamUnit per
        // member (a few requests of a server, one large instance) gets a
        // smaller unit, so that its teams spread over the whole device.
        int64_t total = 0;
        for (int32_t q = g.inst_start; q < g.inst_start + g.inst_count; ++q) total += cost(pl.order[q]);
        const int64_t unit = std::max<int64_t>(kMinTeamUnit, std::min<int64_t>(kTeamUnit, total / resident));
        for (int32_t q = g.inst_start; q < g.inst_start + g.inst_count; ++q) {
            const int32_t i = pl.order[q];
            pl.team[i] = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(tmax, (cost(i) + unit - 1) / unit)));
        }
        // Claim order: largest cost per team member first (it sets the time
        // of an iteration, and an instance of unforeseen iteration count is
        // then long for that reason), larger total cost first among equals.
        std::stable_sort(pl.order.begin() + g.inst_start, pl.order.begin() + g.inst_start + g.inst_count,
                         [&](int32_t a, int32_t b) {
                             const int64_t pa = cost(a) / pl.team[a], pb = cost(b) / pl.team[b];
                             return pa != pb ? pa > pb : cost(a) > cost(b);
                         });
        g.item_start = static_cast<int32_t>(pl.items.size());
        for (int32_t q = g.inst_start; q < g.inst_start + g.inst_count; ++q) {
            const int32_t i = pl.order[q];
            for (int r = 0; r < pl.team[i]; ++r) pl.items.push_back(i | (r << l0::kItemInstBits));
        }
        g.item_count = static_cast<int32_t>(pl.items.size()) - g.item_start;
        g.grid = static_cast<int>(std::min<int64_t>(resident, g.item_count));
    }
    pl.table = l0::align256(static_cast<size_t>(count) * sizeof(l0_problem));
    pl.items_bytes = l0::align256(pl.items.size() * sizeof(int32_t));
    pl.team_bytes = l0::align256(static_cast<size_t>(count) * sizeof(int32_t));
    pl.off_bytes = l0::align256(static_cast<size_t>(count) * sizeof(int64_t));
    pl.counters = l0::align256(pl.groups.size() * sizeof(int32_t));
    pl.ctl = static_cast<size_t>(count) * sizeof(l0::TeamCtl);
    pl.total = pl.table + pl.items_bytes + pl.team_bytes + pl.off_bytes + pl.counters + pl.ctl + pl.scratch;
    return true;
}

struct Candidate {
    int block_threads, words_cap;
};
const Candidate kCandidates[] = {{256, 8192}, {256, 16384}, {512, 16384}, {512, 32768}};

void resolve(const l0_batch_opts* o, int& bt, int& wc) {
    bt = (o && o->block_threads) ? o->block_threads : 256;
    wc = (o && o->words_cap) ? o->words_cap : 8192;
}

l0_status launch_batch(const l0_problem* probs, int32_t count, const l0_batch_opts* opts, const BatchPlan& pl,
                       l0_result* results, char* ws, hipStream_t stream) {
    char* p = ws;
    auto take = [&](size_t bytes) { char* at = p; p += bytes; return at; };
    l0_problem* table = reinterpret_cast<l0_problem*>(take(pl.table));
    int32_t* items = reinterpret_cast<int32_t*>(take(pl.items_bytes));
    int32_t* team = reinterpret_cast<int32_t*>(take(pl.team_bytes));
    int64_t* inst_off = reinterpret_cast<int64_t*>(take(pl.off_bytes));
    unsigned* counters = reinterpret_cast<unsigned*>(take(pl.counters));
    l0::TeamCtl* ctl = reinterpret_cast<l0::TeamCtl*>(take(pl.ctl));
    char* scratch = take(pl.scratch);
    hipError_t e = hipMemcpyAsync(table, probs, sizeof(l0_problem) * count, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(items, pl.items.data(), sizeof(int32_t) * pl.items.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(team, pl.team.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(inst_off, pl.inst_off.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, stream);
    // work counters and control blocks start at zero (a fill kernel)
    if (e == hipSuccess)
        e = l0::launch_zero(reinterpret_cast<int32_t*>(counters),
                            static_cast<int64_t>((pl.counters + pl.ctl) / sizeof(int32_t)), stream);
    const uint64_t limit = l0::wait_limit_ticks();
    for (size_t gi = 0; gi < pl.groups.size() && e == hipSuccess; ++gi) {
        const Group& g = pl.groups[gi];
        l0::BatchParams bp{};
        bp.probs = table;
        bp.items = items + g.item_start;
        bp.team = team;
        bp.inst_off = inst_off;
        bp.count = g.item_count;
        bp.rule = opts ? opts->rule : L0_RULE_L0DEC;
        bp.tol_mode = opts ? opts->tol_mode : L0_TOL_RELATIVE;
        bp.words_cap = g.words_cap;
        bp.stage_d = g.d;
        bp.results = results;
        bp.scratch = scratch;
        bp.ctl = ctl;
        bp.next = counters + gi;
        bp.timing = opts ? opts->timing : nullptr;
        bp.wait_limit = limit;
        void* args[] = {&bp};
        e = hipLaunchKernel(l0::batch_kernel_fn(pl.block_threads, g.range), dim3(static_cast<unsigned>(g.grid)),
                            dim3(static_cast<unsigned>(pl.block_threads)), args, g.lds, stream);
    }
    return from_hip(e);
}

}  // namespace

namespace l0 {

l0_status decode_batched_share(const l0_problem* probs, int32_t count, const l0_batch_opts* opts, l0_result* results,
                               void* workspace, size_t ws_bytes, hipStream_t stream, int share) {
    if (!batch_opts_ok(opts) || share < 1) return L0_ERR_ARG;
    BatchPlan pl;
    if (!problems_ok(probs, count, pl, true)) return L0_ERR_ARG;
    if (!buffer_ok(results, sizeof(l0_result) * static_cast<size_t>(count))) return L0_ERR_ARG;
    if (opts && opts->timing && !buffer_ok(opts->timing, 8 * sizeof(int64_t) * static_cast<size_t>(count)))
        return L0_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return L0_ERR_ARG;
    int bt, wc;
    resolve(opts, bt, wc);
    if (!plan_batch(probs, count, bt, wc, pl, share)) return L0_ERR_ARG;
    if (ws_bytes < pl.total) return L0_ERR_WORKSPACE;
    if (!buffer_ok(workspace, pl.total)) return L0_ERR_ARG;
    return launch_batch(probs, count, opts, pl, results, static_cast<char*>(workspace), stream);
}

}  // namespace l0

extern "C" {

size_t l0_batch_workspace_bytes(const l0_problem* probs, int32_t count, const l0_batch_opts* opts) {
    if (!batch_opts_ok(opts)) return 0;
    BatchPlan base;
    if (!problems_ok(probs, count, base, false)) return 0;
    if (opts) {
        int bt, wc;
        resolve(opts, bt, wc);
        return plan_batch(probs, count, bt, wc, base) ? base.total : 0;
    }
    size_t best = 0;
    for (const Candidate& c : kCandidates)
        if (plan_batch(probs, count, c.block_threads, c.words_cap, base)) best = std::max(best, base.total);
    return best;
}

l0_status l0_decode_batched(const l0_problem* probs, int32_t count, const l0_batch_opts* opts,
                            l0_result* results, void* workspace, size_t ws_bytes, hipStream_t stream) {
    return l0::decode_batched_share(probs, count, opts, results, workspace, ws_bytes, stream, 1);
}

l0_status l0_batch_autotune(const l0_problem* probs, int32_t count, l0_batch_opts* opts, l0_result* results,
                            void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (!opts || !batch_opts_ok(opts)) return L0_ERR_ARG;
    BatchPlan base;
    if (!problems_ok(probs, count, base, true)) return L0_ERR_ARG;
    if (!buffer_ok(results, sizeof(l0_result) * static_cast<size_t>(count))) return L0_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return L0_ERR_ARG;
    // a spread sample: every s-th instance of the processing order
    const std::vector<int32_t>& ord = base.order;
    const int32_t want = std::min<int32_t>(count, 256);
    const int32_t step = std::max<int32_t>(1, count / want);
    std::vector<l0_problem> sample;
    for (int32_t q = 0; q < count && static_cast<int32_t>(sample.size()) < want; q += step) sample.push_back(probs[ord[q]]);
    const int32_t sc = static_cast<int32_t>(sample.size());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return L0_ERR_HIP;
    float best_ms = -1.0f;
    Candidate best{0, 0};
    l0_status st = L0_OK;
    for (const Candidate& c : kCandidates) {
        BatchPlan pl;
        if (!problems_ok(sample.data(), sc, pl, false) ||
            !plan_batch(sample.data(), sc, c.block_threads, c.words_cap, pl))
            continue;
        if (pl.total > ws_bytes || !buffer_ok(workspace, pl.total)) continue;
        l0_batch_opts o = *opts;
        o.timing = nullptr;
        o.block_threads = c.block_threads;
        o.words_cap = c.words_cap;
        float ms = 1e30f;
        for (int rep = 0; rep < 2 && st == L0_OK; ++rep) {
            if (hipEventRecord(e0, stream) != hipSuccess) { st = L0_ERR_HIP; break; }
            st = launch_batch(sample.data(), sc, &o, pl, results, static_cast<char*>(workspace), stream);
            if (st != L0_OK) break;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = L0_ERR_HIP;
                break;
            }
            float t = 0.0f;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) { st = L0_ERR_HIP; break; }
            ms = std::min(ms, t);
        }
        if (st != L0_OK) break;
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != L0_OK) return st;
    if (best_ms < 0.0f) return L0_ERR_WORKSPACE;
    opts->block_threads = best.block_threads;
    opts->words_cap = best.words_cap;
    return L0_OK;
}

}  // extern "C"
