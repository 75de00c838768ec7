// C ABI runtime: handles, validation, device memory, launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
#include <cstring>
#include <vector>

#include "internal.h"
#include "layout.h"
#include "mttkrp.h"

namespace {

thread_local std::string g_err;

mttkrp_status fail(mttkrp_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

mttkrp_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return MTTKRP_EHIP;
}

constexpr uint64_t kAlign = 256;
constexpr uint32_t kMaxParts = 8192;    // partitions per launch at most, below kMaxChain-bound tensors
constexpr uint64_t kMaxChain = 4096;    // nonzeros one lane group adds in one FP32 register chain, at most
constexpr int kAlsBlocks = 512;         // row blocks of the CP-ALS reductions

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Partition cap of a tensor with nnz nonzeros (sizes its carry buffer): the
// default cap, raised where it would make a lane group's run (gsz) longer than
// kMaxChain nonzeros.  The fewest lane groups per workgroup of any launch are
// 16 (R = 64 fp32 rows, 256-thread workgroups).
uint32_t max_parts_for(uint64_t nnz)
{
    const uint64_t need = (nnz + 16 * kMaxChain - 1) / (16 * kMaxChain);
    return (uint32_t)std::max<uint64_t>(kMaxParts, need);
}

bool r_supported(int R) { return R == 16 || R == 32 || R == 64; }

struct Workspace {
    uint64_t carry = 0, grams = 0, V = 0, W = 0, part = 0, colsq = 0, lam = 0, scal = 0, job = 0, M = 0, bf16 = 0;
    uint64_t total = 0;
};

Workspace plan_workspace(const uint32_t* dims, int N, uint64_t nnz, int maxR, int dtype)
{
    Workspace w;
    uint64_t maxI = 0, sumI = 0;
    for (int m = 0; m < N; ++m) {
        maxI = std::max<uint64_t>(maxI, dims[m]);
        sumI += dims[m];
    }
    const uint64_t R = (uint64_t)maxR;
    w.carry = align_up((uint64_t)max_parts_for(nnz) * 2ull * R * 4ull);
    w.grams = align_up((uint64_t)N * R * R * 8ull);
    w.V = align_up(R * R * 8ull);
    w.W = align_up(R * R * 8ull);
    w.part = align_up((uint64_t)kAlsBlocks * R * R * 8ull);
    w.colsq = align_up(R * 8ull);
    w.lam = align_up(R * 8ull);
    w.scal = align_up(8 * 8ull);
    w.job = align_up(sizeof(mk::InvJob));
    w.M = align_up(maxI * R * 4ull);
    w.bf16 = dtype == MTTKRP_BF16 ? (uint64_t)N * kAlign + sumI * R * 2ull : 0;
    w.total = w.carry + w.grams + w.V + w.W + w.part + w.colsq + w.lam + w.scal + w.job + w.M + align_up(w.bf16);
    return w;
}

constexpr uint32_t kAssumedLds = 160 * 1024;   // gfx950 LDS per workgroup, for host-only layouts

// Rows per input mode that the partition kernel can keep in LDS: the hot rows
// of the N-1 input modes, at max_R fp32 values each, must fit next to the
// kernel's bookkeeping.
uint32_t hot_rows_for(int N, int maxR, uint32_t lds_limit, int requested)
{
    if (requested == 0) return 0;
    // Workgroups of 512 threads or more run one to a CU (registers) and own
    // its whole LDS; 256-thread ones (4+ modes) run four to a CU and get a
    // quarter each.
    const uint32_t budget = mk::partition_wg_threads(N - 1) >= 512 ? lds_limit : lds_limit / 4;
    const uint32_t fixed = mk::partition_lds_bytes(N - 1, 16, MTTKRP_FP32, 0);     // slots + bookkeeping
    const uint32_t meta = fixed - 2u * (uint32_t)(mk::partition_wg_threads(N - 1) / 4) * 16u * 4u;
    if (budget <= fixed) return 0;
    uint32_t k = (budget - meta) / ((uint32_t)(N - 1) * (uint32_t)maxR * 4u);
    if (requested > 0 && (uint32_t)requested < k) k = (uint32_t)requested;
    return k;
}

// Whether the copy of output mode n stores 16-bit input coordinates: every
// input dimension <= 65536, at most kMaxIn16 inputs, nonzero-ordered copies
// without hot rows, and the caller did not ask for 32-bit coordinates.
bool copy_idx16(const uint32_t* dims, int N, int n, const mttkrp_opts& o, uint32_t nhot)
{
    if (o.wide_indices || o.hot_steps || nhot || o.partitioner != MTTKRP_PART_NNZ || N - 1 > mk::kMaxIn16) return false;
    for (int m = 0; m < N; ++m)
        if (m != n && dims[m] > 65536u) return false;
    return true;
}

uint64_t copies_bytes(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts* o = nullptr, uint32_t nhot = 0)
{
    uint64_t b = 0;
    const uint64_t pad = (nnz + 31) / 32 * 32;
    for (int n = 0; n < N; ++n) {
        b += mk::mode_device_bytes(nnz, N, dims[n]) + (uint64_t)(N + 4) * kAlign;
        if (o && copy_idx16(dims, N, n, *o, nhot)) b -= pad * 2ull * (uint64_t)(N - 1);   // half-width coordinates
    }
    return b;
}

uint64_t hot_bytes(int N, uint32_t nhot)
{
    return (uint64_t)N * (align_up((uint64_t)nhot * 4ull) + kAlign);
}

}  // namespace

struct mttkrp_layout {
    int N = 0;
    uint32_t dims[MTTKRP_MAX_MODES] = {};
    uint64_t nnz = 0;
    mttkrp_opts opts{};
    int device = 0;
    int cu_count = 256;
    bool host_only = false;
    std::vector<mk::HostMode> host;
    std::vector<mk::HotSet> hot;                       // host-only handles
    uint32_t nhot = 0;                                 // hot rows per input mode
    uint32_t lds_limit = 0;                            // LDS bytes per workgroup on the device
    const uint32_t* hot_rows[MTTKRP_MAX_MODES] = {};   // device tables, slot -> row, per mode
    mk::DevMode dev[MTTKRP_MAX_MODES];
    void* dmem = nullptr;
    uint64_t dbytes = 0;
    bool owns_mem = true;                              // false: dmem is the caller's (mttkrp_layout_build_in)
    float* carry = nullptr;
    mk::AlsWork als;
    mk::InvJob inv_job_host{};                         // host source of als.job (kept alive for the copy)
    double normX2 = 0.0;
    int als_R = 0;
    std::vector<std::vector<uint32_t>> new_of_old;     // relabel: per mode, the new index of each old one
};

// Degree relabelling: per mode, indices renumbered by decreasing nonzero
// count (ties: the lower index first); `out` receives the COO tensor in the
// new numbering and `perm[m][old] = new`.
static void relabel_by_degree(const uint32_t* coo, uint64_t nnz, const uint32_t* dims, int N,
                              std::vector<uint32_t>& out, std::vector<std::vector<uint32_t>>& perm)
{
    perm.assign(N, {});
    for (int m = 0; m < N; ++m) {
        std::vector<uint64_t> deg(dims[m], 0);
        for (uint64_t k = 0; k < nnz; ++k) ++deg[coo[k * N + m]];
        std::vector<uint32_t> order(dims[m]);
        for (uint32_t i = 0; i < dims[m]; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return deg[a] > deg[b]; });
        perm[m].resize(dims[m]);
        for (uint32_t r = 0; r < dims[m]; ++r) perm[m][order[r]] = r;
    }
    out.resize((size_t)nnz * N);
    for (uint64_t k = 0; k < nnz; ++k)
        for (int m = 0; m < N; ++m) out[k * N + m] = perm[m][coo[k * N + m]];
}

extern "C" {

void mttkrp_opts_default(mttkrp_opts* o)
{
    if (!o) return;
    o->parts_per_cu = 8;
    o->factor_dtype = MTTKRP_FP32;
    o->max_R = 64;
    o->hbm_budget_bytes = 0;
    o->host_only = 0;
    o->hot_rows = 0;
    o->build_on_host = 0;
    o->partitioner = MTTKRP_PART_NNZ;
    o->lpt_parts = 0;
    o->hot_steps = 0;
    o->wide_indices = 0;
    o->part_threads = 0;
    o->part_gathers = 0;
    o->relabel = 0;
    o->als_solve = 0;
}

const char* mttkrp_last_error(void) { return g_err.c_str(); }

static mttkrp_status check_opts(const mttkrp_opts* in, mttkrp_opts* o)
{
    mttkrp_opts_default(o);
    if (in) *o = *in;
    if (o->parts_per_cu <= 0) o->parts_per_cu = 8;
    if (o->max_R == 0) o->max_R = 64;
    if (!r_supported(o->max_R)) return fail(MTTKRP_EUNSUPPORTED, "max_R must be 16, 32 or 64");
    if (o->factor_dtype != MTTKRP_FP32 && o->factor_dtype != MTTKRP_BF16)
        return fail(MTTKRP_EINVAL, "factor_dtype must be MTTKRP_FP32 or MTTKRP_BF16");
    if (o->partitioner != MTTKRP_PART_NNZ && o->partitioner != MTTKRP_PART_ROWS_LPT)
        return fail(MTTKRP_EINVAL, "partitioner must be MTTKRP_PART_NNZ or MTTKRP_PART_ROWS_LPT");
    if (o->lpt_parts < 0 || o->lpt_parts > (1 << 20)) return fail(MTTKRP_EINVAL, "lpt_parts must be in [0, 2^20]");
    if (o->hot_steps != 0 && o->hot_steps != 1) return fail(MTTKRP_EINVAL, "hot_steps must be 0 or 1");
    if (o->part_threads < 0 || o->part_gathers < 0 ||
        ((o->part_threads || o->part_gathers) &&
         !mk::tuned_shape_supported(o->part_threads ? o->part_threads : 512, o->part_gathers ? o->part_gathers : 4)))
        return fail(MTTKRP_EINVAL, "part_threads must be 0, 256, 512 or 1024 and part_gathers 0, 2 or 4");
    if (o->relabel != 0 && o->relabel != 1) return fail(MTTKRP_EINVAL, "relabel must be 0 or 1");
    if (o->als_solve != 0 && o->als_solve != 1) return fail(MTTKRP_EINVAL, "als_solve must be 0 or 1");
    if (o->hot_steps) {
        o->partitioner = MTTKRP_PART_NNZ;   // step copies carry their own hot rows and partitions
        o->hot_rows = 0;
    }
    if (o->partitioner == MTTKRP_PART_ROWS_LPT) o->hot_rows = 0;   // scheme-1 copies keep plain coordinates
    return MTTKRP_OK;
}

// Scheme-1 partitions of a build (the caller's count, else one per compute unit).
static uint32_t lpt_kappa(const mttkrp_opts& o, int cu_count)
{
    return o.lpt_parts > 0 ? (uint32_t)o.lpt_parts : (uint32_t)(cu_count > 0 ? cu_count : 256);
}

// Extra device bytes of scheme-1 copies (gaps between partitions and the
// partition tables of the N copies); 0 for the nonzero split.  Before the
// device is known, a compute-unit count of 1024 bounds the default kappa.
static uint64_t lpt_bytes(const mttkrp_opts& o, int N, int cu_count)
{
    if (o.partitioner != MTTKRP_PART_ROWS_LPT) return 0;
    const uint32_t kappa = lpt_kappa(o, cu_count > 0 ? cu_count : 1024);
    return (uint64_t)N * (mk::lpt_extra_bytes(N, kappa) + 4 * kAlign);
}

// Hot rows per input of a hot-steps layout: as many rows of max_R values of
// the factor dtype as fit in the step kernel's LDS beside its wave partials,
// less one zero row.
static uint32_t step_hot_rows(int N, int maxR, int dtype, uint32_t lds_limit)
{
    const int es = dtype == MTTKRP_FP32 ? 4 : 2;
    const uint32_t row = (uint32_t)(N - 1) * (uint32_t)maxR * (uint32_t)es;
    const uint32_t partials = mk::step_kernel_lds_bytes(N - 1, maxR, es, 0) - row;
    if (lds_limit <= partials + 2 * row) return 0;
    return (lds_limit - partials) / row - 1;
}

// Device bytes of the N hot-steps copies (an upper bound: every output row
// padded by up to one step).
static uint64_t step_copies_bytes(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts& o)
{
    const uint32_t P = mk::step_entries(o.max_R, o.factor_dtype);
    uint64_t b = 0;
    for (int n = 0; n < N; ++n) {
        const uint64_t steps = mk::step_copy_steps_bound(nnz, std::min<uint64_t>(nnz, dims[n]), P);
        b += steps * P * 4ull * (uint64_t)N + steps / 32 * 8 + (uint64_t)dims[n] * 4 + (uint64_t)(N + 4) * kAlign;
    }
    return b;
}

static uint64_t layout_copies_bytes(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts& o, uint32_t nhot)
{
    return o.hot_steps ? step_copies_bytes(dims, N, nnz, o) : copies_bytes(dims, N, nnz, &o, nhot);
}

static uint32_t layout_hot_rows(int N, const mttkrp_opts& o, uint32_t lds_limit)
{
    return o.hot_steps ? step_hot_rows(N, o.max_R, o.factor_dtype, lds_limit)
                       : hot_rows_for(N, o.max_R, lds_limit, o.hot_rows);
}

mttkrp_status mttkrp_footprint(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts* opts, uint64_t* bytes)
{
    g_err.clear();
    if (!dims || !bytes) return fail(MTTKRP_EINVAL, "dims and bytes must not be NULL");
    if (N < 3 || N > MTTKRP_MAX_MODES) return fail(MTTKRP_EUNSUPPORTED, "N must be between 3 and 8");
    for (int m = 0; m < N; ++m)
        if (dims[m] == 0 || dims[m] > 0x7fffffffu) return fail(MTTKRP_EINVAL, "dims must be in [1, 2^31-1]");
    mttkrp_opts o;
    mttkrp_status s = check_opts(opts, &o);
    if (s) return s;
    const uint32_t nhot_fp = layout_hot_rows(N, o, kAssumedLds);
    *bytes = layout_copies_bytes(dims, N, nnz, o, nhot_fp) + plan_workspace(dims, N, nnz, o.max_R, o.factor_dtype).total +
             hot_bytes(N, nhot_fp) + lpt_bytes(o, N, 0);
    return MTTKRP_OK;
}

}  // extern "C"

// The build behind mttkrp_layout_build (ext_mem == NULL: the handle allocates
// and owns its device memory, and a device build allocates its own scratch)
// and mttkrp_layout_build_in (the caller's memory and scratch; no allocation).
static mttkrp_status build_impl(const uint32_t* coo_idx, const float* vals, uint64_t nnz, const uint32_t* dims, int N,
                                const mttkrp_opts* opts, void* ext_mem, uint64_t ext_bytes, void* ext_scratch,
                                uint64_t ext_scratch_bytes, hipStream_t stream, mttkrp_handle* out)
{
    if (!out) return fail(MTTKRP_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    if (N < 3 || N > MTTKRP_MAX_MODES) return fail(MTTKRP_EUNSUPPORTED, "N must be between 3 and 8");
    if (nnz && !vals) return fail(MTTKRP_EINVAL, "vals is NULL");
    mttkrp_opts o;
    mttkrp_status s = check_opts(opts, &o);
    if (s) return s;
    bool range_err = false;
    std::string msg = mk::validate_coo(coo_idx, nnz, dims, N, &range_err);
    if (!msg.empty()) return fail(range_err ? MTTKRP_ERANGE : MTTKRP_EINVAL, msg);
    // Degree relabelling: every later step sees the tensor in the new numbering.
    std::vector<uint32_t> relabelled;
    std::vector<std::vector<uint32_t>> new_of_old;
    if (o.relabel) {
        relabel_by_degree(coo_idx, nnz, dims, N, relabelled, new_of_old);
        coo_idx = relabelled.data();
    }

    // Admission first, before any device call (the hot tables are sized for the
    // largest LDS, an upper bound).
    {
        const uint32_t nhot_b = layout_hot_rows(N, o, kAssumedLds);
        const uint64_t bound = layout_copies_bytes(dims, N, nnz, o, nhot_b) +
                               plan_workspace(dims, N, nnz, o.max_R, o.factor_dtype).total +
                               hot_bytes(N, nhot_b) + lpt_bytes(o, N, 0);
        if (!o.host_only && o.hbm_budget_bytes && bound > o.hbm_budget_bytes)
            return fail(MTTKRP_ENOMEM, "footprint " + std::to_string(bound) + " B exceeds the budget of " +
                                           std::to_string(o.hbm_budget_bytes) + " B");
    }
    uint32_t lds_limit = kAssumedLds;
    int dev_id = 0;
    if (!o.host_only) {
        hipError_t e0 = hipGetDevice(&dev_id);
        if (e0 != hipSuccess) return hip_fail(e0, "hipGetDevice");
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id) == hipSuccess && v > 0)
            lds_limit = (uint32_t)v;
    }
    if (o.hot_steps && (N < 3 || N > 4)) return fail(MTTKRP_EUNSUPPORTED, "hot_steps supports 3- and 4-mode tensors");
    const uint32_t nhot = layout_hot_rows(N, o, lds_limit);
    int cus_here = 256;
    if (!o.host_only) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev_id) == hipSuccess && v > 0)
            cus_here = v;
    }
    const bool lpt = o.partitioner == MTTKRP_PART_ROWS_LPT;
    const uint32_t kappa = lpt_kappa(o, cus_here);
    const uint64_t need = layout_copies_bytes(dims, N, nnz, o, nhot) +
                          plan_workspace(dims, N, nnz, o.max_R, o.factor_dtype).total + hot_bytes(N, nhot) +
                          lpt_bytes(o, N, cus_here);
    const uint32_t step_P = o.hot_steps ? mk::step_entries(o.max_R, o.factor_dtype) : 0u;

    auto* h = new mttkrp_layout();
    h->N = N;
    for (int m = 0; m < N; ++m) h->dims[m] = dims[m];
    h->nnz = nnz;
    h->opts = o;
    h->host_only = o.host_only != 0;
    h->nhot = nhot;
    h->lds_limit = lds_limit;
    h->device = dev_id;
    h->new_of_old = std::move(new_of_old);

    const int threads = mk::host_threads();
    std::vector<mk::HotSet> hot = mk::select_hot_rows(coo_idx, nnz, dims, N, nhot);
    mk::BuildScratch scratch;
    if (h->host_only) {
        h->host.resize(N);
        for (int n = 0; n < N; ++n) {
            mk::build_host_mode(coo_idx, vals, nnz, dims, N, n, !o.hot_steps, threads, &hot, h->host[n], &scratch);
            if (lpt) mk::lpt_regroup(h->host[n], kappa);
            if (step_P) {
                // The view shows the step copy: its arrays replace the nonzero-ordered ones.
                mk::StepCopy sc;
                mk::build_step_copy(h->host[n], step_P, nhot, threads, sc);
                mk::HostMode& hm = h->host[n];
                hm.idx = std::move(sc.idx);
                hm.val = std::move(sc.val);
                hm.winfo = std::move(sc.winfo);
                hm.nnz_pad = sc.nsteps_pad * step_P;
                hm.step_P = step_P;
                hm.nsteps = sc.nsteps;
            }
        }
        for (auto& hs : hot) hs.rows.resize(nhot, 0u);
        h->hot = std::move(hot);
        *out = h;
        return MTTKRP_OK;
    }

    hipError_t e = hipSuccess;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
        h->cu_count = cus;
    if (ext_mem) {
        if (ext_bytes < need) {
            delete h;
            return fail(MTTKRP_EINVAL, "dev_mem holds " + std::to_string(ext_bytes) + " B; the layout needs " +
                                           std::to_string(need) + " B (mttkrp_footprint)");
        }
        h->dmem = ext_mem;
        h->owns_mem = false;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > free_b) {
            delete h;
            return fail(MTTKRP_ENOMEM, "footprint " + std::to_string(need) + " B exceeds free device memory (" +
                                           std::to_string(free_b) + " B)");
        }
        e = hipMalloc(&h->dmem, need);
        if (e != hipSuccess) {
            h->dmem = nullptr;
            delete h;
            (void)hipGetLastError();
            return fail(MTTKRP_ENOMEM, "hipMalloc of " + std::to_string(need) + " B failed");
        }
    }
    h->dbytes = need;
    // Releases the device memory of a handle that failed to build (the caller's is left alone).
    auto drop = [&]() {
        if (h->owns_mem) (void)hipFree(h->dmem);
        delete h;
    };
    char* base = static_cast<char*>(h->dmem);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> void* {
        void* p = base + off;
        off += align_up(bytes);
        return p;
    };
    // Workspace.
    const Workspace ws = plan_workspace(dims, N, nnz, o.max_R, o.factor_dtype);
    h->carry = static_cast<float*>(take(ws.carry));
    h->als.grams = static_cast<double*>(take(ws.grams));
    h->als.V = static_cast<double*>(take(ws.V));
    h->als.W = static_cast<double*>(take(ws.W));
    h->als.part = static_cast<double*>(take(ws.part));
    h->als.colsq = static_cast<double*>(take(ws.colsq));
    h->als.lam = static_cast<double*>(take(ws.lam));
    h->als.scal = static_cast<double*>(take(ws.scal));
    h->als.job = static_cast<mk::InvJob*>(take(ws.job));
    h->inv_job_host = mk::InvJob{h->als.grams, h->als.V, h->als.W, h->als.scal + 1};
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->als.job, &h->inv_job_host, sizeof(mk::InvJob), hipMemcpyHostToDevice, stream);
    h->als.M = static_cast<float*>(take(ws.M));
    h->als.max_blocks = kAlsBlocks;
    if (o.factor_dtype == MTTKRP_BF16)
        for (int m = 0; m < N; ++m) h->als.bf16[m] = static_cast<uint16_t*>(take((uint64_t)dims[m] * o.max_R * 2));

    // Hot-row tables (padded to nhot entries; unused slots name row 0).
    for (int m = 0; m < N; ++m) {
        std::vector<uint32_t>& rows = hot[m].rows;
        rows.resize(nhot, 0u);
        void* dst = take(nhot ? (uint64_t)nhot * 4 : 4);
        if (nhot && e == hipSuccess) e = hipMemcpyAsync(dst, rows.data(), (uint64_t)nhot * 4, hipMemcpyHostToDevice, stream);
        h->hot_rows[m] = static_cast<const uint32_t*>(dst);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);

    double normX2 = 0.0;
    // With the caller's memory the device build runs only in the caller's scratch.
    const bool dev_build = !o.build_on_host && !lpt && !o.hot_steps && nhot == 0 && mk::device_build_applies(dims, N, nnz) &&
                           (!ext_mem || (ext_scratch && ext_scratch_bytes >= mk::device_build_scratch_bytes(dims, N, nnz)));
    if (e == hipSuccess && dev_build) {
        // Mode copies sorted and laid out on the device.
        const uint64_t nnz_pad = (nnz + 31) / 32 * 32;
        std::vector<mk::DeviceModeSlots> slots(N);
        for (int n = 0; n < N; ++n) {
            slots[n].idx16 = copy_idx16(dims, N, n, o, nhot);
            for (int j = 0; j < N - 1; ++j)
                slots[n].idx[j] = static_cast<uint32_t*>(take(nnz_pad * (slots[n].idx16 ? 2 : 4)));
            slots[n].val = static_cast<float*>(take(nnz_pad * 4));
            slots[n].winfo = static_cast<uint2*>(take(nnz_pad / 32 * 8));
            slots[n].rows = static_cast<uint32_t*>(take((uint64_t)dims[n] * 4));
        }
        if (off > need) {
            drop();
            return fail(MTTKRP_EHIP, "internal: mode copies exceed the planned device footprint");
        }
        std::vector<mk::DevMode> modes;
        e = mk::build_device_modes(coo_idx, vals, nnz, dims, N, slots, modes, &normX2, ext_mem ? ext_scratch : nullptr,
                                   ext_mem ? ext_scratch_bytes : 0, stream);
        if (e == hipSuccess)
            for (int n = 0; n < N; ++n) h->dev[n] = modes[n];
    }
    else {
        // Mode copies: built on the host one mode at a time into the same buffers, uploaded.
        mk::HostMode hm;
        for (int n = 0; n < N && e == hipSuccess; ++n) {
            mk::build_host_mode(coo_idx, vals, nnz, dims, N, n, false, threads, &hot, hm, &scratch);
            if (n == 0) {
                // |X|^2 with duplicate coordinates merged: duplicates are adjacent in
                // the sorted copy (no row start between them, same other indices).
                uint64_t k = 0;
                while (k < nnz) {
                    double v = hm.val[k];
                    uint64_t j = k + 1;
                    while (j < nnz && !((hm.winfo[2 * (j / 32)] >> (j % 32)) & 1u)) {
                        bool same = true;
                        for (int t = 0; t < N - 1 && same; ++t) same = hm.idx[t][j] == hm.idx[t][k];
                        if (!same) break;
                        v += hm.val[j];
                        ++j;
                    }
                    normX2 += v * v;
                    k = j;
                }
            }
            if (lpt) mk::lpt_regroup(hm, kappa);
            if (step_P) {
                mk::StepCopy sc;
                mk::build_step_copy(hm, step_P, nhot, threads, sc);
                hm.idx = std::move(sc.idx);
                hm.val = std::move(sc.val);
                hm.winfo = std::move(sc.winfo);
                hm.nnz_pad = sc.nsteps_pad * step_P;
                hm.step_P = step_P;
                hm.nsteps = sc.nsteps;
            }
            mk::DevMode& d = h->dev[n];
            d.nnz = hm.nnz;
            d.nnz_pad = hm.nnz_pad;
            d.nrows_nz = hm.nrows_nz;
            d.nempty = hm.nempty;
            d.n_in = N - 1;
            auto up = [&](const void* src, uint64_t bytes) -> void* {
                void* dst = take(bytes ? bytes : 4);
                if (bytes && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
                return dst;
            };
            d.idx16 = copy_idx16(dims, N, n, o, nhot);
            std::vector<uint16_t> narrow;
            for (int j = 0; j < N - 1; ++j) {
                d.in_modes[j] = hm.in_modes[j];
                d.in_dims[j] = dims[hm.in_modes[j]];
                if (d.idx16) {
                    // 16-bit coordinates; the copy waits for this upload before
                    // the buffer is refilled for the next input
                    narrow.assign(hm.idx[j].begin(), hm.idx[j].begin() + hm.nnz_pad);
                    d.idx[j] = static_cast<const uint32_t*>(up(narrow.data(), hm.nnz_pad * 2));
                    if (e == hipSuccess) e = hipStreamSynchronize(stream);
                } else {
                    d.idx[j] = static_cast<const uint32_t*>(up(hm.idx[j].data(), hm.nnz_pad * 4));
                }
            }
            d.val = static_cast<const float*>(up(hm.val.data(), hm.nnz_pad * 4));
            d.winfo = static_cast<const uint2*>(up(hm.winfo.data(), hm.winfo.size() * 4));
            d.row_id = static_cast<const uint32_t*>(up(hm.row_id.data(), hm.row_id.size() * 4));
            d.empty_rows = static_cast<const uint32_t*>(up(hm.empty_rows.data(), hm.empty_rows.size() * 4));
            if (lpt) {
                d.prange = static_cast<const uint64_t*>(up(hm.part_range.data(), hm.part_range.size() * 8));
                d.nprange = kappa;
            }
            d.step_P = hm.step_P;
            d.nsteps = hm.nsteps;
            // The next mode overwrites the host arrays; wait for the copies that read them.
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
        }
    }
    h->normX2 = normX2;
    if (e == hipSuccess && off > need) {
        drop();
        return fail(MTTKRP_EHIP, "internal: mode copies exceed the planned device footprint");
    }
    if (e != hipSuccess) {
        mttkrp_status st = hip_fail(e, "uploading the mode copies");
        drop();
        return st;
    }
    *out = h;
    return MTTKRP_OK;
}

extern "C" {

mttkrp_status mttkrp_layout_build(const uint32_t* coo_idx, const float* vals, uint64_t nnz, const uint32_t* dims,
                                  int N, const mttkrp_opts* opts, hipStream_t stream, mttkrp_handle* out)
{
    g_err.clear();
    return build_impl(coo_idx, vals, nnz, dims, N, opts, nullptr, 0, nullptr, 0, stream, out);
}

mttkrp_status mttkrp_build_scratch_bytes(const uint32_t* dims, int N, uint64_t nnz, const mttkrp_opts* opts,
                                         uint64_t* bytes)
{
    g_err.clear();
    if (!dims || !bytes) return fail(MTTKRP_EINVAL, "dims and bytes must not be NULL");
    if (N < 3 || N > MTTKRP_MAX_MODES) return fail(MTTKRP_EUNSUPPORTED, "N must be between 3 and 8");
    for (int m = 0; m < N; ++m)
        if (dims[m] == 0 || dims[m] > 0x7fffffffu) return fail(MTTKRP_EINVAL, "dims must be in [1, 2^31-1]");
    mttkrp_opts o;
    mttkrp_status s = check_opts(opts, &o);
    if (s) return s;
    *bytes = (!o.build_on_host && o.hot_rows == 0) ? mk::device_build_scratch_bytes(dims, N, nnz) : 0;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_layout_build_in(const uint32_t* coo_idx, const float* vals, uint64_t nnz, const uint32_t* dims,
                                     int N, const mttkrp_opts* opts, void* dev_mem, uint64_t dev_bytes,
                                     void* dev_scratch, uint64_t scratch_bytes, hipStream_t stream, mttkrp_handle* out)
{
    g_err.clear();
    if (!dev_mem || reinterpret_cast<uintptr_t>(dev_mem) % kAlign)
        return fail(MTTKRP_EINVAL, "dev_mem must be a 256-byte aligned device pointer");
    if (dev_scratch && reinterpret_cast<uintptr_t>(dev_scratch) % kAlign)
        return fail(MTTKRP_EINVAL, "dev_scratch must be 256-byte aligned");
    if (opts && opts->host_only) return fail(MTTKRP_EINVAL, "host_only layouts hold no device memory");
    return build_impl(coo_idx, vals, nnz, dims, N, opts, dev_mem, dev_bytes, dev_scratch, scratch_bytes, stream, out);
}

uint64_t mttkrp_layout_bytes(mttkrp_handle h) { return h ? h->dbytes : 0; }

// The partition kernel's shape on this handle for n_in inputs, rank R and
// dtype: the handle's part_threads / part_gathers where a tuned shape applies
// (3-mode tensors, fp32 factors, no hot rows), else the default.
static void part_shape(const mttkrp_layout* h, int n_in, int R, int dtype, int* threads, int* gathers)
{
    mk::default_part_shape(n_in, R, dtype, threads, gathers);
    if (n_in == 2 && dtype == MTTKRP_FP32 && h->nhot == 0 && !h->opts.hot_steps) {
        if (h->opts.part_threads) *threads = h->opts.part_threads;
        if (h->opts.part_gathers) *gathers = h->opts.part_gathers;
    }
}

// Nonzero partitions of one mode copy of nnz nonzeros on this handle, with
// its launch shape (the tuned fields set only where they differ from the default).
static mk::Geometry plan_nnz(const mttkrp_layout* h, uint64_t nnz, int n_in, int R, int dtype)
{
    int th = 0, gu = 0, dth = 0, dgu = 0;
    part_shape(h, n_in, R, dtype, &th, &gu);
    mk::default_part_shape(n_in, R, dtype, &dth, &dgu);
    mk::Geometry g =
        mk::plan_geometry(nnz, n_in, R, dtype, h->opts.parts_per_cu * h->cu_count, max_parts_for(h->nnz), kMaxChain, th);
    if (th != dth || gu != dgu) {
        g.threads = th;
        g.gathers = gu;
    }
    return g;
}

mttkrp_status mttkrp_layout_info(mttkrp_handle h, mttkrp_info* info)
{
    g_err.clear();
    if (!h || !info) return fail(MTTKRP_EINVAL, "NULL handle or info");
    info->cu_count = (uint32_t)h->cu_count;
    info->lds_per_workgroup = h->lds_limit;
    info->hot_rows = h->nhot;
    int th = 0, gu = 0;
    part_shape(h, h->N - 1, h->opts.max_R, MTTKRP_FP32, &th, &gu);
    info->wg_threads = (uint32_t)(h->opts.hot_steps ? mk::step_wg_threads() : th);
    info->gathers_in_flight = h->opts.hot_steps ? 0u : (uint32_t)gu;
    info->parts_per_cu = (uint32_t)h->opts.parts_per_cu;
    info->lpt_parts = h->opts.partitioner == MTTKRP_PART_ROWS_LPT ? lpt_kappa(h->opts, h->cu_count) : 0u;
    info->step_entries = h->opts.hot_steps ? mk::step_entries(h->opts.max_R, h->opts.factor_dtype) : 0u;
    info->idx16_modes = 0u;
    for (int n = 0; n < h->N; ++n)
        if (h->host_only ? copy_idx16(h->dims, h->N, n, h->opts, h->nhot) : h->dev[n].idx16) info->idx16_modes |= 1u << n;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_layout_perm(mttkrp_handle h, int mode, uint32_t* new_of_old)
{
    g_err.clear();
    if (!h || !new_of_old) return fail(MTTKRP_EINVAL, "NULL handle or output");
    if (mode < 0 || mode >= h->N) return fail(MTTKRP_EINVAL, "mode out of range");
    if (h->new_of_old.empty()) return fail(MTTKRP_EINVAL, "the layout was built without relabel");
    std::copy(h->new_of_old[mode].begin(), h->new_of_old[mode].end(), new_of_old);
    return MTTKRP_OK;
}

mttkrp_status mttkrp_lpt_partition(const uint64_t* loads, uint64_t nrows, uint32_t kappa, uint32_t* part,
                                   uint64_t* part_load)
{
    g_err.clear();
    if (kappa == 0) return fail(MTTKRP_EINVAL, "kappa must be at least 1");
    if (nrows && (!loads || !part)) return fail(MTTKRP_EINVAL, "NULL loads or part");
    std::vector<uint64_t> pl;
    const std::vector<uint32_t> p = mk::lpt_assign(loads, nrows, kappa, &pl);
    std::copy(p.begin(), p.end(), part);
    if (part_load) std::copy(pl.begin(), pl.end(), part_load);
    return MTTKRP_OK;
}

mttkrp_status mttkrp_launch_plan(uint64_t nnz, int N, int R, int factor_dtype, int parts_per_cu, uint32_t cu_count,
                                 mttkrp_plan* out)
{
    g_err.clear();
    if (!out) return fail(MTTKRP_EINVAL, "NULL out");
    if (N < 3 || N > MTTKRP_MAX_MODES) return fail(MTTKRP_EUNSUPPORTED, "N must be between 3 and 8");
    if (!r_supported(R)) return fail(MTTKRP_EUNSUPPORTED, "R must be 16, 32 or 64");
    if (factor_dtype != MTTKRP_FP32 && factor_dtype != MTTKRP_BF16)
        return fail(MTTKRP_EINVAL, "factor_dtype must be MTTKRP_FP32 or MTTKRP_BF16");
    if (nnz >= (1ull << 32)) return fail(MTTKRP_EINVAL, "nnz must be below 2^32");
    if (parts_per_cu <= 0) parts_per_cu = 8;
    if (cu_count == 0) cu_count = 256;
    const mk::Geometry g =
        mk::plan_geometry(nnz, N - 1, R, factor_dtype, parts_per_cu * (int)cu_count, max_parts_for(nnz), kMaxChain);
    out->wg_threads = (uint32_t)mk::partition_wg_threads(N - 1);
    out->lane_groups = (uint32_t)g.groups;
    out->lanes_per_group = (uint32_t)g.lanes;
    out->nonzeros_per_group = g.gsz;
    out->nonzeros_per_part = g.wgc;
    out->nparts = nnz ? g.nparts : 0;
    out->carry_bytes = (uint64_t)max_parts_for(nnz) * 2ull * (uint64_t)R * 4ull;
    return MTTKRP_OK;
}

void mttkrp_layout_free(mttkrp_handle h)
{
    if (!h) return;
    if (h->dmem && h->owns_mem) {
        (void)hipDeviceSynchronize();
        (void)hipFree(h->dmem);
    }
    delete h;
}

mttkrp_status mttkrp_layout_view(mttkrp_handle h, int mode, mttkrp_mode_view* v)
{
    g_err.clear();
    if (!h || !v) return fail(MTTKRP_EINVAL, "NULL handle or view");
    if (!h->host_only) return fail(MTTKRP_EINVAL, "views exist only for host-only handles");
    if (mode < 0 || mode >= h->N) return fail(MTTKRP_EINVAL, "mode out of range");
    const mk::HostMode& m = h->host[mode];
    memset(v, 0, sizeof(*v));
    v->nnz = m.nnz;
    v->nnz_pad = m.nnz_pad;
    v->nrows_nz = m.nrows_nz;
    v->nempty = m.nempty;
    v->n_in = (int)m.in_modes.size();
    for (int j = 0; j < v->n_in; ++j) {
        v->in_modes[j] = m.in_modes[j];
        v->idx[j] = m.idx[j].data();
    }
    v->val = m.val.data();
    v->winfo = m.winfo.data();
    v->row_id = m.row_id.data();
    v->empty_rows = m.empty_rows.data();
    v->src_pos = m.src_pos.data();
    v->nhot = h->nhot;
    for (int j = 0; j < v->n_in; ++j) v->hot_rows[j] = h->hot[m.in_modes[j]].rows.data();
    v->step_entries = m.step_P;
    v->nsteps = m.nsteps;
    v->nparts = m.part_range.size() / 2;
    v->part_range = m.part_range.empty() ? nullptr : m.part_range.data();
    return MTTKRP_OK;
}

static mttkrp_status check_run(mttkrp_handle h, int mode, const void* const* factors, const float* out, int R)
{
    if (!h) return fail(MTTKRP_EINVAL, "NULL handle");
    if (h->host_only) return fail(MTTKRP_EINVAL, "host-only handle: build without host_only to run");
    if (mode < 0 || mode >= h->N) return fail(MTTKRP_EINVAL, "mode out of range");
    if (!r_supported(R)) return fail(MTTKRP_EUNSUPPORTED, "R must be 16, 32 or 64");
    if (R > h->opts.max_R) return fail(MTTKRP_EINVAL, "R exceeds the handle's max_R");
    if (!factors || !out) return fail(MTTKRP_EINVAL, "NULL factors or out");
    if (reinterpret_cast<uintptr_t>(out) % 16) return fail(MTTKRP_EINVAL, "out must be 16-byte aligned");
    for (int m = 0; m < h->N; ++m)
        if ((uint64_t)h->dims[m] * (uint64_t)R * 4ull >= 0xFFFFFFF0ull)
            return fail(MTTKRP_EUNSUPPORTED, "factor " + std::to_string(m) + " is 4 GiB or larger");
    for (int m = 0; m < h->N; ++m) {
        if (m == mode) continue;
        if (!factors[m]) return fail(MTTKRP_EINVAL, "factor " + std::to_string(m) + " is NULL");
        if (reinterpret_cast<uintptr_t>(factors[m]) % 16)
            return fail(MTTKRP_EINVAL, "factor " + std::to_string(m) + " must be 16-byte aligned");
    }
    return MTTKRP_OK;
}

// Launch plan of one mode's MTTKRP on this handle (nonzero partitions, or
// wave steps for hot-steps copies, which run at the layout's rank and dtype only).
static mttkrp_status plan_for(mttkrp_handle h, const mk::DevMode& d, int R, int dtype, mk::Geometry* g)
{
    if (d.step_P) {
        if (R != h->opts.max_R || dtype != h->opts.factor_dtype)
            return fail(MTTKRP_EUNSUPPORTED, "this handle's copies are laid out in wave steps for R=" +
                                                 std::to_string(h->opts.max_R) + " and " +
                                                 (h->opts.factor_dtype == MTTKRP_FP32 ? "fp32" : "bf16") +
                                                 " factors only");
        *g = mk::plan_step_geometry(d.nsteps, R, dtype, d.step_P, h->opts.parts_per_cu * h->cu_count,
                                    max_parts_for(h->nnz), kMaxChain, (uint32_t)h->cu_count);
        return MTTKRP_OK;
    }
    *g = plan_nnz(h, d.nnz, d.n_in, R, dtype);
    return MTTKRP_OK;
}

static mttkrp_status run_mode(mttkrp_handle h, int mode, const void* const* factors, int dtype, float* out, int R,
                              hipStream_t stream)
{
    const mk::DevMode& d = h->dev[mode];
    const void* fac[mk::kMaxIn];
    const uint32_t* hot[mk::kMaxIn];
    for (int j = 0; j < d.n_in; ++j) {
        fac[j] = factors[d.in_modes[j]];
        hot[j] = h->hot_rows[d.in_modes[j]];
    }
    mk::Geometry g;
    mttkrp_status ps = plan_for(h, d, R, dtype, &g);
    if (ps) return ps;
    hipError_t e = mk::launch_mttkrp(d, R, dtype, fac, hot, h->nhot, out, h->carry, g, stream);
    if (e != hipSuccess) return hip_fail(e, "MTTKRP launch");
    return MTTKRP_OK;
}

mttkrp_status mttkrp_run(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                         hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = check_run(h, mode, reinterpret_cast<const void* const*>(factors), out, R);
    if (s) return s;
    return run_mode(h, mode, reinterpret_cast<const void* const*>(factors), MTTKRP_FP32, out, R, stream);
}

}  // extern "C"

mttkrp_status mk::set_error(mttkrp_status s, const char* msg) { return fail(s, msg); }

mttkrp_status mk::run_fp32_with_carry(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                      int device, float* carry, uint64_t carry_bytes, hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = check_run(h, mode, reinterpret_cast<const void* const*>(factors), out, R);
    if (s) return s;
    if (h->device != device)
        return fail(MTTKRP_EINVAL, "the current device (" + std::to_string(device) + ") is not the handle's (" +
                                       std::to_string(h->device) + ")");
    const mk::DevMode& d = h->dev[mode];
    const void* fac[mk::kMaxIn];
    const uint32_t* hot[mk::kMaxIn];
    for (int j = 0; j < d.n_in; ++j) {
        fac[j] = factors[d.in_modes[j]];
        hot[j] = h->hot_rows[d.in_modes[j]];
    }
    mk::Geometry g;
    mttkrp_status ps = plan_for(h, d, R, MTTKRP_FP32, &g);
    if (ps) return ps;
    const uint64_t need = (uint64_t)g.nparts * 2ull * (uint64_t)R * sizeof(float);
    if (need > carry_bytes)
        return fail(MTTKRP_ENOMEM, "this launch needs " + std::to_string(need) + " B of carry rows (" +
                                       std::to_string(g.nparts) + " partitions at R=" + std::to_string(R) +
                                       "); the static scratch holds " + std::to_string(carry_bytes) + " B");
    hipError_t e = mk::launch_mttkrp(d, R, MTTKRP_FP32, fac, hot, h->nhot, out, carry, g, stream);
    if (e != hipSuccess) return hip_fail(e, "MTTKRP launch");
    return MTTKRP_OK;
}

extern "C" {

mttkrp_status mttkrp_run_bf16(mttkrp_handle h, int mode, const uint16_t* const* factors, float* out, int R,
                              hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = check_run(h, mode, reinterpret_cast<const void* const*>(factors), out, R);
    if (s) return s;
    return run_mode(h, mode, reinterpret_cast<const void* const*>(factors), MTTKRP_BF16, out, R, stream);
}

mttkrp_status mttkrp_run_scheme2(mttkrp_handle h, int mode, const float* const* factors, float* out, int R,
                                 hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = check_run(h, mode, reinterpret_cast<const void* const*>(factors), out, R);
    if (s) return s;
    if (h->opts.hot_steps) return fail(MTTKRP_EUNSUPPORTED, "scheme 2 runs on nonzero-ordered copies only");
    const mk::DevMode& d = h->dev[mode];
    const void* fac[mk::kMaxIn];
    const uint32_t* hot[mk::kMaxIn];
    for (int j = 0; j < d.n_in; ++j) {
        fac[j] = factors[d.in_modes[j]];
        hot[j] = h->hot_rows[d.in_modes[j]];
    }
    const mk::Geometry g = plan_nnz(h, d.nnz, d.n_in, R, MTTKRP_FP32);
    hipError_t e = mk::launch_mttkrp(d, R, MTTKRP_FP32, fac, hot, h->nhot, out, h->carry, g, stream, true,
                                     h->dims[mode]);
    if (e != hipSuccess) return hip_fail(e, "MTTKRP (scheme 2) launch");
    return MTTKRP_OK;
}

mttkrp_status mttkrp_gather_probe(mttkrp_handle h, int mode, const void* const* factors, int factor_dtype, int R,
                                  int what, hipStream_t stream)
{
    g_err.clear();
    if (factor_dtype != MTTKRP_FP32 && factor_dtype != MTTKRP_BF16)
        return fail(MTTKRP_EINVAL, "factor_dtype must be MTTKRP_FP32 or MTTKRP_BF16");
    if (what < 0 || what > 3)
        return fail(MTTKRP_EINVAL, "what must be 0 (stream), 1 (stream and gathers), 2 (one lane per row "
                                   "gathering) or 3 (L1-resident rows)");
    if (!h) return fail(MTTKRP_EINVAL, "NULL handle");
    if (h->opts.partitioner == MTTKRP_PART_ROWS_LPT || h->opts.hot_steps)
        return fail(MTTKRP_EUNSUPPORTED, "the gather probe runs the nonzero-balanced partitions only");
    // The probe has no output: the handle's own carry workspace stands in for
    // it in the common argument checks.
    mttkrp_status s = check_run(h, mode, factors, h->carry, R);
    if (s) return s;
    const mk::DevMode& d = h->dev[mode];
    const void* fac[mk::kMaxIn];
    for (int j = 0; j < d.n_in; ++j) fac[j] = factors[d.in_modes[j]];
    const mk::Geometry g =
        mk::plan_geometry(d.nnz, d.n_in, R, factor_dtype, h->opts.parts_per_cu * h->cu_count, max_parts_for(h->nnz), kMaxChain);
    hipError_t e = mk::launch_gather_probe(d, R, factor_dtype, fac, h->carry, g, what, stream);
    if (e != hipSuccess) return hip_fail(e, "gather probe launch");
    return MTTKRP_OK;
}

static mttkrp_status check_factors(mttkrp_handle h, const void* const* factors, int R)
{
    if (!h) return fail(MTTKRP_EINVAL, "NULL handle");
    if (h->host_only) return fail(MTTKRP_EINVAL, "host-only handle: build without host_only to run");
    if (!r_supported(R)) return fail(MTTKRP_EUNSUPPORTED, "R must be 16, 32 or 64");
    if (R > h->opts.max_R) return fail(MTTKRP_EINVAL, "R exceeds the handle's max_R");
    if (!factors) return fail(MTTKRP_EINVAL, "NULL factors");
    for (int m = 0; m < h->N; ++m) {
        if (!factors[m]) return fail(MTTKRP_EINVAL, "factor " + std::to_string(m) + " is NULL");
        if (reinterpret_cast<uintptr_t>(factors[m]) % 16)
            return fail(MTTKRP_EINVAL, "factor " + std::to_string(m) + " must be 16-byte aligned");
    }
    return MTTKRP_OK;
}

mttkrp_status cpd_als_init(mttkrp_handle h, const float* const* factors, int R, hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = check_factors(h, reinterpret_cast<const void* const*>(factors), R);
    if (s) return s;
    hipError_t e = hipSuccess;
    for (int m = 0; m < h->N && e == hipSuccess; ++m) {
        e = mk::als_gram(factors[m], h->dims[m], R, h->als.grams + (uint64_t)m * R * R, h->als, stream);
        if (e == hipSuccess && h->opts.factor_dtype == MTTKRP_BF16)
            e = mk::cast_bf16(factors[m], (uint64_t)h->dims[m] * R, h->als.bf16[m], stream);
    }
    if (e == hipSuccess) e = mk::als_hadamard(h->als.grams, h->N, -1, R, h->als.V, h->als.scal + 1, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "cpd_als_init");
    h->als_R = R;
    return MTTKRP_OK;
}

// One sweep, enqueued only (no host synchronisation; capturable).  The
// not-positive-definite flag is cleared at the start when reset_flag is set.
// Row-pass job of the mode-n update of handle h (A = the new factor n).
static mk::DenseJob dense_job(mttkrp_handle h, float* A, int n, int R)
{
    mk::DenseJob j{};
    mk::AlsWork& w = h->als;
    j.M = w.M;
    j.W = w.W;
    j.A = A;
    j.lam = w.lam;
    j.part = w.part;
    j.G_out = w.grams + (uint64_t)n * R * R;
    j.N = h->N;
    mk::plan_dense_blocks(h->dims[n], w.max_blocks, j);
    return j;
}

// Fit job of handle h after the last mode's update (A = the new last factor).
static mk::DenseJob fit_job(mttkrp_handle h, float* A, int R, double* fit_out, double* lam_out)
{
    mk::DenseJob j = dense_job(h, A, h->N - 1, R);
    mk::AlsWork& w = h->als;
    j.G_out = nullptr;
    j.colsq = w.colsq;
    j.grams = w.grams;
    j.fit_out = fit_out;
    j.lam_out = lam_out;
    j.normX2 = h->normX2;
    return j;
}

static mttkrp_status als_sweep(mttkrp_handle h, float* const* factors, double* lambda, int R, double* fit_out,
                               hipStream_t stream, bool reset_flag)
{
    mttkrp_status s = check_factors(h, reinterpret_cast<const void* const*>(factors), R);
    if (s) return s;
    if (h->als_R != R) return fail(MTTKRP_EINVAL, "call cpd_als_init with this R first");
    if (!lambda) return fail(MTTKRP_EINVAL, "NULL lambda");
    mk::AlsWork& w = h->als;
    const int N = h->N;
    const bool bf16 = h->opts.factor_dtype == MTTKRP_BF16;
    const int dtype = bf16 ? MTTKRP_BF16 : MTTKRP_FP32;
    hipError_t e = hipSuccess;
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        const uint32_t I = h->dims[n];
        e = mk::als_normal_eq_inverse(w.job, 1, N, n, R, reset_flag && n == 0, h->opts.als_solve, stream);
        if (e == hipSuccess) {
            const void* fac[MTTKRP_MAX_MODES];
            for (int m = 0; m < N; ++m)
                fac[m] = bf16 ? static_cast<const void*>(w.bf16[m]) : static_cast<const void*>(factors[m]);
            mttkrp_status st = run_mode(h, n, fac, dtype, w.M, R, stream);
            if (st) return st;
        }
        mk::DenseJob j = dense_job(h, factors[n], n, R);
        if (e == hipSuccess)
            e = mk::als_solve_normalize_gram_jobs(j, nullptr, nullptr, 0, 1, R, h->opts.als_solve, stream);
        if (e == hipSuccess && bf16) e = mk::cast_bf16(factors[n], (uint64_t)I * R, w.bf16[n], stream);
    }
    if (e == hipSuccess) {
        mk::DenseJob j = fit_job(h, factors[N - 1], R, fit_out ? fit_out : w.scal, lambda);
        e = mk::als_fit_jobs(j, nullptr, nullptr, 0, 1, R, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "CP-ALS sweep");
    return MTTKRP_OK;
}

static mttkrp_status read_flag(mttkrp_handle h, hipStream_t stream)
{
    double f = 0.0;
    hipError_t e = hipMemcpyAsync(&f, h->als.scal + 1, sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "reading the CP-ALS status");
    if (f != 0.0) return fail(MTTKRP_ENOTSPD, "a normal-equation matrix V is not positive definite");
    return MTTKRP_OK;
}

mttkrp_status cpd_als_iter(mttkrp_handle h, float* const* factors, double* lambda, int R, double* fit_out,
                           hipStream_t stream)
{
    g_err.clear();
    mttkrp_status s = als_sweep(h, factors, lambda, R, fit_out, stream, true);
    if (s) return s;
    return read_flag(h, stream);
}

mttkrp_status cpd_als_iter_async(mttkrp_handle h, float* const* factors, double* lambda, int R, double* fit_out,
                                 hipStream_t stream)
{
    g_err.clear();
    return als_sweep(h, factors, lambda, R, fit_out, stream, false);
}

mttkrp_status cpd_als_status(mttkrp_handle h, hipStream_t stream)
{
    g_err.clear();
    if (!h || h->host_only) return fail(MTTKRP_EINVAL, "NULL or host-only handle");
    mttkrp_status s = read_flag(h, stream);
    if (s == MTTKRP_ENOTSPD) {
        // clear the sticky flag for the next sweeps
        (void)mk::als_hadamard(h->als.grams, h->N, -1, h->als_R ? h->als_R : 16, h->als.V, h->als.scal + 1, 1, stream);
        (void)hipStreamSynchronize(stream);
    }
    return s;
}


}  // extern "C"

// ---------------------------------------------------------------- batches

struct mttkrp_batch {
    int count = 0, N = 0, R = 0;
    int dtype = MTTKRP_FP32;                              // gather precision of the batched MTTKRP
    std::vector<mttkrp_handle> hs;
    void* dmem = nullptr;
    bool owns_mem = true;                                 // false: dmem is the caller's (mttkrp_batch_create_in)
    float* carry = nullptr;
    std::vector<uint64_t> carry_off;                      // per tensor, in floats
    std::vector<std::vector<mk::Geometry>> geo;           // [mode][tensor]
    char* part_desc[MTTKRP_MAX_MODES] = {};               // device descriptor tables
    char* fix_desc[MTTKRP_MAX_MODES] = {};
    uint2* part_work[MTTKRP_MAX_MODES] = {};
    uint2* fix_work[MTTKRP_MAX_MODES] = {};
    uint32_t npart_work[MTTKRP_MAX_MODES] = {};
    uint32_t nfix_work[MTTKRP_MAX_MODES] = {};
    uint32_t grid_part = 0, grid_fix = 0;
    int threads = 0, gathers = 0;                         // tuned partition-kernel shape (0: the default)
    int als_solve = 0;                                    // the layouts' opts.als_solve (all the same)
    std::vector<const void*> last_ptrs[MTTKRP_MAX_MODES]; // pointers of the uploaded descriptors
    mk::InvJob* inv_jobs = nullptr;                       // device: every tensor's normal-equation inverse job
    mk::DenseJob* dense_jobs[MTTKRP_MAX_MODES + 1] = {};  // device: per mode (and [N]: fit) one job per tensor
    uint2* dense_work[MTTKRP_MAX_MODES] = {};             // device: per mode, (tensor, row block) items
    uint32_t ndense_work[MTTKRP_MAX_MODES] = {};
    std::vector<mk::DenseJob> last_jobs[MTTKRP_MAX_MODES + 1];  // contents of the uploaded job tables
};

extern "C" {

void mttkrp_batch_free(mttkrp_batch_handle b)
{
    if (!b) return;
    if (b->dmem && b->owns_mem) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->dmem);
    }
    delete b;
}

}  // extern "C"

// The batch set-up behind mttkrp_batch_create (ext_mem == NULL: allocate,
// upload with blocking copies), mttkrp_batch_create_in (the caller's memory,
// uploads on `stream`, then that stream is synchronised) and
// mttkrp_batch_bytes (bytes_only: report the device bytes, build nothing).
static mttkrp_status batch_impl(const mttkrp_handle* layouts, int count, int R, const mttkrp_opts* opts,
                                void* ext_mem, uint64_t ext_bytes, hipStream_t stream, bool bytes_only,
                                uint64_t* bytes_out, mttkrp_batch_handle* out)
{
    if (!out && !bytes_only) return fail(MTTKRP_EINVAL, "NULL out");
    if (out) *out = nullptr;
    if (!layouts || count <= 0) return fail(MTTKRP_EINVAL, "need at least one layout");
    if (!r_supported(R)) return fail(MTTKRP_EUNSUPPORTED, "R must be 16, 32 or 64");
    mttkrp_opts o;
    mttkrp_status st = check_opts(opts, &o);
    if (st) return st;
    const int N = layouts[0] ? layouts[0]->N : 0;
    uint64_t total_nnz = 0;
    for (int t = 0; t < count; ++t) {
        const mttkrp_handle h = layouts[t];
        if (!h || h->host_only) return fail(MTTKRP_EINVAL, "layout " + std::to_string(t) + " is NULL or host-only");
        if (h->N != N) return fail(MTTKRP_EINVAL, "all layouts of a batch need the same N");
        if (R > h->opts.max_R) return fail(MTTKRP_EINVAL, "R exceeds the max_R of layout " + std::to_string(t));
        if (h->opts.partitioner == MTTKRP_PART_ROWS_LPT)
            return fail(MTTKRP_EUNSUPPORTED, "layout " + std::to_string(t) +
                                                 " uses scheme-1 partitions, which batches do not support");
        if (h->opts.hot_steps)
            return fail(MTTKRP_EUNSUPPORTED, "layout " + std::to_string(t) +
                                                 " has hot-steps copies, which batches do not support");
        if (h->nhot)
            return fail(MTTKRP_EUNSUPPORTED, "layout " + std::to_string(t) +
                                                 " keeps hot rows in LDS; batches take layouts built with hot_rows = 0");
        for (int m = 0; m < N; ++m)
            if ((uint64_t)h->dims[m] * (uint64_t)R * 4ull >= 0xFFFFFFF0ull)
                return fail(MTTKRP_EUNSUPPORTED, "a factor of layout " + std::to_string(t) + " is 4 GiB or larger");
        total_nnz += h->nnz;
    }
    auto* b = new mttkrp_batch();
    b->count = count;
    b->N = N;
    b->R = R;
    b->dtype = o.factor_dtype;
    b->hs.assign(layouts, layouts + count);
    (void)total_nnz;
    const int cus = layouts[0]->cu_count;
    // Each tensor keeps the partitioning mttkrp_run gives it, so a tensor's
    // result is bitwise the same alone and in any batch.
    b->geo.assign(N, std::vector<mk::Geometry>(count));
    std::vector<uint32_t> max_parts(count, 0);
    for (int n = 0; n < N; ++n)
        for (int t = 0; t < count; ++t) {
            const mttkrp_handle h = b->hs[t];
            b->geo[n][t] = plan_nnz(h, h->nnz, N - 1, R, b->dtype);
            max_parts[t] = std::max(max_parts[t], b->geo[n][t].nparts);
        }
    b->als_solve = b->hs[0]->opts.als_solve;
    for (int t = 1; t < count; ++t)
        if (b->hs[t]->opts.als_solve != b->als_solve) {
            delete b;
            return fail(MTTKRP_EINVAL, "the layouts of a batch must share opts.als_solve");
        }
    // One launch runs every tensor: they must share the partition kernel's shape.
    b->threads = b->geo[0][0].threads;
    b->gathers = b->geo[0][0].gathers;
    for (int t = 1; t < count; ++t)
        if (b->geo[0][t].threads != b->threads || b->geo[0][t].gathers != b->gathers) {
            delete b;
            return fail(MTTKRP_EINVAL, "layout " + std::to_string(t) +
                                           " has another part_threads / part_gathers than layout 0; the layouts "
                                           "of a batch share one launch shape");
        }
    // Work lists (largest tensors first, which balances the resident grid).
    std::vector<int> order(count);
    for (int t = 0; t < count; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->hs[x]->nnz > b->hs[y]->nnz; });
    std::vector<std::vector<uint2>> pw(N), fw(N);
    const size_t pdb = mk::part_desc_bytes(N - 1), fdb = mk::fix_desc_bytes();
    std::vector<char> scratch_desc(std::max(pdb, fdb));
    for (int n = 0; n < N; ++n)
        for (int t : order) {
            const mk::Geometry& g = b->geo[n][t];
            const uint32_t np = b->hs[t]->nnz ? g.nparts : 0;
            for (uint32_t p = 0; p < np; ++p) pw[n].push_back(make_uint2((uint32_t)t, p));
            const uint32_t nb = mk::fill_fix_desc(scratch_desc.data(), b->hs[t]->dev[n], g, nullptr, nullptr, R);
            for (uint32_t k = 0; k < nb; ++k) fw[n].push_back(make_uint2((uint32_t)t, k));
        }
    // Sizes are planned for the larger of the fp32 and bf16 geometries, so
    // mttkrp_batch_bytes (which has no dtype) covers batches of either.
    std::vector<uint64_t> pw_cap(N);
    for (int n = 0; n < N; ++n) pw_cap[n] = pw[n].size();
    {
        const int other = b->dtype == MTTKRP_FP32 ? MTTKRP_BF16 : MTTKRP_FP32;
        for (int n = 0; n < N; ++n) {
            uint64_t items = 0;
            for (int t = 0; t < count; ++t) {
                const mttkrp_handle h = b->hs[t];
                const mk::Geometry g2 = plan_nnz(h, h->nnz, N - 1, R, other);
                items += h->nnz ? g2.nparts : 0;
                max_parts[t] = std::max(max_parts[t], g2.nparts);
            }
            pw_cap[n] = std::max<uint64_t>(pw_cap[n], items);
        }
    }
    uint64_t carry_floats = 0;
    b->carry_off.resize(count);
    for (int t = 0; t < count; ++t) {
        b->carry_off[t] = carry_floats;
        carry_floats += (uint64_t)std::max<uint32_t>(max_parts[t], 1) * 2ull * (uint64_t)R;
    }
    // Row-pass work lists of the CP-ALS update: every tensor's row blocks of mode n.
    std::vector<std::vector<uint2>> dw(N);
    for (int n = 0; n < N; ++n)
        for (int t = 0; t < count; ++t) {
            mk::DenseJob j{};
            mk::plan_dense_blocks(b->hs[t]->dims[n], b->hs[t]->als.max_blocks, j);
            for (uint32_t k = 0; k < j.nb; ++k) dw[n].push_back(make_uint2((uint32_t)t, k));
        }
    uint64_t need = align_up(carry_floats * 4) + align_up((uint64_t)count * sizeof(mk::InvJob)) +
                    (uint64_t)(N + 1) * align_up((uint64_t)count * sizeof(mk::DenseJob));
    for (int n = 0; n < N; ++n) need += align_up(dw[n].size() * 8 + 8);
    for (int n = 0; n < N; ++n)
        need += align_up((uint64_t)count * pdb) + align_up((uint64_t)count * fdb) + align_up(pw_cap[n] * 8 + 8) +
                align_up(fw[n].size() * 8 + 8);
    if (bytes_only) {
        delete b;
        *bytes_out = need;
        return MTTKRP_OK;
    }
    hipError_t e = hipSuccess;
    if (ext_mem) {
        if (ext_bytes < need) {
            delete b;
            return fail(MTTKRP_EINVAL, "dev_mem holds " + std::to_string(ext_bytes) + " B; the batch needs " +
                                           std::to_string(need) + " B (mttkrp_batch_bytes)");
        }
        b->dmem = ext_mem;
        b->owns_mem = false;
    } else {
        e = hipMalloc(&b->dmem, need);
        if (e != hipSuccess) {
            b->dmem = nullptr;
            delete b;
            (void)hipGetLastError();
            return fail(MTTKRP_ENOMEM, "hipMalloc of " + std::to_string(need) + " B for the batch failed");
        }
    }
    // Host-to-device copies of the tables: blocking, or on the caller's stream.
    auto upload = [&](void* dst, const void* src, uint64_t n) -> hipError_t {
        return ext_mem ? hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, stream)
                       : hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
    };
    char* base = static_cast<char*>(b->dmem);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char* {
        char* p = base + off;
        off += align_up(bytes);
        return p;
    };
    b->carry = reinterpret_cast<float*>(take(carry_floats * 4));
    b->inv_jobs = reinterpret_cast<mk::InvJob*>(take((uint64_t)count * sizeof(mk::InvJob)));
    std::vector<mk::InvJob> inv_jobs(count);   // kept until the copies are done (end of this function)
    for (int t = 0; t < count; ++t) inv_jobs[t] = b->hs[t]->inv_job_host;
    e = upload(b->inv_jobs, inv_jobs.data(), inv_jobs.size() * sizeof(mk::InvJob));
    for (int n = 0; n <= N; ++n) b->dense_jobs[n] = reinterpret_cast<mk::DenseJob*>(take((uint64_t)count * sizeof(mk::DenseJob)));
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        b->dense_work[n] = reinterpret_cast<uint2*>(take(dw[n].size() * 8 + 8));
        b->ndense_work[n] = (uint32_t)dw[n].size();
        if (!dw[n].empty()) e = upload(b->dense_work[n], dw[n].data(), dw[n].size() * 8);
    }
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        b->part_desc[n] = take((uint64_t)count * pdb);
        b->fix_desc[n] = take((uint64_t)count * fdb);
        b->part_work[n] = reinterpret_cast<uint2*>(take(pw_cap[n] * 8 + 8));
        b->fix_work[n] = reinterpret_cast<uint2*>(take(fw[n].size() * 8 + 8));
        b->npart_work[n] = (uint32_t)pw[n].size();
        b->nfix_work[n] = (uint32_t)fw[n].size();
        if (!pw[n].empty()) e = upload(b->part_work[n], pw[n].data(), pw[n].size() * 8);
        if (e == hipSuccess && !fw[n].empty()) e = upload(b->fix_work[n], fw[n].data(), fw[n].size() * 8);
    }
    if (ext_mem) {
        // the host tables above go out of scope: wait for their copies (this stream only)
        const hipError_t es = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = es;
    }
    if (e != hipSuccess) {
        mttkrp_status s2 = hip_fail(e, "mttkrp_batch_create");
        mttkrp_batch_free(b);
        return s2;
    }
    b->grid_part = (uint32_t)cus * (uint32_t)std::max(1, 1024 / (b->threads ? b->threads : mk::partition_wg_threads(N - 1)));
    b->grid_fix = (uint32_t)cus * 8u;
    *out = b;
    return MTTKRP_OK;
}

extern "C" {

mttkrp_status mttkrp_batch_create(const mttkrp_handle* layouts, int count, int R, const mttkrp_opts* opts,
                                  mttkrp_batch_handle* out)
{
    g_err.clear();
    return batch_impl(layouts, count, R, opts, nullptr, 0, nullptr, false, nullptr, out);
}

mttkrp_status mttkrp_batch_bytes(const mttkrp_handle* layouts, int count, int R, uint64_t* bytes)
{
    g_err.clear();
    if (!bytes) return fail(MTTKRP_EINVAL, "NULL bytes");
    return batch_impl(layouts, count, R, nullptr, nullptr, 0, nullptr, true, bytes, nullptr);
}

mttkrp_status mttkrp_batch_create_in(const mttkrp_handle* layouts, int count, int R, const mttkrp_opts* opts,
                                     void* dev_mem, uint64_t dev_bytes, hipStream_t stream, mttkrp_batch_handle* out)
{
    g_err.clear();
    if (!dev_mem || reinterpret_cast<uintptr_t>(dev_mem) % kAlign)
        return fail(MTTKRP_EINVAL, "dev_mem must be a 256-byte aligned device pointer");
    return batch_impl(layouts, count, R, opts, dev_mem, dev_bytes, stream, false, nullptr, out);
}

}  // extern "C"

static mttkrp_status batch_run_impl(mttkrp_batch_handle b, int mode, const void* const* factors, int dtype,
                                    float* const* outs, hipStream_t stream)
{
    if (!b) return fail(MTTKRP_EINVAL, "NULL batch");
    if (dtype != b->dtype)
        return fail(MTTKRP_EINVAL, std::string("this batch gathers ") + (b->dtype == MTTKRP_FP32 ? "fp32" : "bf16") +
                                       " factors (its factor_dtype at creation)");
    if (mode < 0 || mode >= b->N) return fail(MTTKRP_EINVAL, "mode out of range");
    if (!factors || !outs) return fail(MTTKRP_EINVAL, "NULL factors or outs");
    const int N = b->N, R = b->R;
    // Pointers of this call; re-upload the descriptors only when they change.
    std::vector<const void*> ptrs;
    ptrs.reserve((size_t)b->count * (N + 1));
    for (int t = 0; t < b->count; ++t) {
        for (int m = 0; m < N; ++m) {
            const void* f = factors[(size_t)t * N + m];
            if (m != mode && (!f || reinterpret_cast<uintptr_t>(f) % 16))
                return fail(MTTKRP_EINVAL, "factor " + std::to_string(m) + " of tensor " + std::to_string(t) +
                                               " is NULL or not 16-byte aligned");
            ptrs.push_back(m == mode ? nullptr : f);
        }
        if (!outs[t] || reinterpret_cast<uintptr_t>(outs[t]) % 16)
            return fail(MTTKRP_EINVAL, "output of tensor " + std::to_string(t) + " is NULL or not 16-byte aligned");
        ptrs.push_back(outs[t]);
    }
    hipError_t e = hipSuccess;
    if (ptrs != b->last_ptrs[mode]) {
        const size_t pdb = mk::part_desc_bytes(N - 1), fdb = mk::fix_desc_bytes();
        std::vector<char> pd((size_t)b->count * pdb), fd((size_t)b->count * fdb);
        for (int t = 0; t < b->count; ++t) {
            const mk::DevMode& d = b->hs[t]->dev[mode];
            const mk::Geometry& g = b->geo[mode][t];
            const void* fac[mk::kMaxIn];
            for (int j = 0; j < d.n_in; ++j) fac[j] = factors[(size_t)t * N + d.in_modes[j]];
            float* carry = b->carry + b->carry_off[t];
            mk::fill_part_desc(pd.data() + (size_t)t * pdb, d, R, b->dtype, fac, outs[t], carry, g.gsz);
            mk::fill_fix_desc(fd.data() + (size_t)t * fdb, d, g, carry, outs[t], R);
        }
        // Stream-ordered after the launches that read the old tables; the host
        // copies are waited for before they go out of scope (this stream only).
        e = hipMemcpyAsync(b->part_desc[mode], pd.data(), pd.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b->fix_desc[mode], fd.data(), fd.size(), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "uploading batch descriptors");
        b->last_ptrs[mode] = std::move(ptrs);
    }
    const uint32_t gp = std::min(b->grid_part, std::max<uint32_t>(b->npart_work[mode], 1));
    e = mk::launch_batch_part(N - 1, R, b->dtype, b->threads, b->gathers, b->part_desc[mode], b->part_work[mode],
                              b->npart_work[mode], gp, stream);
    if (e == hipSuccess) {
        const uint32_t gf = std::min(b->grid_fix, std::max<uint32_t>(b->nfix_work[mode], 1));
        e = mk::launch_batch_fixup(b->fix_desc[mode], b->fix_work[mode], b->nfix_work[mode], gf, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "batched MTTKRP launch");
    return MTTKRP_OK;
}

extern "C" {

mttkrp_status mttkrp_batch_run(mttkrp_batch_handle b, int mode, const float* const* factors, float* const* outs,
                               hipStream_t stream)
{
    g_err.clear();
    return batch_run_impl(b, mode, reinterpret_cast<const void* const*>(factors), MTTKRP_FP32, outs, stream);
}

mttkrp_status mttkrp_batch_run_bf16(mttkrp_batch_handle b, int mode, const uint16_t* const* factors,
                                    float* const* outs, hipStream_t stream)
{
    g_err.clear();
    return batch_run_impl(b, mode, reinterpret_cast<const void* const*>(factors), MTTKRP_BF16, outs, stream);
}

}  // extern "C"

// The autotuner's default candidates for N-mode tensors: parts_per_cu 1 to
// 32, and for 3-mode tensors every tuned workgroup size and gathers in flight.
static std::vector<mttkrp_part_shape> default_shapes(int N)
{
    std::vector<mttkrp_part_shape> c;
    for (int ppc : {1, 2, 4, 8, 16, 32}) {
        if (N != 3) {
            c.push_back({ppc, 0, 0});
            continue;
        }
        for (int th : {256, 512, 1024})
            for (int gu : {2, 4}) c.push_back({ppc, th, gu});
    }
    return c;
}

// The autotuner behind mttkrp_batch_autotune (set_shape false: candidates
// change parts_per_cu only), mttkrp_batch_autotune_shape and (single: one
// layout timed through mttkrp_run) mttkrp_autotune_shape.  Each candidate is
// set on every layout, a batch is built unless single, and `reps` all-mode
// passes are timed after a warm-up pass; the fastest four are timed again
// over 4 x reps passes and the fastest of those stays set.
static mttkrp_status autotune_impl(const mttkrp_handle* layouts, int count, int R,
                                   const std::vector<mttkrp_part_shape>& cands, bool set_shape,
                                   const float* const* factors, float* const* outs, int reps, hipStream_t stream,
                                   int* best_out, float* times_ms, bool single = false)
{
    if (!layouts || count <= 0 || !factors || !outs) return fail(MTTKRP_EINVAL, "NULL layouts, factors or outs");
    if (cands.empty()) return fail(MTTKRP_EINVAL, "need at least one candidate");
    for (const mttkrp_part_shape& c : cands) {
        if (c.parts_per_cu < 1 || c.parts_per_cu > 64) return fail(MTTKRP_EINVAL, "parts_per_cu must be in [1, 64]");
        if (set_shape && (c.threads < 0 || c.gathers < 0 ||
                          ((c.threads || c.gathers) &&
                           !mk::tuned_shape_supported(c.threads ? c.threads : 512, c.gathers ? c.gathers : 4))))
            return fail(MTTKRP_EINVAL, "threads must be 0, 256, 512 or 1024 and gathers 0, 2 or 4");
    }
    if (reps < 1) return fail(MTTKRP_EINVAL, "reps must be >= 1");
    for (int t = 0; t < count; ++t)
        if (!layouts[t]) return fail(MTTKRP_EINVAL, "layout " + std::to_string(t) + " is NULL");
    const int N = layouts[0]->N;
    std::vector<mttkrp_part_shape> old(count);
    for (int t = 0; t < count; ++t)
        old[t] = {layouts[t]->opts.parts_per_cu, layouts[t]->opts.part_threads, layouts[t]->opts.part_gathers};
    auto apply = [&](int t, const mttkrp_part_shape& c) {
        layouts[t]->opts.parts_per_cu = c.parts_per_cu;
        if (set_shape) {
            layouts[t]->opts.part_threads = c.threads;
            layouts[t]->opts.part_gathers = c.gathers;
        }
    };
    auto restore = [&]() {
        for (int t = 0; t < count; ++t) {
            layouts[t]->opts.parts_per_cu = old[t].parts_per_cu;
            layouts[t]->opts.part_threads = old[t].threads;
            layouts[t]->opts.part_gathers = old[t].gathers;
        }
    };
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        restore();
        return hip_fail(e, "autotune events");
    }
    std::vector<float*> mode_outs(count);
    mttkrp_status st = MTTKRP_OK;
    // Average time of one all-mode pass of candidate i over r timed passes.
    auto time_candidate = [&](size_t i, int r, float* ms) -> mttkrp_status {
        for (int t = 0; t < count; ++t) apply(t, cands[i]);
        mttkrp_batch_handle b = nullptr;
        mttkrp_status s2 = MTTKRP_OK;
        if (!single) {
            s2 = mttkrp_batch_create(layouts, count, R, nullptr, &b);
            if (s2) return s2;
        }
        hipError_t e2 = hipSuccess;
        for (int pass = 0; pass <= r && s2 == MTTKRP_OK; ++pass) {
            if (pass == 1) e2 = hipEventRecord(ev[0], stream);
            for (int n = 0; n < N && s2 == MTTKRP_OK; ++n) {
                if (single) {
                    s2 = mttkrp_run(layouts[0], n, factors, outs[n], R, stream);
                    continue;
                }
                for (int t = 0; t < count; ++t) mode_outs[t] = outs[(size_t)t * N + n];
                s2 = mttkrp_batch_run(b, n, factors, mode_outs.data(), stream);
            }
        }
        if (s2 == MTTKRP_OK) {
            if (e2 == hipSuccess) e2 = hipEventRecord(ev[1], stream);
            if (e2 == hipSuccess) e2 = hipEventSynchronize(ev[1]);
            if (e2 == hipSuccess) e2 = hipEventElapsedTime(ms, ev[0], ev[1]);
            if (e2 != hipSuccess) s2 = hip_fail(e2, "autotune timing");
        }
        mttkrp_batch_free(b);
        *ms /= (float)r;
        return s2;
    };
    // Two stages: every candidate at `reps` passes, then (when there are
    // more than kFinal) the kFinal fastest again at 4 x reps passes, so that
    // candidates within timing noise of each other are told apart.
    constexpr size_t kFinal = 4;
    std::vector<float> ms(cands.size(), 0.0f);
    for (size_t i = 0; i < cands.size() && st == MTTKRP_OK; ++i) st = time_candidate(i, reps, &ms[i]);
    std::vector<size_t> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return ms[x] < ms[y]; });
    if (st == MTTKRP_OK && cands.size() > kFinal) {
        order.resize(kFinal);
        for (size_t k = 0; k < kFinal && st == MTTKRP_OK; ++k) st = time_candidate(order[k], 4 * reps, &ms[order[k]]);
    }
    int best = -1;
    for (size_t k = 0; k < order.size() && st == MTTKRP_OK; ++k)
        if (best < 0 || ms[order[k]] < ms[best]) best = (int)order[k];
    if (st == MTTKRP_OK && times_ms) std::copy(ms.begin(), ms.end(), times_ms);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st) {
        restore();
        return st;
    }
    for (int t = 0; t < count; ++t) apply(t, cands[best]);
    *best_out = best;
    return MTTKRP_OK;
}

extern "C" {

mttkrp_status mttkrp_batch_autotune(const mttkrp_handle* layouts, int count, int R, const int* candidates,
                                    int n_candidates, const float* const* factors, float* const* outs, int reps,
                                    hipStream_t stream, int* best_ppc, float* times_ms)
{
    g_err.clear();
    static const int kDefault[] = {1, 2, 4, 8, 16};
    if (!best_ppc) return fail(MTTKRP_EINVAL, "NULL best_ppc");
    if (!candidates) {
        candidates = kDefault;
        n_candidates = 5;
    }
    if (n_candidates <= 0) return fail(MTTKRP_EINVAL, "need at least one candidate");
    std::vector<mttkrp_part_shape> c(n_candidates);
    for (int i = 0; i < n_candidates; ++i) c[i] = {candidates[i], 0, 0};
    int best = 0;
    mttkrp_status st = autotune_impl(layouts, count, R, c, false, factors, outs, reps, stream, &best, times_ms);
    if (st) return st;
    *best_ppc = c[best].parts_per_cu;
    return MTTKRP_OK;
}

mttkrp_status mttkrp_batch_autotune_shape(const mttkrp_handle* layouts, int count, int R,
                                          const mttkrp_part_shape* candidates, int n_candidates,
                                          const float* const* factors, float* const* outs, int reps,
                                          hipStream_t stream, mttkrp_part_shape* best, float* times_ms)
{
    g_err.clear();
    if (!best) return fail(MTTKRP_EINVAL, "NULL best");
    if (!layouts || count <= 0 || !layouts[0]) return fail(MTTKRP_EINVAL, "NULL layouts");
    std::vector<mttkrp_part_shape> c;
    if (candidates) {
        if (n_candidates <= 0) return fail(MTTKRP_EINVAL, "need at least one candidate");
        c.assign(candidates, candidates + n_candidates);
    } else {
        c = default_shapes(layouts[0]->N);
    }
    int k = 0;
    mttkrp_status st = autotune_impl(layouts, count, R, c, true, factors, outs, reps, stream, &k, times_ms);
    if (st) return st;
    *best = c[k];
    return MTTKRP_OK;
}

mttkrp_status mttkrp_autotune_shape(mttkrp_handle h, int R, const mttkrp_part_shape* candidates, int n_candidates,
                                    const float* const* factors, float* const* outs, int reps, hipStream_t stream,
                                    mttkrp_part_shape* best, float* times_ms)
{
    g_err.clear();
    if (!best) return fail(MTTKRP_EINVAL, "NULL best");
    if (!h) return fail(MTTKRP_EINVAL, "NULL handle");
    if (h->host_only) return fail(MTTKRP_EINVAL, "host-only handle: build without host_only to run");
    if (h->opts.hot_steps)
        return fail(MTTKRP_EUNSUPPORTED, "hot-steps copies have one launch shape; there is nothing to tune");
    std::vector<mttkrp_part_shape> c;
    if (candidates) {
        if (n_candidates <= 0) return fail(MTTKRP_EINVAL, "need at least one candidate");
        c.assign(candidates, candidates + n_candidates);
    } else {
        c = default_shapes(h->N);
    }
    int k = 0;
    mttkrp_status st = autotune_impl(&h, 1, R, c, true, factors, outs, reps, stream, &k, times_ms, true);
    if (st) return st;
    *best = c[k];
    return MTTKRP_OK;
}

int mttkrp_batch_autotune_default_shapes(int N, mttkrp_part_shape* out)
{
    const std::vector<mttkrp_part_shape> c = default_shapes(N);
    if (out) std::copy(c.begin(), c.end(), out);
    return (int)c.size();
}

mttkrp_status cpd_als_batch_iter_async(mttkrp_batch_handle b, float* const* factors, double* const* lambdas,
                                       double* const* fits, hipStream_t stream)
{
    g_err.clear();
    if (!b) return fail(MTTKRP_EINVAL, "NULL batch");
    if (!factors || !lambdas) return fail(MTTKRP_EINVAL, "NULL factors or lambdas");
    const int N = b->N, R = b->R, C = b->count;
    for (int t = 0; t < C; ++t) {
        mttkrp_handle h = b->hs[t];
        mttkrp_status s = check_factors(h, reinterpret_cast<const void* const*>(factors + (size_t)t * N), R);
        if (s) return fail(s, "tensor " + std::to_string(t) + ": " + g_err);
        if (h->als_R != R) return fail(MTTKRP_EINVAL, "tensor " + std::to_string(t) + ": call cpd_als_init first");
        if (h->opts.factor_dtype != b->dtype)
            return fail(MTTKRP_EINVAL, "tensor " + std::to_string(t) + ": its factor_dtype differs from the batch's "
                                       "(create the batch with the layouts' factor_dtype)");
        if (!lambdas[t]) return fail(MTTKRP_EINVAL, "NULL lambda for tensor " + std::to_string(t));
    }
    std::vector<float*> outs(C);
    for (int t = 0; t < C; ++t) outs[t] = b->hs[t]->als.M;
    // Job tables of this call (factor, lambda and fit pointers); re-uploaded
    // only when they differ from the last call's, which synchronises first.
    hipError_t e = hipSuccess;
    for (int n = 0; n <= N && e == hipSuccess; ++n) {
        std::vector<mk::DenseJob> jobs(C);
        for (int t = 0; t < C; ++t) {
            mttkrp_handle h = b->hs[t];
            float* A = factors[(size_t)t * N + (n < N ? n : N - 1)];
            jobs[t] = n < N ? dense_job(h, A, n, R)
                            : fit_job(h, A, R, (fits && fits[t]) ? fits[t] : h->als.scal, lambdas[t]);
            if (n < N && b->dtype == MTTKRP_BF16) jobs[t].A16 = h->als.bf16[n];
        }
        if (jobs.size() != b->last_jobs[n].size() ||
            std::memcmp(jobs.data(), b->last_jobs[n].data(), jobs.size() * sizeof(mk::DenseJob)) != 0) {
            e = hipMemcpyAsync(b->dense_jobs[n], jobs.data(), jobs.size() * sizeof(mk::DenseJob), hipMemcpyHostToDevice,
                               stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e == hipSuccess) b->last_jobs[n] = std::move(jobs);
        }
    }
    const mk::DenseJob none{};
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        e = mk::als_normal_eq_inverse(b->inv_jobs, C, N, n, R, 0, b->als_solve, stream);
        if (e != hipSuccess) break;
        // The MTTKRP gathers the fp32 factors, or the handles' bf16 copies.
        std::vector<const void*> gather((size_t)C * N);
        for (int t = 0; t < C; ++t)
            for (int m = 0; m < N; ++m)
                gather[(size_t)t * N + m] = b->dtype == MTTKRP_BF16 ? static_cast<const void*>(b->hs[t]->als.bf16[m])
                                                                    : static_cast<const void*>(factors[(size_t)t * N + m]);
        mttkrp_status st = batch_run_impl(b, n, gather.data(), b->dtype, outs.data(), stream);
        if (st) return st;
        e = mk::als_solve_normalize_gram_jobs(none, b->dense_jobs[n], b->dense_work[n], b->ndense_work[n], C, R,
                                              b->als_solve, stream);
        if (e == hipSuccess && b->dtype == MTTKRP_BF16)
            e = mk::cast_bf16_jobs(b->dense_jobs[n], b->dense_work[n], b->ndense_work[n], R, stream);
    }
    if (e == hipSuccess)
        e = mk::als_fit_jobs(none, b->dense_jobs[N], b->dense_work[N - 1], b->ndense_work[N - 1], C, R, stream);
    if (e != hipSuccess) return hip_fail(e, "batched CP-ALS sweep");
    return MTTKRP_OK;
}

}  // extern "C"
