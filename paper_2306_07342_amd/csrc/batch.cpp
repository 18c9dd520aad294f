// Batched emulation: many independent density matrices of uneven size, each
// with its own op program, run by one persistent kernel launch (k_batch).
//
// Host side: every instance's program is planned (in parallel threads) with
// the plan options chosen for its qubit count, the plans are concatenated into
// one device image, the instances are queued largest first, and the arena
// (caller-owned device memory) is laid out.  The launch can be captured into
// a HIP graph and replayed.  An autotuner times candidate tile shapes per
// qubit count on a sample of the batch and caches the choice in a JSON file.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <thread>

#include "vqd_internal.h"

struct vqd_batch {
    struct Inst {
        int n = 0;
        std::vector<vqd::LOp> ops;
        vqd::HostPlan plan;
        uint64_t arena_off = 0;   // amplitudes
        uint32_t out_off = 0;
        double cost = 0;
    };
    std::vector<Inst> inst;
    // parametric templates: one planned structure, per-instance parameters
    struct Template {
        int n = 0;
        std::vector<int> kinds, targets;              // 4 targets per op
        vqd::HostPlan plan;
        std::vector<std::vector<double>> params;      // per instance, 4 per op
        std::vector<uint64_t> arena_off;
        std::vector<uint32_t> out_off;
    };
    std::vector<Template> tmpl;
    // instance index -> (template id or -1, index within inst or the template)
    std::vector<std::pair<int, uint32_t>> refs;
    std::map<int, vqd::PlanOpts> opts_by_n;
    vqd::BatchDev dev;
    std::vector<vqd::BatchItem> items;
    uint64_t arena_amps = 0;
    size_t n_out = 0;
    size_t total_passes = 0;
    double fp64_fma = 0;      // executed FP64 FMAs of one run (all instances)
    double pass_bytes = 0;    // algorithmic HBM bytes of one run (all instances)
    bool compiled = false;
    int device = -1;
    hipGraphExec_t gexec = nullptr;
    void *g_arena = nullptr;
    double *g_out = nullptr;
    // the graph is captured on and replayed from the library's own stream
    // (the legacy default stream cannot be captured), ordered after and
    // before the caller's stream with events
    hipStream_t g_stream = nullptr;
    hipStream_t up_stream = nullptr;   // compile's uploads (into fresh buffers; never waits for
                                       // work on other streams, so it overlaps a running launch)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace vqd {
namespace {

constexpr int kBatchTile = 12;     // k_batch workgroups hold at most 2^12-amplitude tiles

PlanOpts default_opts(int n)
{
    PlanOpts o;
    o.tile_bits = std::min(kBatchTile, 2 * n);
    o.min_contig_bits = 3;
    o.pad_coalesce = false;
    // k_batch stages a full 2^12 tile and keeps 1 KiB of its own beside it
    o.rt_budget = (160 * 1024 - 1024 - (16 << kBatchTile)) / 16;
    // every named op preserves Hermiticity and each instance starts from
    // |0..0><0..0|: half the tiles per pass (the planner falls back for a
    // program with an op that does not preserve it)
    o.hermitian = true;
    o.min_contig_bits = 1;
    return o;
}

void free_batch_dev(BatchDev &d)
{
    free_dev_program(d.prog);
    if (d.buf) (void)hipFree(d.buf);
    d = BatchDev{};
}

void drop_graph(vqd_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_arena = nullptr;
    b->g_out = nullptr;
}

void free_graph_stream(vqd_batch *b)
{
    drop_graph(b);
    if (b->g_stream) (void)hipStreamDestroy(b->g_stream);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    b->g_stream = nullptr;
    b->ev_in = b->ev_out = nullptr;
    if (b->up_stream) (void)hipStreamDestroy(b->up_stream);
    b->up_stream = nullptr;
}

// Plan all instances of `sel` (indices into b->inst) in parallel.
int plan_all(vqd_batch *b, const std::vector<int> &sel, const std::map<int, PlanOpts> &opts)
{
    std::vector<int> rc(sel.size(), VQD_OK);
    std::vector<std::string> msg(sel.size());
    std::atomic<size_t> next(0);
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto worker = [&]() {
        for (;;) {
            const size_t k = next.fetch_add(1);
            if (k >= sel.size()) break;
            auto &I = b->inst[sel[k]];
            auto it = opts.find(I.n);
            const PlanOpts o = (it != opts.end()) ? it->second : default_opts(I.n);
            rc[k] = plan_program(I.n, I.ops, o, I.plan);
            if (rc[k]) msg[k] = vqd_last_error();
        }
    };
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i) th.emplace_back(worker);
    for (auto &t : th) t.join();
    for (size_t k = 0; k < sel.size(); ++k)
        if (rc[k]) return fail(rc[k], "instance " + std::to_string(sel[k]) + ": " + msg[k]);
    return VQD_OK;
}

// Concatenate the plans of `sel` and of template instances (all templates if
// tmpl_n < 0, else those on tmpl_n qubits, tmpl_n == 0: none; at most
// tmpl_cap instances each), lay out arena and outputs, upload.
int build_device(vqd_batch *b, const std::vector<int> &sel, hipStream_t stream, int tmpl_n = -1,
                 size_t tmpl_cap = SIZE_MAX)
{
    HostPlan all;
    std::vector<BatchItem> items;
    uint64_t arena = 0;
    uint32_t outs = 0, max_rt = 0;
    size_t passes = 0;
    double fma = 0, hbm = 0;
    // per instance of n qubits and plan p: the passes' FMAs on the computed
    // amplitudes; bytes: the initial state written, 16 B read and written
    // per computed amplitude per pass, the mirror images of the last pass,
    // and the diagonal read for <Z_i>
    auto account = [&](int n, const HostPlan &p, double count) {
        const double amps = std::ldexp(1.0, 2 * n), f = p.tile_fraction;
        fma += count * p.fma_per_amp * f * amps;
        hbm += count * (16.0 * amps + 32.0 * f * amps * (double)p.passes.size() +
                          (p.hermitian ? 16.0 * (1.0 - f) * amps : 0.0) + 16.0 * std::ldexp(1.0, n));
    };
    for (int i : sel) {
        auto &I = b->inst[i];
        const uint32_t pass_base = (uint32_t)all.passes.size();
        const uint32_t phase_base = (uint32_t)all.phases.size();
        const uint32_t op_base = (uint32_t)all.ops.size();
        const uint32_t mat_base = (uint32_t)all.mats.size();
        for (KPass P : I.plan.passes) {
            if (P.L > (uint32_t)kBatchTile || P.phantom)
                return fail(VQD_E_SIZE, "batched instances need tiles of at most 12 bits and n >= 2");
            P.phase_begin += phase_base;
            P.phase_end += phase_base;
            P.rt_mat += mat_base;
            max_rt = std::max(max_rt, P.rt_count);
            all.passes.push_back(P);
        }
        for (KPhase H : I.plan.phases) {
            H.op_begin += op_base;
            H.op_end += op_base;
            all.phases.push_back(H);
        }
        for (KOp o : I.plan.ops) {
            if (o.kind != KOP_DIAG_RT) o.mat += mat_base;
            all.ops.push_back(o);
        }
        all.mats.insert(all.mats.end(), I.plan.mats.begin(), I.plan.mats.end());
        I.arena_off = arena;
        arena += ((1ull << (2 * I.n)) + 15) & ~15ull;     // 256-byte aligned instances
        I.out_off = outs;
        outs += (uint32_t)I.n;
        I.cost = (double)(I.plan.passes.size() + 1) * (double)(1ull << (2 * I.n));
        BatchItem it{};
        it.mat_base = 0;
        it.arena_off = I.arena_off;
        it.n = (uint32_t)I.n;
        it.pass_begin = pass_base;
        it.pass_end = (uint32_t)all.passes.size();
        it.out_off = I.out_off;
        items.push_back(it);
        passes += I.plan.passes.size();
        account(I.n, I.plan, 1.0);
    }
    std::vector<double> cost;
    for (int i : sel) cost.push_back(b->inst[i].cost);
    // parametric templates: the structure once, a coefficient block per instance
    {
        for (auto &T : b->tmpl) {
            if (T.params.empty() || tmpl_n == 0 || (tmpl_n > 0 && T.n != tmpl_n)) continue;
            const uint32_t pass_base = (uint32_t)all.passes.size();
            const uint32_t phase_base = (uint32_t)all.phases.size();
            const uint32_t op_base = (uint32_t)all.ops.size();
            for (KPass P : T.plan.passes) {
                if (P.L > (uint32_t)kBatchTile || P.phantom)
                    return fail(VQD_E_SIZE, "batched instances need tiles of at most 12 bits and n >= 2");
                P.phase_begin += phase_base;
                P.phase_end += phase_base;
                max_rt = std::max(max_rt, P.rt_count);
                all.passes.push_back(P);
            }
            for (KPhase H : T.plan.phases) {
                H.op_begin += op_base;
                H.op_end += op_base;
                all.phases.push_back(H);
            }
            for (const KOp &o : T.plan.ops) all.ops.push_back(o);
            const size_t block = T.plan.mats.size();
            const size_t mbase = all.mats.size();
            const size_t count = std::min(T.params.size(), tmpl_cap);
            all.mats.resize(mbase + block * count);
            T.arena_off.resize(count);
            T.out_off.resize(count);
            // coefficients of every instance, in host threads
            std::vector<int> rc(count, VQD_OK);
            std::vector<std::string> msg(count);
            std::atomic<size_t> next(0);
            auto worker = [&]() {
                std::vector<LOp> lops;
                std::vector<cd> mats;
                for (;;) {
                    const size_t k = next.fetch_add(1);
                    if (k >= count) break;
                    const int r = template_mats(T.n, T.kinds, T.targets, T.plan, T.params[k].data(), lops, mats);
                    if (r) {
                        rc[k] = r;
                        msg[k] = vqd_last_error();
                        continue;
                    }
                    std::copy(mats.begin(), mats.end(), all.mats.begin() + mbase + k * block);
                }
            };
            const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (unsigned i = 0; i < nt; ++i) th.emplace_back(worker);
            for (auto &t : th) t.join();
            for (size_t k = 0; k < count; ++k)
                if (rc[k]) return fail(rc[k], "template instance " + std::to_string(k) + ": " + msg[k]);
            for (size_t k = 0; k < count; ++k) {
                BatchItem it{};
                it.arena_off = arena;
                it.mat_base = mbase + k * block;
                it.n = (uint32_t)T.n;
                it.pass_begin = pass_base;
                it.pass_end = (uint32_t)all.passes.size();
                it.out_off = outs;
                T.arena_off[k] = arena;
                T.out_off[k] = outs;
                arena += ((1ull << (2 * T.n)) + 15) & ~15ull;
                outs += (uint32_t)T.n;
                items.push_back(it);
                cost.push_back((double)(T.plan.passes.size() + 1) * (double)(1ull << (2 * T.n)));
                passes += T.plan.passes.size();
                account(T.n, T.plan, 1.0);
            }
        }
    }
    // largest first
    std::vector<size_t> order(items.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<BatchItem> queue;
    for (size_t k : order) queue.push_back(items[k]);

    drop_graph(b);
    // a recompiled batch may still be running from its old buffers
    if (b->dev.buf || b->dev.prog.buf) VQD_HIP(hipDeviceSynchronize());
    free_batch_dev(b->dev);
    if (!all.passes.empty())
        if (int rc = upload_plan(all, b->dev.prog, stream)) return rc;
    const size_t bytes = queue.size() * sizeof(BatchItem) + 256;
    if (hipMalloc(&b->dev.buf, bytes) != hipSuccess) return fail(VQD_E_NOMEM, "batch table allocation failed");
    b->dev.items = static_cast<BatchItem *>(b->dev.buf);
    b->dev.counter = reinterpret_cast<uint32_t *>(static_cast<char *>(b->dev.buf) + queue.size() * sizeof(BatchItem));
    VQD_HIP(hipMemcpyAsync(b->dev.items, queue.data(), queue.size() * sizeof(BatchItem), hipMemcpyHostToDevice, stream));
    VQD_HIP(hipStreamSynchronize(stream));
    b->dev.n_items = (uint32_t)queue.size();
    b->dev.max_rt = max_rt;
    b->items = queue;
    b->arena_amps = arena;
    b->n_out = outs;
    b->total_passes = passes;
    b->fp64_fma = fma;
    b->pass_bytes = hbm;
    return VQD_OK;
}

}  // namespace

int check_template(int n, int count, const int *kinds, const int *targets)
{
    if (!kinds || !targets || count < 1) return fail(VQD_E_ARG, "bad template arguments");
    for (int i = 0; i < count; ++i) {
        int nq = 0, np = 0;
        if (kind_arity(kinds[i], &nq, &np) != 0) return fail(VQD_E_ARG, "unknown kind in template op " + std::to_string(i));
        for (int j = 0; j < nq; ++j) {
            const int q = targets[4 * i + j];
            if (q < 0 || q >= n) return fail(VQD_E_ARG, "bad target in template op " + std::to_string(i));
            for (int k = 0; k < j; ++k)
                if (targets[4 * i + k] == q) return fail(VQD_E_ARG, "duplicate target in template op " + std::to_string(i));
        }
    }
    return VQD_OK;
}

int plan_template(int n, const std::vector<int> &kinds, const std::vector<int> &targets, PlanOpts o, HostPlan &plan)
{
    o.record_recipes = true;
    o.keep_identity = true;
    o.relayout = false;
    std::vector<LOp> canon(kinds.size());
    for (size_t j = 0; j < kinds.size(); ++j) {
        double p[4];
        canonical_params(kinds[j], p);
        std::vector<cd> S;
        int k = 0;
        if (int rc = kind_superop(kinds[j], p, S, k)) return rc;
        canon[j] = make_superop_op(k, &targets[4 * j], S.data());
    }
    return plan_program(n, canon, o, plan);
}

int template_mats(int n, const std::vector<int> &kinds, const std::vector<int> &targets, const HostPlan &plan,
                  const double *params, std::vector<LOp> &lops, std::vector<cd> &mats)
{
    // A circuit repeats few (kind, parameters) pairs many times (one angle on
    // every qubit of a layer, one noise channel after every gate): each
    // distinct pair's superoperator is built once per instance, and the ops
    // are filled in place so that the per-thread scratch is reused.
    struct Built {
        int kind, k;
        double p[4];
        std::vector<cd> S;
    };
    thread_local std::vector<Built> memo;
    size_t n_memo = 0;
    lops.resize(kinds.size());
    for (size_t j = 0; j < kinds.size(); ++j) {
        const double *p = params + 4 * j;
        int nq = 0, np = 0;
        if (kind_arity(kinds[j], &nq, &np) != 0) return fail(VQD_E_ARG, "unknown kind in template op");
        size_t hit = n_memo;
        for (size_t m = 0; m < n_memo; ++m) {
            const Built &b = memo[m];
            if (b.kind != kinds[j]) continue;
            bool same = true;
            for (int i = 0; i < np; ++i) same = same && std::memcmp(&b.p[i], &p[i], sizeof(double)) == 0;
            if (same) {
                hit = m;
                break;
            }
        }
        if (hit == n_memo) {
            if (memo.size() <= n_memo) memo.emplace_back();
            Built &b = memo[n_memo];
            b.kind = kinds[j];
            for (int i = 0; i < 4; ++i) b.p[i] = (i < np) ? p[i] : 0.0;
            if (int rc = kind_superop(kinds[j], p, b.S, b.k)) return rc;
            ++n_memo;
        }
        const Built &b = memo[hit];
        fill_superop_op(lops[j], b.k, &targets[4 * j], b.S.data());
    }
    return recompute_mats(n, plan, lops, mats);
}

namespace {

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Minimal JSON object of "key": [tile_bits, contig, microseconds] entries.
std::map<std::string, std::vector<double>> read_cache(const std::string &path)
{
    std::map<std::string, std::vector<double>> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q1 = line.find('"'), q2 = line.find('"', q1 + 1), lb = line.find('['), rb = line.find(']');
        if (q1 == std::string::npos || q2 == std::string::npos || lb == std::string::npos || rb == std::string::npos)
            continue;
        std::vector<double> v;
        std::stringstream ss(line.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(ss, tok, ',')) v.push_back(std::atof(tok.c_str()));
        if (v.size() == 3) m[line.substr(q1 + 1, q2 - q1 - 1)] = v;
    }
    return m;
}

void write_cache(const std::string &path, const std::map<std::string, std::vector<double>> &m)
{
    std::ofstream f(path);
    f << "{\n";
    size_t k = 0;
    for (const auto &kv : m) {
        f << "  \"" << kv.first << "\": [" << (int)kv.second[0] << ", " << (int)kv.second[1] << ", "
          << kv.second[2] << "]" << (++k < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

}  // namespace
}  // namespace vqd

using namespace vqd;

extern "C" {

int vqd_batch_create(vqd_batch **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = new (std::nothrow) vqd_batch();
    if (!*out) return fail(VQD_E_NOMEM, "batch allocation failed");
    return VQD_OK;
}

int vqd_batch_destroy(vqd_batch *b)
{
    clear_error();
    if (!b) return VQD_OK;
    (void)hipDeviceSynchronize();
    free_graph_stream(b);
    free_batch_dev(b->dev);
    delete b;
    return VQD_OK;
}

int vqd_batch_add(vqd_batch *b, const vqd_prog *p, int *index)
{
    clear_error();
    if (!b || !p) return fail(VQD_E_ARG, "null argument");
    if (p->n < 2 || p->n > VQD_MAX_QUBITS) return fail(VQD_E_SIZE, "batched instances need n in [2, 16]");
    vqd_batch::Inst I;
    I.n = p->n;
    I.ops = p->ops;
    b->inst.push_back(std::move(I));
    b->refs.emplace_back(-1, (uint32_t)b->inst.size() - 1);
    b->compiled = false;
    if (index) *index = (int)b->refs.size() - 1;
    return VQD_OK;
}

int vqd_batch_set_opts(vqd_batch *b, int n, const vqd_plan_opts *o)
{
    clear_error();
    if (!b || !o) return fail(VQD_E_ARG, "null argument");
    if (n < 2 || n > VQD_MAX_QUBITS) return fail(VQD_E_SIZE, "n must be in [2, 16]");
    if (o->tile_bits < 4 || o->tile_bits > 12) return fail(VQD_E_ARG, "batched tile_bits must be in [4, 12]");
    b->opts_by_n[n] = to_plan_opts(*o);
    b->opts_by_n[n].relayout = false;     // batched instances keep their layout in place
    b->compiled = false;
    return VQD_OK;
}

int vqd_batch_compile(vqd_batch *b, size_t *arena_bytes, size_t *n_outputs)
{
    clear_error();
    if (!b) return fail(VQD_E_ARG, "null batch");
    size_t n_tmpl = 0;
    for (const auto &T : b->tmpl) n_tmpl += T.params.size();
    if (b->inst.empty() && n_tmpl == 0) return fail(VQD_E_STATE, "empty batch");
    std::vector<int> all(b->inst.size());
    for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
    if (int rc = plan_all(b, all, b->opts_by_n)) return rc;
    for (auto &T : b->tmpl) {
        auto it = b->opts_by_n.find(T.n);
        const PlanOpts o = (it != b->opts_by_n.end()) ? it->second : default_opts(T.n);
        if (int rc = plan_template(T.n, T.kinds, T.targets, o, T.plan)) return rc;
    }
    // the old device buffers are freed first (a device-wide wait), so the
    // uploads go to fresh memory on a stream of their own: they overlap work
    // still running on the caller's streams (an earlier launch of another
    // batch) instead of queueing behind it
    if (!b->up_stream) VQD_HIP(hipStreamCreateWithFlags(&b->up_stream, hipStreamNonBlocking));
    if (int rc = build_device(b, all, b->up_stream)) return rc;
    (void)hipGetDevice(&b->device);
    b->compiled = true;
    if (arena_bytes) *arena_bytes = (size_t)b->arena_amps * 16;
    if (n_outputs) *n_outputs = b->n_out;
    return VQD_OK;
}

int vqd_batch_offsets(const vqd_batch *b, int index, size_t *arena_offset_bytes, size_t *out_offset)
{
    clear_error();
    if (!b || !b->compiled) return fail(VQD_E_STATE, "batch not compiled");
    if (index < 0 || index >= (int)b->refs.size()) return fail(VQD_E_ARG, "instance index out of range");
    const auto ref = b->refs[index];
    uint64_t a = 0;
    uint32_t o = 0;
    if (ref.first < 0) {
        a = b->inst[ref.second].arena_off;
        o = b->inst[ref.second].out_off;
    } else {
        a = b->tmpl[ref.first].arena_off[ref.second];
        o = b->tmpl[ref.first].out_off[ref.second];
    }
    if (arena_offset_bytes) *arena_offset_bytes = (size_t)a * 16;
    if (out_offset) *out_offset = o;
    return VQD_OK;
}

int vqd_batch_add_template(vqd_batch *b, int n, int count, const int *kinds, const int *targets,
                           int *template_id)
{
    clear_error();
    if (!b || !kinds || !targets || count < 1) return fail(VQD_E_ARG, "bad template arguments");
    if (n < 2 || n > VQD_MAX_QUBITS) return fail(VQD_E_SIZE, "batched instances need n in [2, 16]");
    if (int rc = check_template(n, count, kinds, targets)) return rc;
    vqd_batch::Template T;
    T.n = n;
    T.kinds.assign(kinds, kinds + count);
    T.targets.assign(targets, targets + 4 * (size_t)count);
    b->tmpl.push_back(std::move(T));
    b->compiled = false;
    if (template_id) *template_id = (int)b->tmpl.size() - 1;
    return VQD_OK;
}

int vqd_batch_add_instances(vqd_batch *b, int template_id, int count, const double *params, int *first_index)
{
    clear_error();
    if (!b || template_id < 0 || template_id >= (int)b->tmpl.size() || count < 0 || (count && !params))
        return fail(VQD_E_ARG, "bad instance arguments");
    auto &T = b->tmpl[template_id];
    const size_t per = 4 * T.kinds.size();
    for (size_t j = 0; j < per * (size_t)count; ++j)
        if (!std::isfinite(params[j])) return fail(VQD_E_ARG, "non-finite parameter");
    if (first_index) *first_index = (int)b->refs.size();
    for (int i = 0; i < count; ++i) {
        const double *p = params + per * (size_t)i;
        T.params.emplace_back(p, p + per);
        b->refs.emplace_back(template_id, (uint32_t)T.params.size() - 1);
    }
    b->compiled = false;
    return VQD_OK;
}

int vqd_batch_run(vqd_batch *b, void *arena, size_t arena_bytes, double *out, void *hip_stream, int use_graph)
{
    clear_error();
    if (!b || !arena || !out) return fail(VQD_E_ARG, "null argument");
    if (!b->compiled) return fail(VQD_E_STATE, "batch not compiled");
    if (arena_bytes < (size_t)b->arena_amps * 16) return fail(VQD_E_SIZE, "arena smaller than the batch needs");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double2 *ar = static_cast<double2 *>(arena);
    if (!use_graph) return launch_batch(ar, b->dev, out, st);
    if (!b->g_stream) {
        VQD_HIP(hipStreamCreateWithFlags(&b->g_stream, hipStreamNonBlocking));
        VQD_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        VQD_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    }
    hipStream_t cs = b->g_stream;
    if (!b->gexec || b->g_arena != arena || b->g_out != out) {
        drop_graph(b);
        // launch attributes are set by an ordinary first launch
        if (int rc = launch_batch(ar, b->dev, out, st)) return rc;
        VQD_HIP(hipStreamSynchronize(st));
        hipGraph_t g = nullptr;
        VQD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int rc = launch_batch(ar, b->dev, out, cs);
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
        b->g_arena = arena;
        b->g_out = out;
    }
    VQD_HIP(hipEventRecord(b->ev_in, st));
    VQD_HIP(hipStreamWaitEvent(cs, b->ev_in, 0));
    VQD_HIP(hipGraphLaunch(b->gexec, cs));
    VQD_HIP(hipEventRecord(b->ev_out, cs));
    VQD_HIP(hipStreamWaitEvent(st, b->ev_out, 0));
    return VQD_OK;
}

int vqd_batch_autotune(vqd_batch *b, void *arena, size_t arena_bytes, double *out, void *hip_stream,
                       const char *cache_path, int max_per_n)
{
    clear_error();
    if (!b || !arena || !out) return fail(VQD_E_ARG, "null argument");
    if (b->refs.empty()) return fail(VQD_E_STATE, "empty batch");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::map<std::string, std::vector<double>> cache;
    if (cache_path) cache = read_cache(cache_path);
    const std::string arch = arch_name();
    std::map<int, std::vector<int>> by_n;
    for (size_t i = 0; i < b->inst.size(); ++i) by_n[b->inst[i].n].push_back((int)i);
    for (const auto &T : b->tmpl)
        if (!T.params.empty()) by_n[T.n];        // qubit counts with template instances only
    hipEvent_t e0, e1;
    VQD_HIP(hipEventCreate(&e0));
    VQD_HIP(hipEventCreate(&e1));
    int rc = VQD_OK;
    for (auto &kv : by_n) {
        const int n = kv.first;
        const bool herm = default_opts(n).hermitian;
        const std::string key = arch + (herm ? ":herm:n" : ":n") + std::to_string(n);
        auto hit = cache.find(key);
        if (hit != cache.end()) {
            PlanOpts o = default_opts(n);
            o.tile_bits = (int)hit->second[0];
            o.min_contig_bits = (int)hit->second[1];
            b->opts_by_n[n] = o;
            continue;
        }
        const size_t cap = (size_t)std::max(1, max_per_n);
        std::vector<int> sel(kv.second.begin(), kv.second.begin() + std::min<size_t>(kv.second.size(), cap));
        // a sample of template instances only where no ordinary ones are
        const bool use_tmpl = sel.empty();
        std::vector<PlanOpts> cands;
        // Hermitian mode: tiles of whole qubits (even sizes), 1-3 forced qubits
        const std::vector<int> tbs = herm ? std::vector<int>{12, 10, 8} : std::vector<int>{12, 11, 10, 9};
        const std::vector<int> cs = herm ? std::vector<int>{1, 2, 3} : std::vector<int>{0, 2, 3};
        for (int tb : tbs) {
            const int t = std::min(tb, 2 * n);
            for (int c : cs) {
                PlanOpts o = default_opts(n);
                o.tile_bits = t;
                o.min_contig_bits = std::min(c, t);
                bool dup = false;
                for (auto &x : cands) dup |= (x.tile_bits == o.tile_bits && x.min_contig_bits == o.min_contig_bits);
                if (!dup) cands.push_back(o);
            }
        }
        double best_t = 1e30;
        PlanOpts best = default_opts(n);
        for (const PlanOpts &o : cands) {
            std::map<int, PlanOpts> om{{n, o}};
            if ((rc = plan_all(b, sel, om))) break;
            if (use_tmpl)
                for (auto &T : b->tmpl)
                    if (T.n == n && !T.params.empty() && (rc = plan_template(T.n, T.kinds, T.targets, o, T.plan)))
                        break;
            if (rc) break;
            if ((rc = build_device(b, sel, st, use_tmpl ? n : 0, cap))) break;
            if (arena_bytes < b->arena_amps * 16) { rc = fail(VQD_E_SIZE, "arena too small for tuning"); break; }
            if ((rc = launch_batch(static_cast<double2 *>(arena), b->dev, out, st))) break;
            VQD_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 2; ++r)
                if ((rc = launch_batch(static_cast<double2 *>(arena), b->dev, out, st))) break;
            if (rc) break;
            VQD_HIP(hipEventRecord(e1, st));
            VQD_HIP(hipEventSynchronize(e1));
            float ms = 0;
            VQD_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_t) {
                best_t = ms;
                best = o;
            }
        }
        if (rc) break;
        b->opts_by_n[n] = best;
        cache[key] = {(double)best.tile_bits, (double)best.min_contig_bits, best_t * 1e3 / 2};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (cache_path) write_cache(cache_path, cache);
    b->compiled = false;
    return VQD_OK;
}

int vqd_batch_info_get(const vqd_batch *b, vqd_batch_info *out)
{
    clear_error();
    if (!b || !out) return fail(VQD_E_ARG, "null argument");
    size_t n = b->inst.size();
    for (const auto &T : b->tmpl) n += T.params.size();
    out->n_instances = (int)n;
    out->total_passes = (long long)b->total_passes;
    out->arena_bytes = (size_t)b->arena_amps * 16;
    out->n_outputs = b->n_out;
    out->grid_items = b->dev.n_items;
    out->fp64_fma = b->fp64_fma;
    out->pass_bytes = b->pass_bytes;
    return VQD_OK;
}

int vqd_batch_plan_opts(const vqd_batch *b, int n, vqd_plan_opts *o)
{
    clear_error();
    if (!b || !o) return fail(VQD_E_ARG, "null argument");
    auto it = b->opts_by_n.find(n);
    const PlanOpts p = (it != b->opts_by_n.end()) ? it->second : default_opts(n);
    o->tile_bits = p.tile_bits;
    o->min_contig_bits = p.min_contig_bits;
    o->max_ops_per_pass = p.max_ops_per_pass;
    o->fuse_blocks = p.fuse_blocks;
    o->pad_coalesce = p.pad_coalesce;
    o->hermitian = p.hermitian ? 1 : 0;
    o->relayout = 0;
    return VQD_OK;
}

}  // extern "C"

int vqd_template_export(int n, int count, const int *kinds, const int *targets, const double *params,
                        const vqd_plan_opts *opts, void *buf, size_t cap, size_t *needed)
{
    clear_error();
    if (!needed) return fail(VQD_E_ARG, "null argument");
    if (n < 1 || n > VQD_MAX_QUBITS) return fail(VQD_E_SIZE, "n out of range");
    if (int rc = check_template(n, count, kinds, targets)) return rc;
    vqd_plan_opts o;
    vqd_plan_opts_default(&o);
    if (opts) o = *opts;
    const std::vector<int> kv(kinds, kinds + count), tv(targets, targets + 4 * (size_t)count);
    HostPlan plan;
    PlanOpts po = to_plan_opts(o);
    po.relayout = false;
    if (int rc = plan_template(n, kv, tv, po, plan)) return rc;
    if (params) {
        for (size_t j = 0; j < 4 * (size_t)count; ++j)
            if (!std::isfinite(params[j])) return fail(VQD_E_ARG, "non-finite parameter");
        std::vector<LOp> lops;
        std::vector<cd> mats;
        if (int rc = template_mats(n, kv, tv, plan, params, lops, mats)) return rc;
        plan.mats = mats;
    }
    return export_plan(plan, n, o.tile_bits, buf, cap, needed);
}
