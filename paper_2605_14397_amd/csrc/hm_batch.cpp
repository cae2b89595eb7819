// Batched products over many operators (independent meshes): their task
// lists are merged so that one gather, one phase A, one reduction, one
// phase B and one scatter cover every operator, the two phases each one
// queue-driven launch over the merged, byte-balanced task list; the
// sequence is captured once as a HIP graph and replayed.  A small
// autotuner picks the phase-A task size (source leaves per wavefront task)
// and the phase-B window height by timing candidates on the batch itself.
#include <algorithm>
#include <chrono>

#include "hm_op.hpp"

namespace hm {

struct Batch {
    std::vector<Op*> ops;
    int near_prec = HM_F64, far_prec = HM_F64;
    DevBuf bases, tasksA, itemsA, membersA, reduce, tasksB, itemsB, segs, queue;
    std::vector<std::unique_ptr<ApplyWs>> ws;  // the batch's own workspace per operator
    LaunchSet L;
    int64_t max_ne = 0, total_ne = 0;
    std::vector<Segment> hsegs;
    bool use_graph = true;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_nrhs = -1;
    int tuned_leaves = 8;
    double tune_ms[5] = {0, 0, 0, 0, 0};
    int tune_cand[5] = {8, 12, 16, 24, 32};  // smaller tasks only add partial slots (measured 2 and 4: no faster)
    int tuned_window = kTileWindowB;
    double tune_b_ms[3] = {0, 0, 0};
    int tune_b_cand[3] = {8, 4, 2};

    ~Batch()
    {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
    }
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_nrhs = -1;
    }

    // concatenate the operators' task lists with their op index
    void merge(hipStream_t s)
    {
        std::vector<Bases> hb;
        std::vector<TaskA> ta;
        std::vector<PanelRef> ia, ib;
        std::vector<MemberT> ma;
        std::vector<ReduceDesc> rd;
        std::vector<TaskB> tb;
        ws.resize(ops.size());
        for (size_t k = 0; k < ops.size(); ++k) {
            const Variant& v = ops[k]->main;
            ws[k] = v.new_workspace(s);
            hb.push_back(v.host_bases(ws[k]->block.get()));
            const int ia0 = (int)ia.size(), ib0 = (int)ib.size(), ma0 = (int)ma.size();
            ia.insert(ia.end(), v.hItemsA.begin(), v.hItemsA.end());
            ma.insert(ma.end(), v.hMembersA.begin(), v.hMembersA.end());
            ib.insert(ib.end(), v.hItemsB.begin(), v.hItemsB.end());
            for (TaskA t : v.hTasksA) {
                t.item_begin += ia0;
                t.mem_begin += ma0;
                t.op = (int32_t)k;
                ta.push_back(t);
            }
            for (ReduceDesc r : v.hReduce) {
                r.op = (int32_t)k;
                rd.push_back(r);
            }
            // phase-B windows in leaf order (the operator's own list is
            // sorted for a launch of its own)
            for (const TaskB& sec : v.sectionsB) {
                const int tiles = (sec.rows + 15) / 16;
                for (int r0 = 0; r0 < tiles; r0 += v.windowB) {
                    TaskB t = sec;
                    t.item_begin += ib0;
                    t.op = (int32_t)k;
                    t.r0 = r0;
                    t.nt = std::min(v.windowB, tiles - r0);
                    tb.push_back(t);
                }
            }
        }
        L = LaunchSet();
        L.near_prec = near_prec;
        L.far_prec = far_prec;
        // a merged batch keeps its natural order inside each XCD range
        L.splitA = order_tasksA(ta, ia, false);
        L.splitB = order_tasksB(tb, ib, near_prec, far_prec, false);
        upload(bases, hb, s);
        upload(tasksA, ta, s);
        upload(itemsA, ia, s);
        upload(membersA, ma, s);
        upload(reduce, rd, s);
        upload(tasksB, tb, s);
        upload(itemsB, ib, s);
        HM_CHECK_HIP(hipStreamSynchronize(s));
        L.bases = bases.as<Bases>();
        L.tasksA = tasksA.as<TaskA>();
        L.nTasksA = (int)ta.size();
        L.itemsA = itemsA.as<PanelRef>();
        L.membersA = membersA.as<MemberT>();

        L.reduce = reduce.as<ReduceDesc>();
        L.nReduce = (int)rd.size();
        L.tasksB = tasksB.as<TaskB>();
        L.nTasksB = (int)tb.size();
        L.itemsB = itemsB.as<PanelRef>();
        L.maxNtB = 1;
        for (const TaskB& t : tb) L.maxNtB = std::max(L.maxNtB, t.nt);
        if (!queue.get()) queue.alloc(kQueueInts * sizeof(int));
        L.queue = queue.as<int>();
        drop_graph();
    }

    int64_t total_leaves() const
    {
        int64_t n = 0;
        for (const Op* op : ops) n += (int64_t)op->plan.leaves.size();
        return n;
    }

    void set_vectors(int nrhs, const double* const* X, const int64_t* ldx, double* const* Y, const int64_t* ldy,
                     hipStream_t s)
    {
        bool changed = hsegs.size() != ops.size();
        hsegs.resize(ops.size());
        int32_t leaf0 = 0;
        for (size_t k = 0; k < ops.size(); ++k) {
            const Op& op = *ops[k];
            const int64_t lx = ldx ? ldx[k] : 3 * op.ne, ly = ldy ? ldy[k] : 3 * op.ne;
            HM_REQUIRE(X[k] && Y[k], HM_EINVAL, "null vector pointer for operator " + std::to_string(k));
            HM_REQUIRE(lx >= 3 * op.ne && ly >= 3 * op.ne, HM_EINVAL, "leading dimension below 3N");
            Segment g = make_segment(op, op.main, X[k], lx, Y[k], ly, false, (int)k);
            g.leaf0 = leaf0;
            leaf0 += g.nleaf;
            if (std::memcmp(&g, &hsegs[k], sizeof(Segment)) != 0) changed = true;
            hsegs[k] = g;
        }
        (void)nrhs;
        if (changed || !segs.get()) {
            if (!segs.get()) segs.alloc(sizeof(Segment) * ops.size());
            HM_CHECK_HIP(hipMemcpyAsync(segs.get(), hsegs.data(), sizeof(Segment) * ops.size(),
                                        hipMemcpyHostToDevice, s));
        }
    }

    void run(int nrhs, hipStream_t s, hipEvent_t* ev = nullptr)
    {
        if (!use_graph || ev) {
            launch_product(L, nrhs, segs.as<Segment>(), nullptr, (int)ops.size(), total_leaves(), s, ev);
            return;
        }
        if (!exec || graph_nrhs != nrhs) {
            drop_graph();
            if (!cap) HM_CHECK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            HM_CHECK_HIP(hipStreamSynchronize(s));
            HM_CHECK_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            try {
                launch_product(L, nrhs, segs.as<Segment>(), nullptr, (int)ops.size(), total_leaves(), cap, nullptr);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(cap, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HM_CHECK_HIP(hipStreamEndCapture(cap, &graph));
            HM_CHECK_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            graph_nrhs = nrhs;
        }
        HM_CHECK_HIP(hipGraphLaunch(exec, s));
    }
};

static double time_runs(Batch& b, int nrhs, int reps, hipStream_t s)
{
    hipEvent_t e0, e1;
    HM_CHECK_HIP(hipEventCreate(&e0));
    HM_CHECK_HIP(hipEventCreate(&e1));
    b.run(nrhs, s);  // warm
    HM_CHECK_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) b.run(nrhs, s);
    HM_CHECK_HIP(hipEventRecord(e1, s));
    HM_CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HM_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

Batch* batch_create(const std::vector<Op*>& ops, const hm_batch_opts& o, hipStream_t s)
{
    HM_REQUIRE(!ops.empty(), HM_EINVAL, "empty batch");
    std::unique_ptr<Batch> b(new Batch());
    b->ops = ops;
    b->near_prec = ops[0]->main.near_prec;
    b->far_prec = ops[0]->main.far_prec;
    for (Op* op : ops) {
        HM_REQUIRE(op, HM_EINVAL, "null operator in batch");
        HM_REQUIRE(op->main.near_prec == b->near_prec && op->main.far_prec == b->far_prec, HM_EUNSUPPORTED,
                   "all operators of a batch must share one precision form");
        b->max_ne = std::max(b->max_ne, op->ne);
        b->total_ne += op->ne;
    }
    b->use_graph = o.use_graph != 0;
    b->merge(s);
    // without tuning each operator keeps its own layout; report the first's
    b->tuned_leaves = ops[0]->main.leavesPerTaskA;
    b->tuned_window = ops[0]->main.windowB;
    if (o.autotune) {
        // time each phase-A task size on zero vectors of the batch's own shape
        std::vector<DevBuf> xs;
        std::vector<const double*> X;
        std::vector<double*> Y;
        for (Op* op : ops) {
            xs.emplace_back((size_t)kNrhs * 3 * op->ne * sizeof(double));
            HM_CHECK_HIP(hipMemsetAsync(xs.back().get(), 0, xs.back().bytes(), s));
            X.push_back(xs.back().as<double>());
        }
        std::vector<DevBuf> ys;
        for (Op* op : ops) {
            ys.emplace_back((size_t)kNrhs * 3 * op->ne * sizeof(double));
            Y.push_back(ys.back().as<double>());
        }
        b->set_vectors(kNrhs, X.data(), nullptr, Y.data(), nullptr, s);
        // one candidate: rebuild and merge the task lists, then time 5 products
        auto time_config = [&](int lpt, int wnd) {
            for (Op* op : ops) {
                build_tasksA(*op, op->main, lpt);
                build_tasksB(op->main, wnd);
                upload_tasks(op->main, s);
            }
            b->merge(s);
            b->hsegs.clear();
            b->set_vectors(kNrhs, X.data(), nullptr, Y.data(), nullptr, s);
            return time_runs(*b, kNrhs, 5, s);
        };
        // each candidate is timed in two rounds (the second in reverse
        // order) and keeps its faster time, so a slow moment of the device
        // does not decide the choice
        const int w0 = ops[0]->main.windowB;
        for (int c = 0; c < 5; ++c) b->tune_ms[c] = 1e300;
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 5; ++k) {
                const int c = r == 0 ? k : 4 - k;
                b->tune_ms[c] = std::min(b->tune_ms[c], time_config(b->tune_cand[c], w0));
            }
        int best_l = b->tune_cand[0];
        double best = b->tune_ms[0];
        for (int c = 1; c < 5; ++c)
            if (b->tune_ms[c] < best) {
                best = b->tune_ms[c];
                best_l = b->tune_cand[c];
            }
        // then the phase-B window height with the chosen phase-A task size
        for (int c = 0; c < 3; ++c) b->tune_b_ms[c] = 1e300;
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 3; ++k) {
                const int c = r == 0 ? k : 2 - k;
                b->tune_b_ms[c] = std::min(b->tune_b_ms[c], time_config(best_l, b->tune_b_cand[c]));
            }
        int best_w = b->tune_b_cand[0];
        double best_b = b->tune_b_ms[0];
        for (int c = 1; c < 3; ++c)
            if (b->tune_b_ms[c] < best_b) {
                best_b = b->tune_b_ms[c];
                best_w = b->tune_b_cand[c];
            }
        for (Op* op : ops) {
            build_tasksA(*op, op->main, best_l);
            build_tasksB(op->main, best_w);
            upload_tasks(op->main, s);
        }
        b->tuned_leaves = best_l;
        b->tuned_window = best_w;
        b->merge(s);
        b->hsegs.clear();
        HM_CHECK_HIP(hipStreamSynchronize(s));
    }
    return b.release();
}

void batch_apply(Batch& b, int nrhs, const double* const* X, const int64_t* ldx, double* const* Y, const int64_t* ldy,
                 hipStream_t s)
{
    HM_REQUIRE(nrhs >= 1 && nrhs <= kNrhs, HM_EINVAL, "nrhs must be in [1, 16]");
    HM_REQUIRE(X && Y, HM_EINVAL, "null pointer array");
    b.set_vectors(nrhs, X, ldx, Y, ldy, s);
    b.run(nrhs, s);
}

void batch_info(const Batch& b, hm_batch_info* out)
{
    std::memset(out, 0, sizeof(*out));
    out->n_ops = (int)b.ops.size();
    out->total_elements = b.total_ne;
    out->use_graph = b.use_graph ? 1 : 0;
    out->leaves_per_task_a = b.tuned_leaves;
    out->phase_b_window = b.tuned_window;
    for (int c = 0; c < 3; ++c) {
        out->tune_b_candidates[c] = b.tune_b_cand[c];
        out->tune_b_ms[c] = b.tune_b_ms[c];
    }
    for (int c = 0; c < 5; ++c) {
        out->tune_candidates[c] = b.tune_cand[c];
        out->tune_ms[c] = b.tune_ms[c];
    }
    int64_t bytes = 0;
    for (const Op* op : b.ops) bytes += op->main.bytes_near + op->main.bytes_far;
    out->bytes_operators = bytes;
}

void batch_destroy(Batch* b) { delete b; }

}  // namespace hm
