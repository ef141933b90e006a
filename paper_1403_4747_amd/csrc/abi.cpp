// C ABI of libfda: plan build and upload, matvec, right-hand side, GMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>

#include "../../include/fda.h"
#include "dsetup.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "operators.hpp"
#include "plan.hpp"

using namespace fda;

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

struct fda_mlp {
    fda::Mlp *m = nullptr;
    int device = 0;
};

struct fda_plan {
    HostPlan hp;
    DevPlan d;
    fda_mlp *mlp = nullptr;  // borrowed: learned preconditioner for FDA_PRECOND_MLP
    int device = 0;
    std::vector<void *> allocs;      // build-time device allocations
    int cap_nrhs = 0;                // capacity of the work buffers below
    double2 *xt = nullptr, *yt = nullptr;
    std::vector<void *> work;        // per-capacity allocations
    fda_stats stats{};
    int64_t device_bytes = 0;
    double m2m_flops = 0, l2l_flops = 0;  // per upward / downward pass
    // The low-rank M2L pairs of every merged level stay on the host so that
    // the merged work list can be rebuilt for another configuration
    // (fda_m2l_set_config, fda_autotune).
    struct M2LLevelHost {
        int level = 0;
        int64_t nstates = 0;                                          // states of the level
        std::vector<std::vector<std::pair<int32_t, int32_t>>> by_op;  // per translation: (source, target) state
        std::vector<int32_t> prank;                                   // padded rank per translation
        fda::M2LLevelArgs la;                                         // tbase set when the list is built
    };
    std::vector<M2LLevelHost> m2l_host;
    std::vector<void *> m2l_allocs;  // device arrays of the merged list
    int64_t m2l_bytes = 0;
    fda_m2l_config m2l_cfg{};
    // Batches (captured graphs) that hold pointers to the work buffers and
    // the merged M2L list: while one exists, nothing may reallocate them.
    int live_batches = 0;
};

namespace {

struct HipError {
    hipError_t e;
    const char *what;
};

inline void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw HipError{e, what};
}

template <class T>
T *dalloc(fda_plan *p, size_t count, std::vector<void *> &list) {
    if (count == 0) count = 1;
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, sizeof(T) * count);
    if (e != hipSuccess) throw BuildError{FDA_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed"};
    list.push_back(ptr);
    p->device_bytes += (int64_t)(sizeof(T) * count);
    return (T *)ptr;
}

template <class T>
T *upload(fda_plan *p, const std::vector<T> &v) {
    T *d = dalloc<T>(p, v.size(), p->allocs);
    if (!v.empty()) hip_check(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "upload");
    return d;
}

double2 *upload_cplx(fda_plan *p, const std::vector<cplx> &v) {
    double2 *d = dalloc<double2>(p, v.size(), p->allocs);
    if (!v.empty()) hip_check(hipMemcpy(d, v.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice), "upload");
    return d;
}

// The plan's copy of an FP64 device operator array: itself for FP64 plans;
// an FP32 copy for FP32 plans (the FP64 array stays allocated until the plan
// is freed only if it is referenced elsewhere; here it is released at once).
void *to_storage(fda_plan *p, double2 *a64, size_t n) {
    if (p->d.prec != FDA_PREC_FP32 || a64 == nullptr) return a64;
    float2 *a32 = dalloc<float2>(p, n, p->allocs);
    hip_check(launch_to_f32(a64, a32, (int64_t)n, nullptr), "to f32");
    hip_check(hipDeviceSynchronize(), "to f32");
    auto it = std::find(p->allocs.begin(), p->allocs.end(), (void *)a64);
    if (it != p->allocs.end()) {
        (void)hipFree(a64);
        p->allocs.erase(it);
        p->device_bytes -= (int64_t)(sizeof(double2) * n);
    }
    return a32;
}

// Host-side builder of a gathered-GEMM work list (kernels.hpp, GWork).
struct GWorkHost {
    std::vector<int32_t> hdr, src, dstcol;
    int64_t ncol = 0;
    std::vector<std::vector<int32_t>> parts;  // per destination: scratch columns
    std::vector<int32_t> dest;                // destination state of each entry of parts
    std::unordered_map<int32_t, int32_t> dest_index;
    // one work item: matrix `mat` times the gathered states `srcs`; the
    // products go to new scratch columns that are summed into `dsts`
    void add(int32_t mat, const std::vector<int32_t> &srcs, const std::vector<int32_t> &dsts) {
        hdr.push_back(mat);
        hdr.push_back((int32_t)ncol);
        hdr.push_back((int32_t)srcs.size());
        hdr.push_back(0);
        for (int b = 0; b < kGemmCols; ++b) {
            src.push_back(b < (int)srcs.size() ? srcs[b] : -1);
            dstcol.push_back(b < (int)dsts.size() ? dsts[b] : -1);
        }
        for (size_t b = 0; b < dsts.size(); ++b) {
            auto it = dest_index.find(dsts[b]);
            int32_t di;
            if (it == dest_index.end()) {
                di = (int32_t)dest.size();
                dest_index[dsts[b]] = di;
                dest.push_back(dsts[b]);
                parts.emplace_back();
            } else {
                di = it->second;
            }
            parts[di].push_back((int32_t)(ncol + b));
        }
        ncol += (int64_t)srcs.size();
    }
};

// m: rows of the list's matrices (the destination-major units are 16-row
// tiles of every destination)
GWork upload_gwork(fda_plan *p, const GWorkHost &g, int m) {
    GWork w;
    w.nwork = (int)(g.hdr.size() / 4);
    w.ncol = g.ncol;
    w.hdr = (int4 *)upload(p, g.hdr);
    w.src = upload(p, g.src);
    bool single = true;
    for (const auto &pl : g.parts) single = single && pl.size() == 1;
    if (single) {  // one product per destination: written in place
        w.dst = upload(p, g.dstcol);
        return w;
    }
    w.nred = (int)g.dest.size();
    std::vector<int32_t> off{0}, list;
    for (const auto &pl : g.parts) {
        list.insert(list.end(), pl.begin(), pl.end());
        off.push_back((int32_t)list.size());
    }
    w.rd_dst = upload(p, g.dest);
    w.rd_off = upload(p, off);
    w.rd_list = upload(p, list);
    // destination-major form: (matrix, source state) of every list entry
    // (scratch column c is column c - first of its item)
    std::vector<int32_t> mat(g.ncol), srcst(g.ncol), ent, units;
    for (size_t i = 0; i < g.hdr.size() / 4; ++i)
        for (int32_t b = 0; b < g.hdr[4 * i + 2]; ++b) {
            mat[g.hdr[4 * i + 1] + b] = g.hdr[4 * i];
            srcst[g.hdr[4 * i + 1] + b] = g.src[i * kGemmCols + b];
        }
    for (int32_t c : list) ent.insert(ent.end(), {mat[c], srcst[c]});
    const int nt = (m + 15) / 16;
    for (int32_t t = 0; t < w.nred; ++t)
        for (int32_t rt = 0; rt < nt; ++rt) units.insert(units.end(), {t, rt});
    if (p->d.prec != FDA_PREC_FP32 && !ent.empty() && !units.empty()) {  // FP64 plans only
        w.dm_ent = (int2 *)upload(p, ent);
        w.dm_units = (int2 *)upload(p, units);
        w.dm_nunits = (int)(units.size() / 2);
    }
    return w;
}

void free_work(fda_plan *p) {
    for (void *q : p->work) (void)hipFree(q);
    p->work.clear();
    p->cap_nrhs = 0;
    p->xt = p->yt = nullptr;
    for (auto &l : p->d.lv) l.s = l.c = l.m2l.tmp = l.m2m.tmp = l.l2l.tmp = nullptr;
}

// Work buffers for `nrhs` right-hand sides: tree-order vectors and the
// per-level outgoing / incoming states.
void ensure_capacity(fda_plan *p, int nrhs) {
    if (nrhs <= p->cap_nrhs) return;
    if (p->live_batches > 0)
        throw BuildError{FDA_EINVAL, "the plan's work buffers hold " + std::to_string(p->cap_nrhs) +
                                         " columns and a batch graph references them; free the batch before a "
                                         "call with more columns"};
    free_work(p);
    const int64_t N = p->d.n;
    p->xt = dalloc<double2>(p, (size_t)N * nrhs, p->work);
    p->yt = dalloc<double2>(p, (size_t)N * nrhs, p->work);
    // storage elements: double2 (FP64 plan) or float2 (two floats, FP32 plan)
    const size_t es = p->d.prec == FDA_PREC_FP32 ? 1 : 2;  // in units of float2
    // the per-pair products of M2M, M2L and L2L share one scratch buffer:
    // the stages run one after another on the caller's stream
    size_t scratch = 0;
    for (int l = p->d.top; l <= p->d.depth && p->d.has_far; ++l) {
        DevLevel &lv = p->d.lv[l];
        lv.s = dalloc<float2>(p, es * (size_t)lv.sstride * nrhs, p->work);
        lv.c = dalloc<float2>(p, es * (size_t)lv.cstride * nrhs, p->work);
        scratch = std::max(scratch, (size_t)lv.m2l.ncol * lv.kd);
        if (l < p->d.depth) {
            const DevLevel &C = p->d.lv[l + 1];
            scratch = std::max(scratch, (size_t)lv.m2m.ncol * lv.ku);
            scratch = std::max(scratch, (size_t)lv.l2l.ncol * C.kd);
        }
    }
    M2LMerged &mm = p->d.m2l_all;
    scratch = std::max(scratch, (size_t)mm.nscratch);
    if (scratch > 0) {
        float2 *tmp = dalloc<float2>(p, es * scratch * nrhs, p->work);
        for (int l = p->d.top; l <= p->d.depth && p->d.has_far; ++l) {
            DevLevel &lv = p->d.lv[l];
            lv.m2l.tmp = tmp;
            if (l < p->d.depth) lv.m2m.tmp = lv.l2l.tmp = tmp;
        }
        mm.tmp = tmp;
    }
    if (mm.nwork > 0) {
        for (auto &la : mm.hargs) {
            la.X = p->d.lv[la.level].s;
            la.Y = p->d.lv[la.level].c;
        }
        hip_check(hipMemcpy(mm.args, mm.hargs.data(), sizeof(M2LLevelArgs) * mm.hargs.size(), hipMemcpyHostToDevice),
                  "M2L level table");
    }
    p->cap_nrhs = nrhs;
}

// Gauss-Legendre rule on [-1, 1] by the Golub-Welsch construction: the
// nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// Legendre polynomials (zero diagonal, off-diagonal j / sqrt(4 j^2 - 1)), and
// each weight is 2 (the integral of 1) times the squared first component of
// the node's normalised eigenvector.  The eigenproblem (n <= 64) is solved
// by cyclic Jacobi rotations on the dense matrix.
void legendre_nodes(int n, double *x, double *w) {
    std::vector<double> A((size_t)n * n, 0.0), Q((size_t)n * n, 0.0);
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    auto q = [&](int i, int j) -> double & { return Q[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) q(i, i) = 1.0;
    for (int j = 1; j < n; ++j) a(j - 1, j) = a(j, j - 1) = j / std::sqrt(4.0 * j * j - 1.0);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
        if (off < 1e-40) break;
        for (int p = 0; p < n; ++p)
            for (int r = p + 1; r < n; ++r) {
                if (a(p, r) == 0.0) continue;
                // rotation in the (p, r) plane that zeroes a(p, r): with
                // theta = (a_rr - a_pp) / (2 a_pr), t = tan of the angle
                const double th = (a(r, r) - a(p, p)) / (2.0 * a(p, r));
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, r of A and Q
                    const double akp = a(k, p), akr = a(k, r);
                    a(k, p) = c * akp - sn * akr;
                    a(k, r) = sn * akp + c * akr;
                    const double qkp = q(k, p), qkr = q(k, r);
                    q(k, p) = c * qkp - sn * qkr;
                    q(k, r) = sn * qkp + c * qkr;
                }
                for (int k = 0; k < n; ++k) {  // rows p, r of A
                    const double apk = a(p, k), ark = a(r, k);
                    a(p, k) = c * apk - sn * ark;
                    a(r, k) = sn * apk + c * ark;
                }
            }
    }
    std::vector<std::pair<double, double>> nw(n);
    for (int j = 0; j < n; ++j) nw[j] = {a(j, j), 2.0 * q(0, j) * q(0, j)};
    std::sort(nw.begin(), nw.end());
    // the rule is symmetric about 0: average each node with its mirror
    for (int j = 0; j < n; ++j) {
        const auto &m = nw[n - 1 - j];
        x[j] = 0.5 * (nw[j].first - m.first);
        w[j] = 0.5 * (nw[j].second + m.second);
    }
    // the weights integrate 1 exactly
    double sw = 0.0;
    for (int j = 0; j < n; ++j) sw += w[j];
    for (int j = 0; j < n; ++j) w[j] *= 2.0 / sw;
}

void quadrature_constants() {
    double b[7][3], w[7], gx[32], gw[32];
    const double s15 = std::sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    b[0][0] = b[0][1] = b[0][2] = 1.0 / 3.0;
    w[0] = 9.0 / 40.0;
    for (int p = 0; p < 3; ++p) {
        for (int q = 0; q < 3; ++q) {
            b[1 + p][q] = (q == p) ? 1 - 2 * a1 : a1;
            b[4 + p][q] = (q == p) ? 1 - 2 * a2 : a2;
        }
        w[1 + p] = (155.0 - s15) / 1200.0;
        w[4 + p] = (155.0 + s15) / 1200.0;
    }
    legendre_nodes(32, gx, gw);
    hip_check(set_quadrature_constants(b, w, gx, gw), "quadrature constants");
}

template <class T>
T *upload_to(fda_plan *p, const std::vector<T> &v, std::vector<void *> &list) {
    T *d = dalloc<T>(p, v.size(), list);
    if (!v.empty()) hip_check(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "upload");
    return d;
}

void build_m2l_list(fda_plan *p, M2LMerged &mm, std::vector<void *> &fresh);

// The merged low-rank M2L work list of the plan's configuration p->m2l_cfg:
// per level, the pairs of every translation in work items of `width` pairs
// (16 for ranks above 64: the kernel holds at most 8 phase-1 tiles per item)
// and a reduction entry for every state of the level, summing its pair
// products in a fixed order (translation, then pair: the same for every
// configuration).  The new device arrays
// replace the previous list's only once all of them are in place (on an
// error the previous list stays); the caller has made sure that none of the
// previous arrays is in use.
void build_m2l_merged(fda_plan *p) {
    std::vector<void *> fresh;
    const int64_t bytes0 = p->device_bytes;
    M2LMerged nm;
    try {
        build_m2l_list(p, nm, fresh);
    } catch (...) {
        for (void *q : fresh) (void)hipFree(q);
        p->device_bytes = bytes0;
        throw;
    }
    M2LMerged &mm = p->d.m2l_all;
    nm.tmp = mm.tmp;
    mm = std::move(nm);
    for (void *q : p->m2l_allocs) hipFree(q);
    p->device_bytes -= p->m2l_bytes;
    p->m2l_allocs = std::move(fresh);
    p->m2l_bytes = p->device_bytes - bytes0;
}

void build_m2l_list(fda_plan *p, M2LMerged &mm, std::vector<void *> &fresh) {
    std::vector<int32_t> hdr, src, dst, off{0}, list, lev;
    std::vector<int32_t> ent, nst;  // many-column form: per list entry and per state
    std::vector<std::vector<int32_t>> queue[8];  // per XCD queue (or queue 0 only): header + sources of each item
    std::vector<M2LLevelArgs> args;
    int64_t nscratch = 0, nz = 0;
    const bool xcd = p->m2l_cfg.xcd_order != 0;
    for (const auto &lh : p->m2l_host) {
        const size_t width = p->m2l_cfg.width[lh.level] == 16 ? 16 : kGemmCols;
        GWorkHost g;
        for (size_t op = 0; op < lh.by_op.size(); ++op) {
            const auto &v = lh.by_op[op];
            const size_t step = lh.prank[op] > 64 ? 16 : width;
            for (size_t q0 = 0; q0 < v.size(); q0 += step) {
                size_t q1 = std::min(v.size(), q0 + step);
                std::vector<int32_t> srcs, dsts;
                for (size_t q = q0; q < q1; ++q) {
                    srcs.push_back(v[q].first);
                    dsts.push_back(v[q].second);
                }
                g.add((int32_t)op, srcs, dsts);
            }
        }
        const int slot = (int)args.size();
        M2LLevelArgs la = lh.la;
        la.tbase = nscratch;
        la.ldt = (la.kd + 3) & ~3;
        la.zbase = nz;
        args.push_back(la);
        nscratch += g.ncol * (int64_t)la.ldt;
        nz += g.ncol * (int64_t)la.rmax;
        std::vector<int32_t> col_op(g.ncol, 0);  // translation of each pair column
        for (size_t i = 0; i < g.hdr.size() / 4; ++i)
            for (int32_t b = 0; b < g.hdr[4 * i + 2]; ++b) col_op[g.hdr[4 * i + 1] + b] = g.hdr[4 * i];
        // XCD order: each level's items are split into 8 contiguous chunks,
        // one per XCD queue, so every XCD gets the same share of every level
        // (and consecutive items of a translation share an L2)
        const int64_t ni = (int64_t)g.hdr.size() / 4;
        for (int x = 0; x < (xcd ? 8 : 1); ++x)
            for (int64_t i = xcd ? ni * x / 8 : 0; i < (xcd ? ni * (x + 1) / 8 : ni); ++i) {
                std::vector<int32_t> item{g.hdr[4 * i], g.hdr[4 * i + 1], g.hdr[4 * i + 2], slot};
                item.insert(item.end(), g.src.begin() + i * kGemmCols, g.src.begin() + (i + 1) * kGemmCols);
                queue[x].push_back(std::move(item));
            }
        for (int64_t s = 0; s < lh.nstates; ++s) {
            dst.push_back((int32_t)s);
            lev.push_back(slot);
            auto it = g.dest_index.find((int32_t)s);
            int32_t steps = 0;
            if (it != g.dest_index.end()) {
                const auto &pl = g.parts[it->second];
                list.insert(list.end(), pl.begin(), pl.end());
                for (int32_t c : pl) {
                    const int32_t op = col_op[c], ks = lh.prank[op] / 4;
                    ent.insert(ent.end(), {c, op, ks, 0});
                    steps += ks;
                }
            }
            off.push_back((int32_t)list.size());
            nst.push_back(steps);
        }
    }
    // launch order: XCD order has block b run on XCD b % 8 (round-robin
    // dispatch) take item b / 8 of that XCD's queue, short queues padded
    // with empty items; otherwise block b takes item b
    size_t qmax = 0;
    for (auto &q : queue) qmax = std::max(qmax, q.size());
    for (size_t t = 0; t < qmax; ++t)
        for (int x = 0; x < (xcd ? 8 : 1); ++x) {
            if (t < queue[x].size()) {
                const auto &it = queue[x][t];
                hdr.insert(hdr.end(), it.begin(), it.begin() + 4);
                src.insert(src.end(), it.begin() + 4, it.end());
            } else {
                hdr.insert(hdr.end(), {0, 0, 0, 0});
                src.insert(src.end(), kGemmCols, -1);
            }
        }
    mm.nwork = (int)(hdr.size() / 4);
    mm.nred = (int)dst.size();
    mm.nlev = (int)args.size();
    // reduction blocks per level: kRedRows (state, row) entries each
    std::vector<int32_t> rblock{0}, rstate{0};
    for (size_t q = 0; q < args.size(); ++q) {
        const int64_t ns = p->m2l_host[q].nstates, entries = ns * args[q].kd;
        rblock.push_back(rblock.back() + (int32_t)((entries + kRedRows - 1) / kRedRows));
        rstate.push_back(rstate.back() + (int32_t)ns);
    }
    mm.nredblocks = rblock.back();
    // destination-major units of the many-column form, the last level slot
    // (the longest lists) first; the form needs its Z (rmax rows per pair)
    // to fit in the scratch of the kd-row columns
    std::vector<int32_t> units;
    if (nz <= nscratch)
        for (int q = (int)args.size() - 1; q >= 0; --q) {
            const int nt = (args[q].kd + 15) / 16;
            for (int64_t s = 0; s < p->m2l_host[q].nstates; ++s)
                for (int rt = 0; rt < nt; ++rt) units.insert(units.end(), {rstate[q] + (int32_t)s, rt, q, 0});
        }
    mm.nzunits = (int)(units.size() / 4);
    mm.nscratch = nscratch;
    mm.hargs = args;
    mm.variant = p->m2l_cfg.variant;
    if (mm.nwork > 0) {
        mm.hdr = (int4 *)upload_to(p, hdr, fresh);
        mm.src = upload_to(p, src, fresh);
        mm.rd_dst = upload_to(p, dst, fresh);
        mm.rd_off = upload_to(p, off, fresh);
        mm.rd_list = upload_to(p, list, fresh);
        mm.rd_lev = upload_to(p, lev, fresh);
        mm.rd_block = upload_to(p, rblock, fresh);
        mm.rd_state = upload_to(p, rstate, fresh);
        if (mm.nzunits > 0) {
            mm.rd_ent = (int4 *)upload_to(p, ent, fresh);
            mm.rd_nst = upload_to(p, nst, fresh);
            mm.zunits = (int4 *)upload_to(p, units, fresh);
        }
        mm.args = dalloc<M2LLevelArgs>(p, args.size(), fresh);
        if (p->cap_nrhs > 0) {
            // work buffers exist: point the level table at them
            for (auto &la : mm.hargs) {
                la.X = p->d.lv[la.level].s;
                la.Y = p->d.lv[la.level].c;
            }
            hip_check(hipMemcpy(mm.args, mm.hargs.data(), sizeof(M2LLevelArgs) * mm.hargs.size(),
                                hipMemcpyHostToDevice),
                      "M2L level table");
        }
    }
}

void upload_plan(fda_plan *p, const HostOps &ops, DevTranslations &tr) {
    HostPlan &hp = p->hp;
    DevPlan &d = p->d;
    const int L = hp.depth;
    d.n = hp.n;
    d.nleaf = (int)hp.nleaf;
    d.depth = L;
    d.top = hp.top;
    d.max_leaf = hp.max_leaf_count;
    d.k = hp.k;
    d.h_max = hp.h_max;
    d.alpha = make_double2(hp.alpha.real(), hp.alpha.imag());
    p->m2l_cfg.variant = 0;
    p->m2l_cfg.xcd_order = 1;
    bool any = false;
    for (int l = hp.top; l <= L; ++l)
        if (!hp.lv[l].offsets.empty()) any = true;
    d.has_far = any;

    d.perm = upload(p, hp.perm);
    d.tri = upload(p, hp.tri);
    d.cen = upload(p, hp.cen);
    d.nrm = upload(p, hp.nrm);
    d.area = upload(p, hp.area);
    d.leaf_off = upload(p, hp.leaf_off);
    // near field
    std::vector<int32_t> nl_off(hp.nf_list_off.begin(), hp.nf_list_off.end());
    d.nf_list_off = upload(p, nl_off);
    d.nf_list = upload(p, hp.nf_list);
    d.nf_blk_off = upload(p, hp.nf_blk_off);
    d.nf_ncol = upload(p, hp.nf_ncol);
    std::vector<int64_t> col_off(d.nleaf + 1, 0);
    std::vector<int32_t> cols, self_col(d.nleaf, 0);
    int max_ncol = 0;
    for (int b = 0; b < d.nleaf; ++b) {
        int c = 0;
        for (int64_t q = hp.nf_list_off[b]; q < hp.nf_list_off[b + 1]; ++q) {
            int s = hp.nf_list[q];
            if (s == b) self_col[b] = c;
            for (int64_t e = hp.leaf_off[s]; e < hp.leaf_off[s + 1]; ++e) {
                cols.push_back((int32_t)e);
                ++c;
            }
        }
        col_off[b + 1] = (int64_t)cols.size();
        max_ncol = std::max(max_ncol, c);
    }
    // rows up to kP2PShortCols columns stage x in LDS (k_p2p); longer rows
    // read it through the column list (k_p2p_direct, no LDS), so the row
    // length is bounded only by the 32-bit entry index of a leaf's block in
    // the quadrature kernel
    for (int b = 0; b < d.nleaf; ++b)
        if ((int64_t)hp.nf_ncol[b] * (hp.leaf_off[b + 1] - hp.leaf_off[b]) > INT32_MAX)
            throw BuildError{FDA_EINVAL, "near-field block of one leaf above 2^31 entries (lower max_leaf)"};
    d.max_ncol = max_ncol;
    {
        // near-field work items: rows of one leaf, about kP2PItemEntries
        // block entries each; short rows first
        std::vector<int32_t> items[2];
        int cols_short = 0;
        for (int b = 0; b < d.nleaf; ++b) {
            const int nc = hp.nf_ncol[b], nt = (int)(hp.leaf_off[b + 1] - hp.leaf_off[b]);
            const int rows = std::max(4, kP2PItemEntries / std::max(nc, 1));
            const int g = nc <= kP2PShortCols ? 0 : 1;
            if (g == 0) cols_short = std::max(cols_short, nc);
            for (int r0 = 0; r0 < nt; r0 += rows) items[g].insert(items[g].end(), {b, r0, std::min(nt, r0 + rows), 0});
        }
        d.p2p_nshort = (int)(items[0].size() / 4);
        d.p2p_nitems = d.p2p_nshort + (int)(items[1].size() / 4);
        d.p2p_cols_short = cols_short;
        items[0].insert(items[0].end(), items[1].begin(), items[1].end());
        d.p2p_items = (int4 *)upload(p, items[0]);
    }
    d.nf_col_off = upload(p, col_off);
    d.nf_cols = upload(p, cols);
    d.nf_self_col = upload(p, self_col);
    d.prec = hp.opt.prec == FDA_PREC_FP32 ? 1 : 0;
    d.nf_vals = nullptr;  // filled after the near-field quadrature (fda_build)
    // block-Jacobi storage
    std::vector<int64_t> bj_off(d.nleaf + 1, 0);
    for (int b = 0; b < d.nleaf; ++b) {
        int64_t n = hp.leaf_off[b + 1] - hp.leaf_off[b];
        bj_off[b + 1] = bj_off[b] + n * n;
    }
    d.bj_off = upload(p, bj_off);
    {
        const double lam = 2.0 * 3.14159265358979323846 / hp.k;
        std::vector<float> sc(2 * (size_t)d.nleaf);
        for (int b = 0; b < d.nleaf; ++b) {
            sc[2 * b] = (float)(hp.lv[hp.leaf_level[b]].w / lam);
            sc[2 * b + 1] = (float)(hp.h_max / lam);
        }
        d.leaf_scalars = upload(p, sc);
        std::vector<int64_t> roff;
        std::vector<int32_t> rleaf, rn;
        for (int b = 0; b < d.nleaf; ++b)
            for (int64_t e = hp.leaf_off[b]; e < hp.leaf_off[b + 1]; e += kMlpLeaf) {
                roff.push_back(e);
                rleaf.push_back(b);
                rn.push_back((int32_t)std::min<int64_t>(kMlpLeaf, hp.leaf_off[b + 1] - e));
            }
        d.mlp_nrows = (int64_t)roff.size();
        d.mlp_row_off = upload(p, roff);
        d.mlp_row_leaf = upload(p, rleaf);
        d.mlp_row_n = upload(p, rn);
    }
    d.bj_inv = dalloc<double2>(p, (size_t)bj_off[d.nleaf], p->allocs);

    d.lv.assign(L + 1, DevLevel());
    if (!d.has_far) return;
    d.S = to_storage(p, upload_cplx(p, ops.S), ops.S.size());
    if (!ops.SB.empty()) d.rhs.S = to_storage(p, upload_cplx(p, ops.SB), ops.SB.size());
    d.T = to_storage(p, upload_cplx(p, ops.T), ops.T.size());
    d.leaf_sop = upload(p, ops.sop);
    d.leaf_top = upload(p, ops.top);
    for (int l = hp.top; l <= L; ++l) {
        const Level &lv = hp.lv[l];
        DevLevel &dl = d.lv[l];
        dl.nbox = lv.nbox;
        if (!lv.leaves.empty()) {
            std::vector<int32_t> box;
            for (int32_t t : lv.leaves) box.push_back(hp.leaf_box[t]);
            dl.nleaves = (int)lv.leaves.size();
            dl.leaf_ids = upload(p, lv.leaves);
            dl.leaf_box = upload(p, box);
        }
        dl.nslot = lv.nslot;
        dl.ku = lv.ku;
        dl.kd = lv.kd;
        if (lv.ku > 1024 || lv.kd > 1024) throw BuildError{FDA_EINVAL, "compressed rank above 1024"};
        dl.sstride = lv.nbox * lv.nslot * (int64_t)lv.ku;
        dl.cstride = lv.nbox * lv.nslot * (int64_t)lv.kd;
        dl.K = to_storage(p, tr.K[l], lv.offsets.size() * (size_t)lv.kd * lv.ku);
        if (!tr.rmax.empty() && tr.rmax[l] > 0 && lv.kd <= 256) {
            dl.Ulr = to_storage(p, tr.Ulr[l], lv.offsets.size() * (size_t)lv.kd * tr.rmax[l]);
            dl.Vlr = to_storage(p, tr.Vlr[l], lv.offsets.size() * (size_t)tr.rmax[l] * ((lv.ku + 3) / 4 * 4));
            dl.lr_rank = tr.lr_rank[l];
            dl.rmax = tr.rmax[l];
        }
        // M2L pairs sorted by translation; work items of <= 32 pairs; the
        // pairs of every target state in a fixed order
        {
            const size_t no = lv.offsets.size();
            std::vector<std::vector<std::pair<int32_t, int32_t>>> by_op(no);  // (src state, tgt state)
            for (int64_t b = 0; b < lv.nbox; ++b)
                for (size_t q = 0; q < lv.il[b].size(); ++q) {
                    int op = lv.il_ops[b][q];
                    int sl = lv.il_slots[b][q];
                    by_op[op].push_back({(int32_t)(lv.il[b][q] * lv.nslot + sl), (int32_t)(b * lv.nslot + sl)});
                }
            // the low-rank kernel holds at most 8 phase-1 tiles per item:
            // translations of padded rank above 64 get 16-column items
            std::vector<int32_t> prank(no, 0);
            if (dl.rmax > 0)
                for (size_t op = 0; op < no; ++op) {
                    const int rt = tr.true_rank[l][op];
                    prank[op] = std::min(std::min(lv.kd, lv.ku), (rt + 3) / 4 * 4);
                }
            if (dl.rmax > 0) {
                // low-rank level: its pairs go to the merged list, built
                // below for the plan's configuration
                dl.merged = true;
                fda_plan::M2LLevelHost lh;
                lh.level = l;
                lh.nstates = lv.nbox * (int64_t)lv.nslot;
                lh.by_op = std::move(by_op);
                lh.prank = std::move(prank);
                lh.la.U = dl.Ulr;
                lh.la.V = dl.Vlr;
                lh.la.rank = dl.lr_rank;
                lh.la.kd = lv.kd;
                lh.la.ku = lv.ku;
                lh.la.rmax = dl.rmax;
                lh.la.level = l;
                lh.la.xstride = dl.sstride;
                lh.la.ystride = dl.cstride;
                p->m2l_host.push_back(std::move(lh));
                p->m2l_cfg.width[l] = kGemmCols;
            } else {
                GWorkHost g;
                for (size_t op = 0; op < no; ++op) {
                    const auto &v = by_op[op];
                    for (size_t q0 = 0; q0 < v.size(); q0 += kGemmCols) {
                        size_t q1 = std::min(v.size(), q0 + kGemmCols);
                        std::vector<int32_t> srcs, dsts;
                        for (size_t q = q0; q < q1; ++q) {
                            srcs.push_back(v[q].first);
                            dsts.push_back(v[q].second);
                        }
                        g.add((int32_t)op, srcs, dsts);
                    }
                }
                dl.m2l = upload_gwork(p, g, lv.kd);
            }
        }
        if (l < L) {
            const Level &C = hp.lv[l + 1];
            dl.M = to_storage(p, tr.M[l], 8 * (size_t)lv.nslot * lv.ku * C.ku);
            dl.Lo = to_storage(p, tr.Lo[l], 8 * (size_t)lv.nslot * C.kd * lv.kd);
            // M2M: per (child octant, parent slot), the parents with a child
            // in that octant, in chunks
            GWorkHost gm;
            for (int o = 0; o < 8; ++o)
                for (int s = 0; s < lv.nslot; ++s) {
                    std::vector<int32_t> srcs, dsts;
                    auto flush = [&]() {
                        if (!srcs.empty()) gm.add(o * lv.nslot + s, srcs, dsts);
                        srcs.clear();
                        dsts.clear();
                    };
                    for (int64_t b = 0; b < lv.nbox; ++b)
                        for (int32_t c = lv.child_begin[b]; c < lv.child_begin[b + 1]; ++c)
                            if (C.octant[c] == o) {
                                srcs.push_back(c * C.nslot + lv.cslot[s]);
                                dsts.push_back((int32_t)(b * lv.nslot + s));
                                if ((int)srcs.size() == kGemmCols) flush();
                            }
                    flush();
                }
            dl.m2m = upload_gwork(p, gm, lv.ku);
            p->m2m_flops += 8.0 * lv.ku * C.ku * (double)gm.ncol;
            // L2L: per (child octant, parent slot), the children in that
            // octant, in chunks; summed into the child slot fed by the parent slot
            GWorkHost gl;
            for (int o = 0; o < 8; ++o)
                for (int s = 0; s < lv.nslot; ++s) {
                    const int cs = lv.cslot[s];
                    std::vector<int32_t> srcs, dsts;
                    auto flush = [&]() {
                        if (!srcs.empty()) gl.add(o * lv.nslot + s, srcs, dsts);
                        srcs.clear();
                        dsts.clear();
                    };
                    for (int64_t c = 0; c < C.nbox; ++c)
                        if (C.octant[c] == o) {
                            srcs.push_back((int32_t)(C.parent[c] * lv.nslot + s));
                            dsts.push_back((int32_t)(c * C.nslot + cs));
                            if ((int)srcs.size() == kGemmCols) flush();
                        }
                    flush();
                }
            dl.l2l = upload_gwork(p, gl, C.kd);
            p->l2l_flops += 8.0 * C.kd * lv.kd * (double)gl.ncol;
        }
    }
    build_m2l_merged(p);
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

}  // namespace

extern "C" {

void fda_default_options(fda_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_leaf = 64;
    o->p_min = 0;
    o->p0 = 1;
    o->svd_eps = 0.0;
    o->alpha_re = 0.0;
    o->alpha_im = 0.0;
    o->hf_wavelengths = 1.9;
    o->rho_c = 1.0;
    o->leaf_min_h = 2.5;
    o->prec = FDA_PREC_FP64;
    o->nrhs_max = 64;
    o->device = 0;
    o->verbose = 0;
    o->svd_method = 1;
}

const char *fda_last_error(void) { return g_last_error.c_str(); }

const char *fda_version(void) { return "fda-mi355x 0.1 (gfx950)"; }

int fda_inspect(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k, double eps,
                const fda_options *opt, fda_stats *st) {
    g_last_error.clear();
    if (!st) return fail(FDA_EINVAL, "st is NULL");
    fda_options o;
    fda_default_options(&o);
    if (opt) o = *opt;
    try {
        HostPlan hp;
        host_setup(verts, nv, tris, nt, k, eps, o, hp);
        fill_stats(hp, st);
    } catch (const BuildError &e) {
        return fail(e.code, e.msg);
    } catch (const std::exception &e) {
        return fail(FDA_ENOMEM, e.what());
    }
    return FDA_OK;
}

int fda_build(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double k, double eps,
              const fda_options *opt, fda_plan **out) {
    g_last_error.clear();
    if (!out) return fail(FDA_EINVAL, "out is NULL");
    *out = nullptr;
    fda_options o;
    fda_default_options(&o);
    if (opt) o = *opt;
    if (o.nrhs_max < 1 || o.nrhs_max > 4096) return fail(FDA_EINVAL, "nrhs_max must be in [1, 4096]");
    if (o.prec != FDA_PREC_FP64 && o.prec != FDA_PREC_FP32) return fail(FDA_EINVAL, "prec must be FDA_PREC_FP64 or FDA_PREC_FP32");
    if (o.svd_method != 0 && o.svd_method != 1) return fail(FDA_EINVAL, "svd_method must be 0 or 1");
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<fda_plan> p(new fda_plan());
    p->device = o.device;
    rocblas_handle rb = nullptr;
    DevTranslations tr;
    std::vector<std::vector<int32_t>> lr_rank_host;
    std::vector<int> tr_rmax(25, 0);
    std::vector<double> tr_mean(25, 0.0);
    double phase[8] = {0};
    auto tick = std::chrono::steady_clock::now();
    auto lap = [&](int q) {  // wall time of build phase q (device work synchronised)
        hipDeviceSynchronize();
        auto now = std::chrono::steady_clock::now();
        phase[q] += std::chrono::duration<double>(now - tick).count();
        tick = now;
    };
    try {
        hip_check(hipSetDevice(o.device), "hipSetDevice");
        host_setup(verts, nv, tris, nt, k, eps, o, p->hp);
        lap(0);
        bool any = false;
        for (int l = p->hp.top; l <= p->hp.depth; ++l)
            if (!p->hp.lv[l].offsets.empty()) any = true;
        if (any) {
            if (rocblas_create_handle(&rb) != rocblas_status_success) throw BuildError{FDA_EHIP, "rocblas_create_handle failed"};
            device_factors(p->hp, rb);
            lap(1);
            device_translations(p->hp, rb, tr);
            lap(2);
            device_lowrank_m2l(p->hp, rb, tr, kLowRankMax);
            lap(3);
            lr_rank_host.assign(p->hp.depth + 1, {});
            for (int l = 0; l <= p->hp.depth; ++l) {
                tr_rmax[l] = tr.rmax[l];
                tr_mean[l] = tr.mean_rank[l];
                if (tr.rmax[l] > 0 && p->hp.lv[l].kd <= 256) lr_rank_host[l] = tr.true_rank[l];
            }
            p->allocs.insert(p->allocs.end(), tr.allocs.begin(), tr.allocs.end());
            p->device_bytes += tr.bytes;
            tr.allocs.clear();
        }
        HostOps ops;
        form_operators(p->hp, ops);
        lap(4);
        quadrature_constants();
        upload_plan(p.get(), ops, tr);
        lap(5);
        {
            // near-field quadrature in FP64; block-Jacobi inverses from it;
            // FP32 plans keep the off-diagonal entries in FP32 and the self
            // terms in FP64
            double2 *v64 = dalloc<double2>(p.get(), (size_t)p->hp.near_nnz, p->allocs);
            hip_check(launch_near_blocks(p->d, v64, nullptr), "near-field blocks");
            hip_check(launch_bj_invert(p->d, v64, nullptr), "block-Jacobi inverses");
            if (p->d.prec == FDA_PREC_FP32) {
                p->d.nf_vals = dalloc<float2>(p.get(), (size_t)p->hp.near_nnz, p->allocs);
                p->d.nf_diag = dalloc<double2>(p.get(), (size_t)p->d.n, p->allocs);
                hip_check(launch_near_split(p->d, v64, p->d.nf_vals, p->d.nf_diag, nullptr), "near-field split");
                hip_check(hipDeviceSynchronize(), "near split");
                auto it = std::find(p->allocs.begin(), p->allocs.end(), (void *)v64);
                hipFree(v64);
                p->allocs.erase(it);
                p->device_bytes -= (int64_t)(sizeof(double2) * p->hp.near_nnz);
            } else {
                p->d.nf_vals = v64;
            }
            if (p->hp.opt.neumann_rhs) {
                // the right-hand operator B: its own near-field blocks (same
                // pattern and quadrature), stored like A's
                double2 *b64 = dalloc<double2>(p.get(), (size_t)p->hp.near_nnz, p->allocs);
                hip_check(launch_near_blocks(p->d, b64, nullptr, 1), "near-field blocks of B");
                if (p->d.prec == FDA_PREC_FP32) {
                    p->d.rhs.nf_vals = dalloc<float2>(p.get(), (size_t)p->hp.near_nnz, p->allocs);
                    p->d.rhs.nf_diag = dalloc<double2>(p.get(), (size_t)p->d.n, p->allocs);
                    hip_check(launch_near_split(p->d, b64, p->d.rhs.nf_vals, p->d.rhs.nf_diag, nullptr),
                              "near-field split of B");
                    hip_check(hipDeviceSynchronize(), "near split");
                    auto it = std::find(p->allocs.begin(), p->allocs.end(), (void *)b64);
                    hipFree(b64);
                    p->allocs.erase(it);
                    p->device_bytes -= (int64_t)(sizeof(double2) * p->hp.near_nnz);
                } else {
                    p->d.rhs.nf_vals = b64;
                }
                p->d.has_rhs = true;
            }
        }
        hip_check(hipDeviceSynchronize(), "build synchronize");
        lap(6);
    } catch (const BuildError &e) {
        for (void *q : tr.allocs) hipFree(q);
        for (void *q : p->allocs) hipFree(q);
        if (rb) rocblas_destroy_handle(rb);
        return fail(e.code, e.msg);
    } catch (const HipError &e) {
        for (void *q : tr.allocs) hipFree(q);
        for (void *q : p->allocs) hipFree(q);
        if (rb) rocblas_destroy_handle(rb);
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc &) {
        for (void *q : tr.allocs) hipFree(q);
        for (void *q : p->allocs) hipFree(q);
        if (rb) rocblas_destroy_handle(rb);
        return fail(FDA_ENOMEM, "host allocation failed");
    }
    if (rb) rocblas_destroy_handle(rb);
    fill_stats(p->hp, &p->stats);
    p->stats.m2m_flops = p->m2m_flops;
    p->stats.l2l_flops = p->l2l_flops;
    p->stats.mlp_rows = p->d.mlp_nrows;
    {
        // algorithmic M2L flops per level: low-rank levels count
        // 8 r (kd + ku) real flops per pair with the SVD rank r of its
        // translation (before the kernel pads it to a multiple of 4); full
        // levels 8 kd ku
        int64_t tot = 0;
        const int64_t es = p->d.prec == FDA_PREC_FP32 ? 8 : 16;  // bytes per complex entry
        for (int l = 0; l <= p->hp.depth && l < 24; ++l) {
            const Level &lv = p->hp.lv[l];
            double f = 0;
            if (!lr_rank_host.empty() && !lr_rank_host[l].empty()) {
                for (const auto &ops : lv.il_ops)
                    for (int op : ops) f += 8.0 * lr_rank_host[l][op] * (lv.kd + lv.ku);
                for (int r : lr_rank_host[l]) p->stats.m2l_factor_bytes += es * r * (int64_t)(lv.kd + lv.ku);
                p->stats.m2l_state_bytes += es * lv.nbox * (int64_t)lv.nslot * (lv.kd + lv.ku);
                p->stats.m2l_rank_max[l] = tr_rmax[l];
            } else {
                int64_t pairs = 0;
                for (auto &x : lv.il) pairs += (int64_t)x.size();
                f = 8.0 * pairs * lv.kd * lv.ku;
            }
            p->stats.m2l_rank_mean[l] = tr_mean[l];
            p->stats.m2l_level_flops[l] = f;
            tot += (int64_t)f;
        }
        p->stats.m2l_flops = tot;
    }
    p->stats.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < 8; ++q) p->stats.build_phase_seconds[q] = phase[q];
    p->stats.device_bytes = p->device_bytes;
    if (p->d.has_far) {
        // a side stream (default priority) for the near field; without it
        // the near field runs on the caller's stream before the far field
        fda::DevPlan &d = p->d;
        if (hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&d.join, hipEventDisableTiming) != hipSuccess) {
            if (d.side) hipStreamDestroy(d.side);
            if (d.fork) hipEventDestroy(d.fork);
            if (d.join) hipEventDestroy(d.join);
            d.side = nullptr;
            d.fork = d.join = nullptr;
            hipGetLastError();
        }
    }
    *out = p.release();
    return FDA_OK;
}

int fda_plan_stats(const fda_plan *plan, fda_stats *st) {
    if (!plan || !st) return fail(FDA_EINVAL, "NULL argument");
    *st = plan->stats;
    st->device_bytes = plan->device_bytes;
    return FDA_OK;
}

void fda_free(fda_plan *plan) {
    if (!plan) return;
    hipSetDevice(plan->device);
    if (plan->d.side) {
        hipStreamSynchronize(plan->d.side);
        hipStreamDestroy(plan->d.side);
        hipEventDestroy(plan->d.fork);
        hipEventDestroy(plan->d.join);
    }
    free_work(plan);
    for (void *q : plan->m2l_allocs) hipFree(q);
    for (void *q : plan->allocs) hipFree(q);
    delete plan;
}

int fda_matvec(fda_plan *plan, const void *x_dev, void *y_dev, int64_t nrhs, int64_t ld, void *stream) {
    g_last_error.clear();
    if (!plan || !x_dev || !y_dev) return fail(FDA_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > plan->hp.opt.nrhs_max) return fail(FDA_EINVAL, "nrhs out of range");
    if (ld < plan->d.n) return fail(FDA_EINVAL, "ld < N");
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        ensure_capacity(plan, (int)nrhs);
        hipStream_t st = as_stream(stream);
        hip_check(launch_permute_in(plan->d, (const double2 *)x_dev, ld, plan->xt, (int)nrhs, st), "permute");
        hip_check(launch_matvec_tree(plan->d, plan->xt, plan->yt, (int)nrhs, st, nullptr, nullptr), "matvec");
        hip_check(launch_permute_out(plan->d, plan->yt, (double2 *)y_dev, ld, (int)nrhs, st), "permute");
    } catch (const BuildError &e) {
        return fail(e.code, e.msg);
    } catch (const HipError &e) {
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return FDA_OK;
}

int bm_rhs_neumann(fda_plan *plan, const void *g_dev, void *b_dev, int64_t nrhs, int64_t ld, void *stream) {
    g_last_error.clear();
    if (!plan || !g_dev || !b_dev) return fail(FDA_EINVAL, "NULL argument");
    if (!plan->d.has_rhs) return fail(FDA_EINVAL, "plan built without neumann_rhs (the operator B)");
    if (nrhs < 1 || nrhs > plan->hp.opt.nrhs_max) return fail(FDA_EINVAL, "nrhs out of range");
    if (ld < plan->d.n) return fail(FDA_EINVAL, "ld < N");
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        ensure_capacity(plan, (int)nrhs);
        hipStream_t st = as_stream(stream);
        hip_check(launch_permute_in(plan->d, (const double2 *)g_dev, ld, plan->xt, (int)nrhs, st), "permute");
        hip_check(launch_matvec_tree(plan->d, plan->xt, plan->yt, (int)nrhs, st, nullptr, nullptr, &plan->d.rhs),
                  "B product");
        hip_check(launch_permute_out(plan->d, plan->yt, (double2 *)b_dev, ld, (int)nrhs, st), "permute");
    } catch (const BuildError &e) {
        return fail(e.code, e.msg);
    } catch (const HipError &e) {
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return FDA_OK;
}

int fda_profile_matvec(fda_plan *plan, const void *x_dev, void *y_dev, int64_t nrhs, int64_t ld, int32_t reps,
                       void *stream, fda_profile_result *out) {
    g_last_error.clear();
    if (!plan || !x_dev || !y_dev || !out || reps < 1) return fail(FDA_EINVAL, "bad argument");
    if (nrhs < 1 || nrhs > plan->hp.opt.nrhs_max || ld < plan->d.n) return fail(FDA_EINVAL, "nrhs / ld out of range");
    std::memset(out, 0, sizeof(*out));
    hipEvent_t ev[9], lev[50];  // 2 per level (full-rank M2L) + 2 around the merged low-rank M2L
    for (auto &e : ev) hipEventCreate(&e);
    for (auto &e : lev) hipEventCreate(&e);
    int rc = FDA_OK;
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        ensure_capacity(plan, (int)nrhs);
        hipStream_t st = as_stream(stream);
        const int L = plan->d.depth;
        for (int r = 0; r < reps; ++r) {
            // record every level's pair (outside the timed region) so that
            // elapsed-time queries are valid for levels without M2L work
            for (int l = 0; l < 25; ++l) {
                hipEventRecord(lev[2 * l], st);
                hipEventRecord(lev[2 * l + 1], st);
            }
            hip_check(hipEventRecord(ev[7], st), "event");
            hip_check(launch_permute_in(plan->d, (const double2 *)x_dev, ld, plan->xt, (int)nrhs, st), "permute");
            hip_check(launch_matvec_tree(plan->d, plan->xt, plan->yt, (int)nrhs, st, ev, lev), "matvec");
            hip_check(launch_permute_out(plan->d, plan->yt, (double2 *)y_dev, ld, (int)nrhs, st), "permute");
            hip_check(hipEventRecord(ev[8], st), "event");
            hip_check(hipEventSynchronize(ev[8]), "sync");
            float ms;
            double *stage[5] = {&out->near_ms, &out->s2m_ms, &out->m2m_ms, &out->m2l_ms, &out->l2l_ms};
            for (int q = 0; q < 5; ++q) {
                hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
                *stage[q] += ms;
            }
            float a, b;
            hipEventElapsedTime(&ms, ev[5], ev[6]);
            out->l2t_ms += ms;
            hipEventElapsedTime(&a, ev[7], ev[0]);
            hipEventElapsedTime(&b, ev[6], ev[8]);
            out->perm_ms += a + b;
            hipEventElapsedTime(&ms, ev[7], ev[8]);
            out->total_ms += ms;
            for (int l = 0; l <= L && l < 24; ++l) {
                hipEventElapsedTime(&ms, lev[2 * l], lev[2 * l + 1]);
                out->m2l_gemm_ms[l] += ms;
            }
            hipEventElapsedTime(&ms, lev[48], lev[49]);
            out->m2l_lowrank_ms += ms;
        }
        double *all[9] = {&out->near_ms, &out->s2m_ms, &out->m2m_ms,  &out->m2l_ms,        &out->l2l_ms,
                          &out->l2t_ms,  &out->total_ms, &out->perm_ms, &out->m2l_lowrank_ms};
        for (auto *v : all) *v /= reps;
        for (int l = 0; l < 24; ++l) out->m2l_gemm_ms[l] /= reps;
    } catch (const HipError &e) {
        rc = fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const BuildError &e) {
        rc = fail(e.code, e.msg);
    }
    for (auto &e : ev) hipEventDestroy(e);
    for (auto &e : lev) hipEventDestroy(e);
    return rc;
}

int fda_m2l_get_config(const fda_plan *plan, fda_m2l_config *out) {
    g_last_error.clear();
    if (!plan || !out) return fail(FDA_EINVAL, "NULL argument");
    *out = plan->m2l_cfg;
    for (int l = 0; l < 24; ++l) out->width[l] = 0;
    for (const auto &lh : plan->m2l_host) out->width[lh.level] = plan->m2l_cfg.width[lh.level];
    return FDA_OK;
}

namespace {

// Switch the plan to configuration c (rebuilding the merged list when the
// order or a width changes); the device is idle on return.
void apply_m2l_config(fda_plan *p, const fda_m2l_config &c) {
    hip_check(hipDeviceSynchronize(), "sync");
    const fda_m2l_config old = p->m2l_cfg;
    bool rebuild = c.xcd_order != old.xcd_order;
    for (const auto &lh : p->m2l_host) rebuild = rebuild || c.width[lh.level] != old.width[lh.level];
    if (rebuild && p->live_batches > 0)
        throw BuildError{FDA_EINVAL, "a batch graph references the plan's M2L work list; free the batch before "
                                     "changing the item order or widths"};
    p->m2l_cfg.variant = c.variant;
    p->m2l_cfg.xcd_order = c.xcd_order;
    for (const auto &lh : p->m2l_host) p->m2l_cfg.width[lh.level] = c.width[lh.level];
    if (rebuild) {
        try {
            build_m2l_merged(p);
        } catch (...) {
            p->m2l_cfg = old;
            throw;
        }
    }
    p->d.m2l_all.variant = p->m2l_cfg.variant;
}

}  // namespace

int fda_m2l_set_config(fda_plan *plan, const fda_m2l_config *cfg) {
    g_last_error.clear();
    if (!plan || !cfg) return fail(FDA_EINVAL, "NULL argument");
    if (cfg->variant < 0 || cfg->variant >= kM2LVariants) return fail(FDA_EINVAL, "variant out of range");
    if (cfg->xcd_order != 0 && cfg->xcd_order != 1) return fail(FDA_EINVAL, "xcd_order must be 0 or 1");
    for (const auto &lh : plan->m2l_host)
        if (cfg->width[lh.level] != 16 && cfg->width[lh.level] != 32)
            return fail(FDA_EINVAL, "width must be 16 or 32 on level " + std::to_string(lh.level));
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        apply_m2l_config(plan, *cfg);
    } catch (const BuildError &e) {
        return fail(e.code, e.msg);
    } catch (const HipError &e) {
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    return FDA_OK;
}

int fda_autotune(fda_plan *plan, int32_t reps, void *stream, fda_tune_result *out) {
    g_last_error.clear();
    if (!plan || !out) return fail(FDA_EINVAL, "NULL argument");
    if (reps < 1 || reps > 1000) return fail(FDA_EINVAL, "reps out of range");
    if (plan->live_batches > 0) return fail(FDA_EINVAL, "a batch graph references the plan; free it before tuning");
    std::memset(out, 0, sizeof(*out));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FDA_OK;
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hipStream_t st = as_stream(stream);
        out->nlevels = (int32_t)plan->m2l_host.size();
        if (plan->d.m2l_all.nwork > 0) {
            ensure_capacity(plan, 1);
            // current states everywhere: one product of the zero vector
            hip_check(hipMemsetAsync(plan->xt, 0, sizeof(double2) * (size_t)plan->d.n, st), "memset");
            hip_check(launch_matvec_tree(plan->d, plan->xt, plan->yt, 1, st, nullptr, nullptr), "matvec");
            hip_check(hipStreamSynchronize(st), "sync");
            // median of reps launches of the merged M2L (after one untimed)
            auto time_m2l = [&]() {
                hip_check(launch_m2l_merged(plan->d, 1, st), "M2L");
                std::vector<float> t(reps);
                for (int r = 0; r < reps; ++r) {
                    hip_check(hipEventRecord(e0, st), "event");
                    hip_check(launch_m2l_merged(plan->d, 1, st), "M2L");
                    hip_check(hipEventRecord(e1, st), "event");
                    hip_check(hipEventSynchronize(e1), "sync");
                    hip_check(hipEventElapsedTime(&t[r], e0, e1), "elapsed");
                }
                std::sort(t.begin(), t.end());
                ++out->candidates;
                return (double)t[reps / 2];
            };
            fda_m2l_config cur = plan->m2l_cfg;
            double best = time_m2l();
            out->ms_before = best;
            auto trial = [&](const fda_m2l_config &c) {
                apply_m2l_config(plan, c);
                const double t = time_m2l();
                if (t < 0.97 * best) {  // clear of the run-to-run spread of the timings
                    best = t;
                    cur = c;
                } else {
                    apply_m2l_config(plan, cur);
                }
            };
            const int v0 = cur.variant;
            for (int v = 0; v < kM2LVariants; ++v) {
                if (v == v0) continue;
                fda_m2l_config c = cur;
                c.variant = v;
                trial(c);
            }
            {
                fda_m2l_config c = cur;
                c.xcd_order = 1 - c.xcd_order;
                trial(c);
            }
            for (const auto &lh : plan->m2l_host) {
                fda_m2l_config c = cur;
                c.width[lh.level] = c.width[lh.level] == 16 ? 32 : 16;
                trial(c);
            }
            out->ms_after = time_m2l();
            --out->candidates;  // the final timing repeats the chosen one
        }
        fda_m2l_get_config(plan, &out->best);
    } catch (const HipError &e) {
        rc = fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const BuildError &e) {
        rc = fail(e.code, e.msg);
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    return rc;
}

int bm_rhs_planewave(fda_plan *plan, const double *dirs, int64_t nrhs, void *b_dev, int64_t ld, void *stream) {
    g_last_error.clear();
    if (!plan || !dirs || !b_dev) return fail(FDA_EINVAL, "NULL argument");
    if (nrhs < 1 || ld < plan->d.n) return fail(FDA_EINVAL, "nrhs / ld out of range");
    for (int64_t i = 0; i < 3 * nrhs; ++i)
        if (!std::isfinite(dirs[i])) return fail(FDA_EINVAL, "non-finite direction");
    double *dd = nullptr;
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        hip_check(hipMalloc(&dd, sizeof(double) * 3 * nrhs), "hipMalloc");
        hipStream_t st = as_stream(stream);
        hip_check(hipMemcpyAsync(dd, dirs, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, st), "copy");
        hip_check(launch_rhs_planewave(plan->d, dd, (int)nrhs, (double2 *)b_dev, ld, st), "rhs");
        hip_check(hipStreamSynchronize(st), "sync");
    } catch (const HipError &e) {
        if (dd) hipFree(dd);
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    hipFree(dd);
    return FDA_OK;
}

// ------------------------------------------------------------------ GMRES

int bm_solve(fda_plan *plan, const void *b_dev, void *x_dev, int64_t nrhs, int64_t ld, double tol, int32_t restart,
             int32_t maxit, int32_t precond, bm_stats *stp, void *stream) {
    g_last_error.clear();
    if (!plan || !b_dev || !x_dev) return fail(FDA_EINVAL, "NULL argument");
    if (nrhs < 1 || nrhs > plan->hp.opt.nrhs_max || ld < plan->d.n) return fail(FDA_EINVAL, "nrhs / ld out of range");
    if (!(tol > 0) || restart < 1 || restart > 500 || maxit < 1) return fail(FDA_EINVAL, "bad tol / restart / maxit");
    if (precond != FDA_PRECOND_NONE && precond != FDA_PRECOND_BLOCK_JACOBI && precond != FDA_PRECOND_MLP)
        return fail(FDA_EINVAL, "bad precond");
    if (precond == FDA_PRECOND_MLP && (!plan->mlp || !plan->mlp->m))
        return fail(FDA_EINVAL, "FDA_PRECOND_MLP needs a network attached with fda_plan_set_mlp");
    auto t0 = std::chrono::steady_clock::now();
    bm_stats st{};
    const int nr = (int)nrhs, m = restart;
    const int64_t N = plan->d.n;
    hipStream_t s = as_stream(stream);
    std::vector<void *> tmp, pinned;
    auto talloc = [&](size_t bytes) {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) throw BuildError{FDA_ENOMEM, "GMRES workspace allocation failed"};
        tmp.push_back(q);
        return q;
    };
    int rc = FDA_OK;
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        ensure_capacity(plan, nr);
        const size_t vec = sizeof(double2) * (size_t)N * nr;
        double2 *V = (double2 *)talloc(vec * (m + 1));
        double2 *Zs = (double2 *)talloc(vec * m);  // preconditioned basis (flexible GMRES)
        double2 *w = (double2 *)talloc(vec);
        double2 *bt = (double2 *)talloc(vec);
        double2 *xt = (double2 *)talloc(vec);
        double2 *r = (double2 *)talloc(vec);
        double2 *partial = (double2 *)talloc(sizeof(double2) * kRedBlocks * (m + 1) * nr);
        double2 *hd = (double2 *)talloc(sizeof(double2) * (m + 1) * nr);
        double2 *h2 = (double2 *)talloc(sizeof(double2) * (m + 1) * nr);
        double2 *sc = (double2 *)talloc(sizeof(double2) * nr);
        int32_t *act_d = (int32_t *)talloc(sizeof(int32_t) * nr);
        std::vector<int32_t> act(nr, 1);
        // pinned host copies of one Arnoldi step's inner products (the two
        // Gram-Schmidt passes and the norm), read after a single sync
        double2 *hpin[3];
        for (auto &q : hpin) {
            if (hipHostMalloc((void **)&q, sizeof(double2) * (m + 1) * nr, hipHostMallocDefault) != hipSuccess)
                throw BuildError{FDA_ENOMEM, "GMRES pinned buffer allocation failed"};
            pinned.push_back(q);
        }
        // inner products of Vb's mm columns with w into hd, copied to `pin`
        // (stream-ordered: the next kernel that writes hd runs after the copy)
        auto dots_async = [&](const double2 *Vb, int mm, const double2 *wv, double2 *pin) {
            hip_check(launch_multidot(Vb, mm, nr, wv, N, partial, hd, s), "dots");
            hip_check(hipMemcpyAsync(pin, hd, sizeof(double2) * mm * nr, hipMemcpyDeviceToHost, s), "d2h");
        };

        auto dots = [&](const double2 *Vb, int mm, const double2 *wv, std::vector<cplx> &outv) {
            hip_check(launch_multidot(Vb, mm, nr, wv, N, partial, hd, s), "dots");
            outv.resize((size_t)mm * nr);
            hip_check(hipMemcpyAsync(outv.data(), hd, sizeof(double2) * mm * nr, hipMemcpyDeviceToHost, s), "d2h");
            hip_check(hipStreamSynchronize(s), "sync");
        };
        auto norms = [&](const double2 *wv, std::vector<double> &nv) {
            // ||w_c|| via the multidot of w with itself (V = w, m = 1)
            std::vector<cplx> o;
            dots(wv, 1, wv, o);
            nv.resize(nr);
            for (int c = 0; c < nr; ++c) nv[c] = std::sqrt(std::max(0.0, o[c].real()));
        };
        auto apply_A = [&](const double2 *in, double2 *out) {
            hip_check(launch_matvec_tree(plan->d, in, out, nr, s, nullptr, nullptr), "matvec");
        };
        // learned preconditioner workspace (one column at a time)
        float *feat = nullptr, *yml = nullptr;
        double2 *vnorm = nullptr;  // row scales
        double2 *zbj = nullptr;
        int *bad = nullptr;
        if (precond == FDA_PRECOND_MLP) {
            feat = (float *)talloc(sizeof(float) * (size_t)plan->d.mlp_nrows * kMlpIn);
            yml = (float *)talloc(sizeof(float) * (size_t)plan->d.mlp_nrows * kMlpOut);
            vnorm = (double2 *)talloc(sizeof(double2) * (size_t)plan->d.mlp_nrows);
            zbj = (double2 *)talloc(sizeof(double2) * (size_t)N);
            bad = (int *)talloc(sizeof(int));
        }
        // FDA_PRECOND_MLP is judged against block Jacobi: the first kJudge
        // products use block Jacobi, the next kJudge the network; if the
        // network reduced the (Givens) residual estimate by less over its
        // window than block Jacobi did over the first, the rest of the solve
        // uses block Jacobi.  Flexible GMRES allows the switch at any step.
        constexpr int kJudge = 6;
        int cur_pc = precond == FDA_PRECOND_MLP ? FDA_PRECOND_BLOCK_JACOBI : precond;
        int judge_state = precond == FDA_PRECOND_MLP ? 0 : -1;  // 0: BJ window, 1: MLP window, 2: done
        int judge_steps = 0;
        double judge_res0 = 1.0, judge_rate_bj = 0.0;
        auto apply_M = [&](const double2 *in, double2 *out) {
            if (cur_pc == FDA_PRECOND_BLOCK_JACOBI) {
                hip_check(launch_bj_apply(plan->d, in, out, nr, nullptr, s), "precond");
            } else if (cur_pc == FDA_PRECOND_MLP) {
                for (int c = 0; c < nr; ++c) {
                    const double2 *vc = in + (size_t)c * N;
                    double2 *oc = out + (size_t)c * N;
                    int flag = 0;
                    hip_check(hipMemcpyAsync(bad, &flag, sizeof(int), hipMemcpyHostToDevice, s), "h2d");
                    mlp_features(plan->d, vc, plan->d.leaf_scalars, feat, vnorm, zbj, s);
                    plan->mlp->m->forward(feat, plan->d.mlp_nrows, yml, s);
                    mlp_apply(plan->d, yml, vnorm, zbj, oc, bad, s);
                    hip_check(hipGetLastError(), "mlp preconditioner");
                    hip_check(hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, s), "d2h");
                    hip_check(hipStreamSynchronize(s), "sync");
                    if (flag) {  // non-finite network output: fall back to block Jacobi
                        hip_check(hipMemcpyAsync(oc, zbj, sizeof(double2) * (size_t)N, hipMemcpyDeviceToDevice, s),
                                  "fallback");
                        st.mlp_fallbacks++;
                    }
                }
            } else {
                hip_check(hipMemcpyAsync(out, in, vec, hipMemcpyDeviceToDevice, s), "copy");
            }
        };

        hip_check(launch_permute_in(plan->d, (const double2 *)b_dev, ld, bt, nr, s), "permute");
        hip_check(launch_fill_zero(xt, (int64_t)N * nr, s), "zero");
        std::vector<double> bnorm, beta;
        norms(bt, bnorm);
        for (int c = 0; c < nr; ++c)
            if (bnorm[c] == 0) bnorm[c] = 1.0;
        hip_check(hipMemcpyAsync(r, bt, vec, hipMemcpyDeviceToDevice, s), "copy");
        int iters = 0;
        std::vector<int> coliters(nr, 0);
        double worst = 0;
        for (;;) {
            norms(r, beta);
            worst = 0;
            bool all = true;
            for (int c = 0; c < nr; ++c) {
                double rel = beta[c] / bnorm[c];
                worst = std::max(worst, rel);
                act[c] = rel > tol ? 1 : 0;
                if (act[c]) all = false;
                if (!std::isfinite(rel)) throw BuildError{FDA_EBREAKDOWN, "non-finite residual"};
            }
            if (all) break;
            if (iters >= maxit) {
                rc = FDA_NOTCONV;
                break;
            }
            if (iters == 0) judge_res0 = worst;
            hip_check(hipMemcpyAsync(act_d, act.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, s), "h2d");
            // V_0 = r / beta
            std::vector<cplx> scl(nr);
            for (int c = 0; c < nr; ++c) scl[c] = beta[c] > 0 ? 1.0 / beta[c] : 0.0;
            hip_check(hipMemcpyAsync(sc, scl.data(), sizeof(double2) * nr, hipMemcpyHostToDevice, s), "h2d");
            hip_check(launch_scale_cols(r, sc, V, N, nr, s), "scale");
            std::vector<std::vector<cplx>> H(nr, std::vector<cplx>((size_t)(m + 1) * m, 0.0));
            std::vector<std::vector<cplx>> cs(nr, std::vector<cplx>(m)), sn(nr, std::vector<cplx>(m));
            std::vector<std::vector<cplx>> g(nr, std::vector<cplx>(m + 1, 0.0));
            for (int c = 0; c < nr; ++c) g[c][0] = beta[c];
            int jdone = 0;
            std::vector<char> done(nr, 0);
            std::vector<int> jcnt(nr, 0);
            for (int j = 0; j < m; ++j) {
                double2 *zj = Zs + (size_t)j * N * nr;
                apply_M(V + (size_t)j * N * nr, zj);
                apply_A(zj, w);
                ++iters;
                // classical Gram-Schmidt, twice, and the normalisation, all on
                // the device; the host reads the step's inner products once
                dots_async(V, j + 1, w, hpin[0]);
                hip_check(launch_multi_axpy(V, j + 1, nr, hd, -1.0, w, N, nullptr, s), "cgs");
                dots_async(V, j + 1, w, hpin[1]);
                hip_check(launch_multi_axpy(V, j + 1, nr, hd, -1.0, w, N, nullptr, s), "cgs");
                dots_async(w, 1, w, hpin[2]);
                hip_check(launch_inv_norm(hd, sc, nr, s), "norm");
                hip_check(launch_scale_cols(w, sc, V + (size_t)(j + 1) * N * nr, N, nr, s), "scale");
                hip_check(hipStreamSynchronize(s), "sync");
                const double2 *h1 = hpin[0], *h2v = hpin[1];
                std::vector<double> hn(nr);
                for (int c = 0; c < nr; ++c) hn[c] = std::sqrt(std::max(0.0, hpin[2][c].x));
                bool all_ok = true;
                for (int c = 0; c < nr; ++c) {
                    if (!act[c] || done[c]) continue;
                    coliters[c]++;
                    jcnt[c] = j + 1;
                    auto &Hc = H[c];
                    for (int i = 0; i <= j; ++i) {
                        const double2 a1 = h1[(size_t)c * (j + 1) + i], a2 = h2v[(size_t)c * (j + 1) + i];
                        Hc[i + (size_t)j * (m + 1)] = cplx(a1.x, a1.y) + cplx(a2.x, a2.y);
                    }
                    Hc[j + 1 + (size_t)j * (m + 1)] = hn[c];
                    for (int i = 0; i < j; ++i) {
                        cplx a = Hc[i + (size_t)j * (m + 1)], b = Hc[i + 1 + (size_t)j * (m + 1)];
                        Hc[i + (size_t)j * (m + 1)] = std::conj(cs[c][i]) * a + std::conj(sn[c][i]) * b;
                        Hc[i + 1 + (size_t)j * (m + 1)] = -sn[c][i] * a + cs[c][i] * b;
                    }
                    cplx a = Hc[j + (size_t)j * (m + 1)], b = Hc[j + 1 + (size_t)j * (m + 1)];
                    double den = std::sqrt(std::norm(a) + std::norm(b));
                    if (!std::isfinite(den)) throw BuildError{FDA_EBREAKDOWN, "non-finite Arnoldi value"};
                    cs[c][j] = den > 0 ? a / den : cplx(1.0);
                    sn[c][j] = den > 0 ? b / den : cplx(0.0);
                    Hc[j + (size_t)j * (m + 1)] = den;
                    Hc[j + 1 + (size_t)j * (m + 1)] = 0.0;
                    g[c][j + 1] = -sn[c][j] * g[c][j];
                    g[c][j] = std::conj(cs[c][j]) * g[c][j];
                    if (std::abs(g[c][j + 1]) / bnorm[c] <= tol || hn[c] == 0.0) done[c] = 1;
                    if (!done[c]) all_ok = false;
                }
                jdone = j + 1;
                if (judge_state >= 0 && judge_state < 2) {
                    double res = 0;  // worst Givens residual estimate of the active columns
                    for (int c = 0; c < nr; ++c)
                        if (act[c]) res = std::max(res, std::abs(g[c][jcnt[c]]) / bnorm[c]);
                    if (++judge_steps == kJudge) {
                        const double rate = judge_res0 > 0 ? res / judge_res0 : 0.0;
                        if (judge_state == 0) {
                            judge_rate_bj = rate;
                            cur_pc = FDA_PRECOND_MLP;
                            judge_state = 1;
                        } else {
                            if (rate > judge_rate_bj) {
                                cur_pc = FDA_PRECOND_BLOCK_JACOBI;
                                st.mlp_rejected = 1;
                            }
                            judge_state = 2;
                        }
                        judge_res0 = res;
                        judge_steps = 0;
                    }
                }
                if (all_ok || iters >= maxit) break;
            }
            // y = H^-1 g per column, then x += Z y (flexible GMRES: Z_j = M(V_j))
            std::vector<cplx> Y((size_t)(m + 1) * nr, 0.0);
            for (int c = 0; c < nr; ++c) {
                if (!act[c]) continue;
                int jj = jcnt[c];
                auto &Hc = H[c];
                for (int i = jj - 1; i >= 0; --i) {
                    cplx sum = g[c][i];
                    for (int q = i + 1; q < jj; ++q) sum -= Hc[i + (size_t)q * (m + 1)] * Y[(size_t)c * jdone + q];
                    Y[(size_t)c * jdone + i] = sum / Hc[i + (size_t)i * (m + 1)];
                }
            }
            hip_check(hipMemcpyAsync(h2, Y.data(), sizeof(double2) * (size_t)jdone * nr, hipMemcpyHostToDevice, s), "h2d");
            // x += Z y (Y is zero for inactive columns)
            hip_check(launch_multi_axpy(Zs, jdone, nr, h2, 1.0, xt, N, nullptr, s), "x update");
            // true residual r = b - A x
            apply_A(xt, w);
            hip_check(launch_sub(bt, w, r, (int64_t)N * nr, s), "residual");
            st.restarts++;
        }
        hip_check(launch_permute_out(plan->d, xt, (double2 *)x_dev, ld, nr, s), "permute");
        hip_check(hipStreamSynchronize(s), "sync");
        st.iterations = iters;
        st.rel_residual = worst;
        for (int c = 0; c < nr && c < 64; ++c) st.col_iterations[c] = coliters[c];
    } catch (const BuildError &e) {
        rc = fail(e.code, e.msg);
    } catch (const HipError &e) {
        rc = fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const MlpError &e) {
        rc = fail(FDA_EHIP, e.msg);
    }
    hipStreamSynchronize(s);
    for (void *q : tmp) hipFree(q);
    for (void *q : pinned) hipHostFree(q);
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stp) *stp = st;
    if (rc == FDA_NOTCONV) g_last_error = "GMRES reached maxit before the tolerance";
    return rc;
}


// ------------------------------------------------------------ learned preconditioner

#define MLP_GUARD(body)                                                      \
    try {                                                                    \
        body                                                                 \
    } catch (const MlpError &e) {                                            \
        return fail(FDA_EHIP, e.msg);                                        \
    } catch (const HipError &e) {                                            \
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e)); \
    } catch (const BuildError &e) {                                          \
        return fail(e.code, e.msg);                                          \
    } catch (const std::bad_alloc &) {                                       \
        return fail(FDA_ENOMEM, "host allocation failed");                   \
    }

int fda_mlp_create(int32_t hidden, uint64_t seed, int32_t device, fda_mlp **out) {
    g_last_error.clear();
    if (!out) return fail(FDA_EINVAL, "NULL argument");
    *out = nullptr;
    if (hidden < 1 || hidden > 4096) return fail(FDA_EINVAL, "hidden width must be in [1, 4096]");
    MLP_GUARD({
        hip_check(hipSetDevice(device), "hipSetDevice");
        fda_mlp *h = new fda_mlp();
        h->device = device;
        try {
            h->m = mlp_create(hidden, seed);
        } catch (...) {
            delete h;
            throw;
        }
        hip_check(hipDeviceSynchronize(), "sync");
        *out = h;
    })
    return FDA_OK;
}

void fda_mlp_free(fda_mlp *mlp) {
    if (!mlp) return;
    hipSetDevice(mlp->device);
    hipDeviceSynchronize();
    mlp_free(mlp->m);
    delete mlp;
}

int64_t fda_mlp_num_params(const fda_mlp *mlp) { return mlp && mlp->m ? (int64_t)mlp->m->nparam : -1; }

int32_t fda_mlp_hidden(const fda_mlp *mlp) { return mlp && mlp->m ? mlp->m->hidden : -1; }

int fda_mlp_get_params(const fda_mlp *mlp, float *params, int64_t n) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !params) return fail(FDA_EINVAL, "NULL argument");
    if (n != (int64_t)mlp->m->nparam) return fail(FDA_EINVAL, "parameter count mismatch");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(params, mlp->m->w, sizeof(float) * n, hipMemcpyDeviceToHost), "d2h");
    })
    return FDA_OK;
}

int fda_mlp_set_params(fda_mlp *mlp, const float *params, int64_t n) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !params) return fail(FDA_EINVAL, "NULL argument");
    if (n != (int64_t)mlp->m->nparam) return fail(FDA_EINVAL, "parameter count mismatch");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return fail(FDA_EINVAL, "non-finite parameter");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(mlp->m->w, params, sizeof(float) * n, hipMemcpyHostToDevice), "h2d");
        mlp->m->sync_bf16(nullptr);
        hip_check(hipDeviceSynchronize(), "sync");
    })
    return FDA_OK;
}

int fda_mlp_forward(fda_mlp *mlp, const float *X_dev, int64_t rows, float *Y_dev, void *stream) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !X_dev || !Y_dev) return fail(FDA_EINVAL, "NULL argument");
    if (rows < 1 || rows > (int64_t)1 << 30) return fail(FDA_EINVAL, "rows out of range");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        hip_check(hipStreamSynchronize(as_stream(stream)), "sync");
        mlp->m->forward(X_dev, rows, Y_dev, as_stream(stream));
        hip_check(hipGetLastError(), "forward");
    })
    return FDA_OK;
}

int fda_mlp_forward_noalloc(fda_mlp *mlp, const float *X_dev, int64_t rows, float *Y_dev, void *stream) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !X_dev || !Y_dev) return fail(FDA_EINVAL, "NULL argument");
    const int64_t cap = mlp_noalloc_max_rows(mlp->m->hidden);
    if (rows < 1 || rows > cap)
        return fail(FDA_EINVAL, "rows must be in [1, " + std::to_string(cap) +
                                    "]: the static scratch holds 2 x rows x hidden <= " +
                                    std::to_string(kMlpNoAllocFloats) + " floats");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        mlp->m->forward_noalloc(X_dev, rows, Y_dev, mlp->device, as_stream(stream));
        hip_check(hipGetLastError(), "forward");
    })
    return FDA_OK;
}

int fda_mlp_gradient(fda_mlp *mlp, const float *X_dev, const float *T_dev, const float *M_dev, int64_t rows,
                     float *grad_dev, double *loss, void *stream) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !X_dev || !T_dev || !M_dev || !grad_dev) return fail(FDA_EINVAL, "NULL argument");
    if (rows < 1 || rows > (int64_t)1 << 24) return fail(FDA_EINVAL, "rows out of range");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        hipStream_t s = as_stream(stream);
        hip_check(hipStreamSynchronize(s), "sync");
        const double sse = mlp_gradient(mlp->m, X_dev, T_dev, M_dev, rows, grad_dev, s);
        if (loss) *loss = sse / ((double)rows * kMlpOut);
    })
    return FDA_OK;
}

int fda_mlp_train(fda_mlp *mlp, const float *X_dev, const float *T_dev, const float *M_dev, int64_t rows,
                  int32_t epochs, int32_t batch, float lr, uint64_t seed, double *losses, void *stream) {
    g_last_error.clear();
    if (!mlp || !mlp->m || !X_dev || !T_dev || !M_dev) return fail(FDA_EINVAL, "NULL argument");
    if (rows < 1 || rows > ((int64_t)1 << 31) - 1) return fail(FDA_EINVAL, "rows out of range");
    if (epochs < 1 || batch < 1 || batch > (1 << 16) || !(lr > 0) || !std::isfinite(lr))
        return fail(FDA_EINVAL, "bad epochs / batch / lr");
    MLP_GUARD({
        hip_check(hipSetDevice(mlp->device), "hipSetDevice");
        hipStream_t s = as_stream(stream);
        hip_check(hipStreamSynchronize(s), "sync");
        std::vector<double> l = mlp_train(mlp->m, X_dev, T_dev, M_dev, rows, epochs, batch, lr, seed, s);
        if (losses) std::copy(l.begin(), l.end(), losses);
        for (double v : l)
            if (!std::isfinite(v)) return fail(FDA_EBREAKDOWN, "training loss is not finite");
    })
    return FDA_OK;
}

int fda_mlp_samples(fda_plan *plan, const void *r_dev, const void *e_dev, int64_t nrhs, int64_t ld, float *X_dev,
                    float *T_dev, float *M_dev, void *stream) {
    g_last_error.clear();
    if (!plan || !r_dev || !X_dev) return fail(FDA_EINVAL, "NULL argument");
    if ((e_dev == nullptr) != (T_dev == nullptr) || (T_dev == nullptr) != (M_dev == nullptr))
        return fail(FDA_EINVAL, "e_dev, T_dev and M_dev are given together");
    if (nrhs < 1 || nrhs > plan->hp.opt.nrhs_max || ld < plan->d.n) return fail(FDA_EINVAL, "nrhs / ld out of range");
    double2 *vnorm = nullptr;  // row scales
    double2 *z = nullptr;
    int rc = FDA_OK;
    try {
        hip_check(hipSetDevice(plan->device), "hipSetDevice");
        ensure_capacity(plan, (int)nrhs);
        hipStream_t s = as_stream(stream);
        const int64_t N = plan->d.n, nl = plan->d.mlp_nrows;
        hip_check(hipMalloc(&vnorm, sizeof(double2) * nl), "alloc");
        hip_check(hipMalloc(&z, sizeof(double2) * N), "alloc");
        hip_check(launch_permute_in(plan->d, (const double2 *)r_dev, ld, plan->xt, (int)nrhs, s), "permute");
        if (e_dev)
            hip_check(launch_permute_in(plan->d, (const double2 *)e_dev, ld, plan->yt, (int)nrhs, s), "permute");
        for (int64_t c = 0; c < nrhs; ++c) {
            mlp_features(plan->d, plan->xt + c * N, plan->d.leaf_scalars, X_dev + c * nl * kMlpIn, vnorm, z, s);
            if (e_dev)
                mlp_targets(plan->d, plan->yt + c * N, z, vnorm, T_dev + c * nl * kMlpOut, M_dev + c * nl * kMlpOut,
                            s);
        }
        hip_check(hipGetLastError(), "features");
        hip_check(hipStreamSynchronize(s), "sync");
    } catch (const HipError &e) {
        rc = fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const BuildError &e) {
        rc = fail(e.code, e.msg);
    }
    if (rc != FDA_OK) hipStreamSynchronize(as_stream(stream));
    hipFree(vnorm);
    hipFree(z);
    return rc;
}

int fda_plan_leaves(const fda_plan *plan, int32_t *perm, int64_t n, int64_t *leaf_off, int64_t nleaf) {
    g_last_error.clear();
    if (!plan) return fail(FDA_EINVAL, "NULL plan");
    const HostPlan &hp = plan->hp;
    if (perm) {
        if (n != (int64_t)hp.perm.size()) return fail(FDA_EINVAL, "perm length must be N");
        std::copy(hp.perm.begin(), hp.perm.end(), perm);
    }
    if (leaf_off) {
        if (nleaf + 1 != (int64_t)hp.leaf_off.size()) return fail(FDA_EINVAL, "leaf_off length must be nleaf + 1");
        std::copy(hp.leaf_off.begin(), hp.leaf_off.end(), leaf_off);
    }
    return FDA_OK;
}

int fda_plan_set_mlp(fda_plan *plan, fda_mlp *mlp) {
    g_last_error.clear();
    if (!plan) return fail(FDA_EINVAL, "NULL plan");
    if (mlp && mlp->device != plan->device) return fail(FDA_EINVAL, "network and plan are on different devices");
    plan->mlp = mlp;
    return FDA_OK;
}


// ------------------------------------------------------------ many meshes in one graph

struct fda_batch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<fda_plan *> plans;  // each holds one count in live_batches while the batch exists
    int device = 0;
    int nplans = 0;
};

static void batch_release(fda_batch *b) {
    if (!b) return;
    for (fda_plan *p : b->plans) --p->live_batches;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (auto e : b->events) hipEventDestroy(e);
    for (auto s : b->streams) hipStreamDestroy(s);
    delete b;
}

int fda_batch_create(fda_plan *const *plans, int32_t nplans, const void *const *x_devs, void *const *y_devs,
                     const int64_t *nrhs, fda_batch **out) {
    g_last_error.clear();
    if (!out) return fail(FDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || !x_devs || !y_devs || !nrhs || nplans < 1 || nplans > 4096)
        return fail(FDA_EINVAL, "bad plans / buffers / nplans");
    const int dev = plans[0] ? plans[0]->device : 0;
    for (int i = 0; i < nplans; ++i) {
        if (!plans[i] || !x_devs[i] || !y_devs[i]) return fail(FDA_EINVAL, "NULL plan or buffer");
        if (plans[i]->device != dev) return fail(FDA_EINVAL, "plans on different devices");
        if (nrhs[i] < 1 || nrhs[i] > plans[i]->hp.opt.nrhs_max) return fail(FDA_EINVAL, "nrhs out of range");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(FDA_EINVAL, "a plan appears twice (its work buffers are shared)");
    }
    fda_batch *b = new fda_batch();
    b->device = dev;
    b->nplans = nplans;
    hipStream_t s0 = nullptr;
    bool capturing = false;
    try {
        hip_check(hipSetDevice(dev), "hipSetDevice");
        // work buffers are allocated before capture (nothing allocates inside the graph)
        for (int i = 0; i < nplans; ++i) ensure_capacity(plans[i], (int)nrhs[i]);
        hip_check(hipDeviceSynchronize(), "sync");
        const int nstream = std::min(nplans, 16);
        b->streams.resize(nstream + 1, nullptr);
        for (auto &s : b->streams) hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
        b->events.resize(nstream + 1, nullptr);
        for (auto &e : b->events) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        s0 = b->streams[0];
        hip_check(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "begin capture");
        capturing = true;
        hip_check(hipEventRecord(b->events[0], s0), "fork");
        for (int q = 1; q <= nstream; ++q) hip_check(hipStreamWaitEvent(b->streams[q], b->events[0], 0), "fork wait");
        // plans go round-robin to the branch streams; each branch runs its
        // plans one after another, the branches run concurrently
        for (int i = 0; i < nplans; ++i) {
            fda_plan *p = plans[i];
            hipStream_t st = b->streams[1 + i % nstream];
            const int nr = (int)nrhs[i];
            hip_check(launch_permute_in(p->d, (const double2 *)x_devs[i], p->d.n, p->xt, nr, st), "permute");
            hip_check(launch_matvec_tree(p->d, p->xt, p->yt, nr, st, nullptr, nullptr), "matvec");
            hip_check(launch_permute_out(p->d, p->yt, (double2 *)y_devs[i], p->d.n, nr, st), "permute");
        }
        for (int q = 1; q <= nstream; ++q) {
            hip_check(hipEventRecord(b->events[q], b->streams[q]), "join");
            hip_check(hipStreamWaitEvent(s0, b->events[q], 0), "join wait");
        }
        capturing = false;
        hip_check(hipStreamEndCapture(s0, &b->graph), "end capture");
        hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate");
        for (int i = 0; i < nplans; ++i) {
            b->plans.push_back(plans[i]);
            ++plans[i]->live_batches;
        }
    } catch (const BuildError &e) {
        if (capturing) {
            hipGraph_t g = nullptr;
            hipStreamEndCapture(s0, &g);
            if (g) hipGraphDestroy(g);
        }
        batch_release(b);
        return fail(e.code, e.msg);
    } catch (const HipError &e) {
        if (capturing) {
            hipGraph_t g = nullptr;
            hipStreamEndCapture(s0, &g);
            if (g) hipGraphDestroy(g);
        }
        batch_release(b);
        return fail(FDA_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
    }
    *out = b;
    return FDA_OK;
}

int fda_batch_launch(fda_batch *batch, void *stream) {
    g_last_error.clear();
    if (!batch || !batch->exec) return fail(FDA_EINVAL, "NULL batch");
    hipError_t e = hipSetDevice(batch->device);
    if (e == hipSuccess) e = hipGraphLaunch(batch->exec, as_stream(stream));
    if (e != hipSuccess) return fail(FDA_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
    return FDA_OK;
}

void fda_batch_free(fda_batch *batch) {
    if (!batch) return;
    hipSetDevice(batch->device);
    hipDeviceSynchronize();
    batch_release(batch);
}

}  // extern "C"
