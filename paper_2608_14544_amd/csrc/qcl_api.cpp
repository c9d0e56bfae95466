// Host side of the C ABI declared in qcl.h: validation, model set-up,
// ensemble layout and kernel dispatch.  No device memory is allocated
// outside qcl_create_model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "qcl_internal.hpp"

namespace {

thread_local std::string g_last_error;

qcl_status fail(qcl_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

qcl_status device_fail(hipError_t e, const char *what)
{
    return fail(QCL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite_all(const double *x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i]))
            return false;
    return true;
}

bool symmetric(const double *a, int n)
{
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i)
        scale = std::max(scale, std::fabs(a[i]));
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (std::fabs(a[i * n + j] - a[j * n + i]) > 1e-12 * std::max(scale, 1e-300))
                return false;
    return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned256(const void *p) { return ((uintptr_t)p & 255) == 0; }

size_t real_size(int32_t prec) { return prec == QCL_FP64 ? sizeof(double) : sizeof(float); }

int64_t leading_dim(int64_t n_traj) { return std::max<int64_t>(64, (n_traj + 63) / 64 * 64); }

// Orthonormal basis of the span of the M coupling rows K_j (each the T
// upper-triangle slots of K_j) by pivoted Gram-Schmidt with
// re-orthogonalisation; coef[j][r] = <K_j, B_r>.  Directions whose residual
// falls below 1e-13 of the largest row are dropped, so sum_r coef B_r
// reproduces every K_j to that relative accuracy.  Returns the rank.
int factor_couplings(int M, int T, const std::vector<double> &kmat, std::vector<double> &basis,
                     std::vector<double> &coef)
{
    auto dot = [T](const double *x, const double *y) {
        double s = 0.0;
        for (int i = 0; i < T; ++i)
            s += x[i] * y[i];
        return s;
    };
    std::vector<double> res(kmat);
    double kmax = 0.0;
    for (int j = 0; j < M; ++j)
        kmax = std::max(kmax, std::sqrt(dot(&kmat[(size_t)j * T], &kmat[(size_t)j * T])));
    basis.clear();
    int rank = 0;
    while (rank < T && kmax > 0.0) {
        int best = -1;
        double bn = 0.0;
        for (int j = 0; j < M; ++j) {
            const double nj = std::sqrt(dot(&res[(size_t)j * T], &res[(size_t)j * T]));
            if (nj > bn) {
                bn = nj;
                best = j;
            }
        }
        if (best < 0 || bn <= 1e-13 * kmax)
            break;
        std::vector<double> b(res.begin() + (size_t)best * T, res.begin() + (size_t)(best + 1) * T);
        for (int pass = 0; pass < 2; ++pass) {
            for (int r = 0; r < rank; ++r) {
                const double pr = dot(b.data(), &basis[(size_t)r * T]);
                for (int i = 0; i < T; ++i)
                    b[i] -= pr * basis[(size_t)r * T + i];
            }
            const double nb = std::sqrt(dot(b.data(), b.data()));
            for (int i = 0; i < T; ++i)
                b[i] /= nb;
        }
        basis.insert(basis.end(), b.begin(), b.end());
        ++rank;
        for (int j = 0; j < M; ++j)
            for (int pass = 0; pass < 2; ++pass) {
                const double pr = dot(&res[(size_t)j * T], b.data());
                for (int i = 0; i < T; ++i)
                    res[(size_t)j * T + i] -= pr * b[i];
            }
    }
    coef.assign((size_t)M * std::max(rank, 1), 0.0);
    for (int j = 0; j < M; ++j)
        for (int r = 0; r < rank; ++r)
            coef[(size_t)j * rank + r] = dot(&kmat[(size_t)j * T], &basis[(size_t)r * T]);
    return rank;
}

// Rows of a partials buffer: one per tile, then the scratch rows of the
// pairwise passes of the reduction (at most 1/8 + 1/64 of them); the
// per-bin excluded counts of qcl_reduce_observables follow.
int64_t partials_rows(int64_t n_traj)
{
    const int64_t t = qcl::n_tiles(n_traj);
    return t + (t + 7) / 8 + (t + 63) / 64;
}

qcl_status check_model(qcl_model m)
{
    if (!m)
        return fail(QCL_ERR_INVALID_ARG, "model is NULL");
    return QCL_OK;
}

// Kernels read the model's constant block on the device that holds it:
// the calling thread's current device must be that device.
qcl_status check_device(const qcl_model_s &m)
{
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return device_fail(e, "hipGetDevice");
    if (dev != m.device)
        return fail(QCL_ERR_INVALID_ARG, "the model lives on device %d but device %d is current", m.device, dev);
    return QCL_OK;
}

qcl_status check_ensemble(const qcl_model_s &m, const qcl_ensemble *e)
{
    if (!e)
        return fail(QCL_ERR_INVALID_ARG, "ensemble is NULL");
    if (e->prec != QCL_FP64 && e->prec != QCL_FP32_ACC64)
        return fail(QCL_ERR_INVALID_ARG, "unknown precision %d", e->prec);
    if (e->n_traj < 0)
        return fail(QCL_ERR_INVALID_ARG, "n_traj < 0");
    if (e->n_traj > ((int64_t)1 << 40))
        return fail(QCL_ERR_INVALID_ARG, "n_traj too large");
    if (e->ld < e->n_traj || e->ld % 64 != 0)
        return fail(QCL_ERR_INVALID_ARG, "ld must be >= n_traj and a multiple of 64");
    if (e->traj_offset < 0 || e->step < 0)
        return fail(QCL_ERR_INVALID_ARG, "traj_offset and step must be >= 0");
    if (e->n_traj > 0) {
        if (!e->q || !e->p || !e->u || !e->w || !e->phase || !e->a || !e->b)
            return fail(QCL_ERR_INVALID_ARG, "ensemble array pointer is NULL");
        if (!aligned256(e->q) || !aligned256(e->p) || !aligned256(e->u) || !aligned256(e->w) ||
            !aligned256(e->phase) || !aligned256(e->a) || !aligned256(e->b) || !aligned256(e->flags))
            return fail(QCL_ERR_INVALID_ARG, "ensemble arrays must be 256-byte aligned");
    }
    if (m.source && e->prec != QCL_FP64 && !m.user_propagate32)
        return fail(QCL_ERR_UNSUPPORTED,
                    "this supplied potential runs binary64 ensembles only (its source defines no binary32 "
                    "functions and no QCL_SOURCE_FP32)");
    return QCL_OK;
}

qcl_status check_propagate(qcl_model m, const qcl_ensemble *ens, const qcl_prop_desc *pd, const double *partials)
{
    if (qcl_status st = check_model(m))
        return st;
    if (qcl_status st = check_ensemble(*m, ens))
        return st;
    if (!pd)
        return fail(QCL_ERR_INVALID_ARG, "prop is NULL");
    if (!(pd->dt > 0.0) || !std::isfinite(pd->dt))
        return fail(QCL_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (pd->n_steps < 0 || pd->cadence < 1 || pd->n_out < 1)
        return fail(QCL_ERR_INVALID_ARG, "n_steps >= 0, cadence >= 1 and n_out >= 1 required");
    if (pd->scheme != QCL_TRANS_NORMALIZED && pd->scheme != QCL_TRANS_LINEAR)
        return fail(QCL_ERR_INVALID_ARG, "unknown transition scheme %d", pd->scheme);
    if (pd->occupancy != 0 && pd->occupancy != 2 && pd->occupancy != 3)
        return fail(QCL_ERR_INVALID_ARG, "occupancy must be 0, 2 or 3");
    if (pd->workgroups_per_cu < 0 || pd->workgroups_per_cu > 32)
        return fail(QCL_ERR_INVALID_ARG, "workgroups_per_cu must be in [0, 32]");
    const int64_t last_bin = (ens->step + pd->n_steps) / pd->cadence;
    if (last_bin >= pd->n_out)
        return fail(QCL_ERR_INVALID_ARG, "bin %lld would be written but n_out is %d", (long long)last_bin,
                    pd->n_out);
    if (ens->step + (int64_t)pd->n_steps > ((int64_t)1 << 33))
        return fail(QCL_ERR_INVALID_ARG, "global step counter out of range");
    if (ens->n_traj > 0 && (!partials || !aligned256(partials)))
        return fail(QCL_ERR_INVALID_ARG, "partials is NULL or not 256-byte aligned");
    if (ens->n_traj > 0 && pd->n_steps > 0)
        return check_device(*m);
    return QCL_OK;
}

qcl_status check_reduce(qcl_model m, const double *partials, int64_t n_traj, int32_t n_out, const double *out)
{
    if (qcl_status st = check_model(m))
        return st;
    if (n_traj < 1)
        return fail(QCL_ERR_INVALID_ARG, "n_traj must be >= 1 to average");
    if (n_out < 1)
        return fail(QCL_ERR_INVALID_ARG, "n_out must be >= 1");
    if (!partials || !out || !aligned256(partials) || !aligned256(out))
        return fail(QCL_ERR_INVALID_ARG, "partials/out NULL or not 256-byte aligned");
    return QCL_OK;
}

// Items of one batch that share a kernel: same specialisation (two-state
// closed form with M modes, or general N states with modes padded to MP),
// precision and transition rule.
struct BatchClass {
    bool fast2;
    int n, modes, prec, scheme, occ, wpc;
    const qcl_model_s *src;      // the model, for a supplied potential (its own program); else null
    std::vector<int32_t> order;  // item indices, most expensive tile first
    size_t item_bytes = 0;
    size_t counter_offset = 0;   // one 8-byte tile counter
    size_t offset = 0;           // descriptor array
    int64_t total_tiles = 0;
    double cost = 0;             // estimated walker-steps x per-step weight
};

struct BatchPlan {
    std::vector<BatchClass> classes;
    size_t bytes = 0;
};

// Side streams for running the classes of one batched call concurrently:
// forked from the caller's stream by an event and joined back into it, so
// the call stays ordered on the caller's stream.  Created on a device's
// first multi-class call (default priority) and kept until the process
// ends; the mutex keeps the fork/join sequences of concurrent host threads
// apart.  HIP spreads a process's streams over a few hardware queues (four
// by default) in turn, and the caller's stream holds one of them: with
// three side streams each has a queue of its own (a fourth shared one with
// the third, and the classes on those two ran one after the other).
constexpr int kSideStreams = 3;
struct Fan {
    bool ready = false;
    hipStream_t s[kSideStreams];
    hipEvent_t fork;
    hipEvent_t join[kSideStreams];
};
std::mutex g_fan_mutex;
std::vector<Fan> g_fans;

hipError_t device_fan(Fan *&out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if ((int)g_fans.size() <= dev)
        g_fans.resize(dev + 1);
    Fan &f = g_fans[dev];
    if (!f.ready) {
        for (int k = 0; k < kSideStreams; ++k)
            if ((e = hipStreamCreateWithFlags(&f.s[k], hipStreamNonBlocking)) != hipSuccess)
                return e;
        if ((e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming)) != hipSuccess)
            return e;
        for (int k = 0; k < kSideStreams; ++k)
            if ((e = hipEventCreateWithFlags(&f.join[k], hipEventDisableTiming)) != hipSuccess)
                return e;
        f.ready = true;
    }
    out = &f;
    return hipSuccess;
}

qcl_status plan_batch(const qcl_batch_item *items, int32_t n_items, BatchPlan &plan)
{
    if (n_items < 0 || (n_items > 0 && !items))
        return fail(QCL_ERR_INVALID_ARG, "items is NULL or n_items < 0");
    if (n_items > (1 << 20))
        return fail(QCL_ERR_INVALID_ARG, "at most 2^20 items per batch");
    std::vector<double> weight(n_items, 0.0);
    for (int32_t i = 0; i < n_items; ++i) {
        const qcl_batch_item &it = items[i];
        if (qcl_status st = check_propagate(it.model, it.ens, &it.prop, it.partials))
            return fail(st, "item %d: %s", i, g_last_error.c_str());
        if (it.ens->n_traj == 0 || it.prop.n_steps == 0)
            continue;
        const qcl_model_s &m = *it.model;
        // general kernels are specialised on padded modes and rank bucket;
        // a model with a supplied potential is a class of its own (its program)
        const int poly = m.degree > 1 ? 1 : 0;
        const int modes = m.fast2 ? m.m + 16 * poly
                                  : qcl::padded_modes(m.m) * 64 + m.rank_pad + 32 * poly + 16 * (m.n_pairs > 0) +
                                        8 * (m.n_pairs > 0 && qcl::sq_pad(m.n_sq) == 8) +
                                        4 * (m.n_pairs > 0 && qcl::sq_pad(m.n_sq) == qcl::kSq);
        BatchClass *c = nullptr;
        const int occ = qcl::occupancy_variant(m, it.ens->prec, it.prop.occupancy);
        const qcl_model_s *src = m.source ? &m : nullptr;
        for (BatchClass &k : plan.classes)
            if (k.fast2 == m.fast2 && k.n == m.n && k.modes == modes && k.prec == it.ens->prec &&
                k.scheme == it.prop.scheme && k.occ == occ && k.wpc == it.prop.workgroups_per_cu && k.src == src)
                c = &k;
        if (!c) {
            plan.classes.push_back(
                BatchClass{m.fast2, m.n, modes, it.ens->prec, it.prop.scheme, occ, it.prop.workgroups_per_cu, src});
            c = &plan.classes.back();
            c->item_bytes = qcl::batch_item(m, *it.ens, it.prop, nullptr, 0, nullptr);
            if (c->item_bytes == 0)
                return fail(QCL_ERR_UNSUPPORTED, "item %d: no batched kernel for this model", i);
        }
        c->order.push_back(i);
        // per-step work in vector instructions, from the compiled kernels:
        // about 10 per padded mode (3 times that with higher powers) plus
        // the electronic part (solve, transition, forces), about 300, 700
        // and 1250 for 2, 3 and 4 states and growing as N^3 beyond; the
        // closed-form two-state kernels about 100 plus 25 per mode.  It
        // orders tiles and spreads classes over the side streams, so it
        // only needs to be roughly proportional to the time
        const double per_step =
            m.fast2 ? 100.0 + 25.0 * m.m * (m.degree > 1 ? 2 : 1)
                    : 10.0 * qcl::padded_modes(m.m) * (m.degree > 1 ? 3 : 1) +
                          (m.n <= 2 ? 300.0 : m.n == 3 ? 700.0 : 1250.0 * (m.n * m.n * m.n) / 64.0);
        weight[i] = per_step * it.prop.n_steps;
        const int64_t t = qcl::n_tiles(it.ens->n_traj);
        c->total_tiles += t;
        c->cost += weight[i] * (double)it.ens->n_traj;
    }
    // a walker array or partials buffer may appear in one item only
    std::vector<std::pair<const void *, int32_t>> keys;
    keys.reserve(3 * (size_t)n_items);
    for (int32_t i = 0; i < n_items; ++i) {
        keys.push_back({items[i].ens, i});
        if (items[i].ens->n_traj > 0) {
            keys.push_back({items[i].ens->q, i});
            keys.push_back({items[i].partials, i});
        }
    }
    std::sort(keys.begin(), keys.end());
    for (size_t k = 1; k < keys.size(); ++k)
        if (keys[k].first == keys[k - 1].first && keys[k].second != keys[k - 1].second)
            return fail(QCL_ERR_INVALID_ARG, "items %d and %d share an ensemble or partials buffer",
                        keys[k - 1].second, keys[k].second);
    // heaviest class first, heaviest tile first inside a class
    std::stable_sort(plan.classes.begin(), plan.classes.end(),
                     [](const BatchClass &x, const BatchClass &y) { return x.cost > y.cost; });
    size_t off = 0;
    for (BatchClass &c : plan.classes) {
        std::stable_sort(c.order.begin(), c.order.end(), [&](int32_t x, int32_t y) { return weight[x] > weight[y]; });
        c.counter_offset = off;
        c.offset = off + 256;
        off = align256(c.offset + c.item_bytes * c.order.size());
    }
    plan.bytes = off;
    return QCL_OK;
}

// Eigendecomposition A = V diag(e) V^T of a symmetric n x n matrix (row
// major) by cyclic Jacobi rotations in binary64, until every off-diagonal
// entry is below 1e-15 of the norm; eigenvectors in the columns of V.
void jacobi_sym(int n, std::vector<double> A, std::vector<double> &e, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        V[(size_t)i * n + i] = 1.0;
    double norm = 0.0;
    for (double x : A)
        norm += x * x;
    norm = std::sqrt(norm);
    for (int sweep = 0; sweep < 100 && norm > 0.0; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q)
                off = std::max(off, std::fabs(A[(size_t)p * n + q]));
        if (off <= 1e-15 * norm)
            break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0)
                    continue;
                // rotation angle that zeroes A_pq (Golub and Van Loan, Sec. 8.5)
                const double theta = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A G
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- G^T A
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V G
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    e.resize(n);
    for (int i = 0; i < n; ++i)
        e[i] = A[(size_t)i * n + i];
}

// The squared mode combinations y_s = c_s . q of a model's bilinear terms,
// with slot weights lam_sr such that sum_s lam_sr y_s^2 / 2 equals the
// terms' part of slot r, sum_p q_i q_j B_p[r].  Two factorisations:
//  - per term, ((q_i + q_j)^2 - (q_i - q_j)^2) / 4: two combinations with
//    coefficients +-1 and weights +-B_p / 2, exact in binary64;
//  - per slot r, the eigendecomposition of the M x M matrix C^r with
//    C^r_ij = C^r_ji = the sum of B_p[r] over the terms on (i, j): one
//    combination per eigenvalue above 1e-13 of the largest, weighted only
//    in its own slot (exact to rounding).
// The one with fewer combinations is kept; returns their number.
int bilinear_squares(int n, int M, int P, const int32_t *pairs, const double *b, std::vector<double> &c,
                     std::vector<double> &lam)
{
    const int T = n * (n + 1) / 2;
    auto slot_value = [&](int p, int r) {
        for (int a = 0, s = 0; a < n; ++a)
            for (int bb = a; bb < n; ++bb, ++s)
                if (s == r)
                    return b[(size_t)p * n * n + a * n + bb];
        return 0.0;
    };
    // the slot matrices and their eigen-combinations
    std::vector<double> ec, el;
    int n_eig = 0;
    double emax = 0.0;
    std::vector<std::vector<double>> evals(T), evecs(T);
    for (int r = 0; r < T; ++r) {
        std::vector<double> C((size_t)M * M, 0.0);
        for (int p = 0; p < P; ++p) {
            const int i = pairs[2 * p], j = pairs[2 * p + 1];
            const double v = slot_value(p, r);
            C[(size_t)i * M + j] += v;
            C[(size_t)j * M + i] += v;
        }
        jacobi_sym(M, C, evals[r], evecs[r]);
        for (double x : evals[r])
            emax = std::max(emax, std::fabs(x));
    }
    for (int r = 0; r < T; ++r)
        for (int k = 0; k < M; ++k)
            if (std::fabs(evals[r][k]) > 1e-13 * emax) {
                ++n_eig;
                for (int j = 0; j < M; ++j)
                    ec.push_back(evecs[r][(size_t)j * M + k]);
                for (int rr = 0; rr < T; ++rr)
                    el.push_back(rr == r ? evals[r][k] : 0.0);
            }
    if (n_eig < 2 * P) {
        c.swap(ec);
        lam.swap(el);
        return n_eig;
    }
    c.assign((size_t)2 * P * M, 0.0);
    lam.assign((size_t)2 * P * T, 0.0);
    for (int p = 0; p < P; ++p) {
        const int i = pairs[2 * p], j = pairs[2 * p + 1];
        c[(size_t)(2 * p) * M + i] += 1.0;
        c[(size_t)(2 * p) * M + j] += 1.0;
        c[(size_t)(2 * p + 1) * M + i] += 1.0;
        c[(size_t)(2 * p + 1) * M + j] -= 1.0;
        for (int r = 0; r < T; ++r) {
            lam[(size_t)(2 * p) * T + r] = 0.5 * slot_value(p, r);
            lam[(size_t)(2 * p + 1) * T + r] = -0.5 * slot_value(p, r);
        }
    }
    return 2 * P;
}

// Builds a model (linear when poly and bil are NULL); see qcl_create_model,
// qcl_create_model_poly and qcl_create_model_bilinear.
qcl_status create_model(const qcl_model_desc *d, const qcl_poly_desc *poly, const qcl_bilinear_desc *bil,
                        qcl_model *out)
{
    if (!d || !out)
        return fail(QCL_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const int n = d->n_states, M = d->n_modes;
    if (n < 2 || n > QCL_MAX_STATES)
        return fail(QCL_ERR_INVALID_ARG, "n_states %d outside [2, %d]", n, QCL_MAX_STATES);
    if (M < 1 || M > QCL_MAX_MODES)
        return fail(QCL_ERR_INVALID_ARG, "n_modes %d outside [1, %d]", M, QCL_MAX_MODES);
    if (!d->mass || !d->omega || !d->v0 || !d->k)
        return fail(QCL_ERR_INVALID_ARG, "model array is NULL");
    if (!(d->hbar > 0.0) || !std::isfinite(d->hbar))
        return fail(QCL_ERR_INVALID_ARG, "hbar must be finite and > 0");
    if (!finite_all(d->mass, M) || !finite_all(d->omega, M) || !finite_all(d->v0, n * n) ||
        !finite_all(d->k, (int64_t)M * n * n))
        return fail(QCL_ERR_INVALID_ARG, "non-finite model parameter");
    for (int j = 0; j < M; ++j)
        if (!(d->mass[j] > 0.0) || !(d->omega[j] > 0.0))
            return fail(QCL_ERR_INVALID_ARG, "mass and omega must be > 0 (mode %d)", j);
    if (!symmetric(d->v0, n))
        return fail(QCL_ERR_INVALID_ARG, "V0 is not symmetric");
    for (int j = 0; j < M; ++j)
        if (!symmetric(d->k + (size_t)j * n * n, n))
            return fail(QCL_ERR_INVALID_ARG, "K_%d is not symmetric", j);
    // a bilinear model runs on the kernels of models with higher powers
    const int D = poly ? poly->degree : bil ? 2 : 1;
    if (n > 4 && M > QCL_MAX_MODES_MANY)
        return fail(QCL_ERR_UNSUPPORTED, "models with %d states support at most %d modes (got %d)", n,
                    QCL_MAX_MODES_MANY, M);
    if (n > 4 && poly)
        return fail(QCL_ERR_UNSUPPORTED, "higher powers need at most 4 states (got %d)", n);
    if (poly) {
        if (D < 2 || D > 4)
            return fail(QCL_ERR_INVALID_ARG, "poly degree %d outside [2, 4]", D);
        if (!poly->a)
            return fail(QCL_ERR_INVALID_ARG, "poly->a is NULL");
        if (!finite_all(poly->a, (int64_t)M * (D - 1) * n * n))
            return fail(QCL_ERR_INVALID_ARG, "non-finite higher-power coefficient");
        for (int j = 0; j < M; ++j)
            for (int k = 2; k <= D; ++k)
                if (!symmetric(poly->a + ((size_t)j * (D - 1) + (k - 2)) * n * n, n))
                    return fail(QCL_ERR_INVALID_ARG, "A_%d,%d is not symmetric", j, k);
    }
    if (bil) {
        if (bil->n_pairs < 1 || bil->n_pairs > QCL_MAX_PAIRS)
            return fail(QCL_ERR_INVALID_ARG, "n_pairs %d outside [1, %d]", bil->n_pairs, QCL_MAX_PAIRS);
        if (!bil->pairs || !bil->b)
            return fail(QCL_ERR_INVALID_ARG, "bil->pairs or bil->b is NULL");
        for (int p = 0; p < bil->n_pairs; ++p) {
            const int i = bil->pairs[2 * p], j = bil->pairs[2 * p + 1];
            if (i < 0 || j < 0 || i >= M || j >= M || i == j)
                return fail(QCL_ERR_INVALID_ARG, "bilinear term %d: modes (%d, %d) invalid", p, i, j);
        }
        if (!finite_all(bil->b, (int64_t)bil->n_pairs * n * n))
            return fail(QCL_ERR_INVALID_ARG, "non-finite bilinear coefficient");
        for (int p = 0; p < bil->n_pairs; ++p)
            if (!symmetric(bil->b + (size_t)p * n * n, n))
                return fail(QCL_ERR_INVALID_ARG, "B_%d is not symmetric", p);
        if (n > 4)
            return fail(QCL_ERR_UNSUPPORTED, "bilinear terms need at most 4 states (got %d)", n);
        if (M > QCL_MAX_MODES_BILINEAR)
            return fail(QCL_ERR_UNSUPPORTED, "bilinear models support at most %d modes (got %d)",
                        QCL_MAX_MODES_BILINEAR, M);
    }
    std::vector<double> sq_c, sq_lam;
    int n_sq = 0;
    if (bil) {
        n_sq = bilinear_squares(n, M, bil->n_pairs, bil->pairs, bil->b, sq_c, sq_lam);
        if (n_sq > qcl::kSq)
            return fail(QCL_ERR_UNSUPPORTED, "the bilinear terms need %d squared mode combinations (at most %d)", n_sq,
                        qcl::kSq);
        if (n_sq > 8 && M > 16)
            return fail(QCL_ERR_UNSUPPORTED, "bilinear terms needing more than 8 squared combinations support at most "
                        "16 modes (got %d)", M);
    }

    qcl_model_s *m = new (std::nothrow) qcl_model_s();
    if (!m)
        return fail(QCL_ERR_OUT_OF_MEMORY, "host allocation failed");
    m->n = n;
    m->m = M;
    m->hbar = d->hbar;
    m->mass.assign(d->mass, d->mass + M);
    m->omega.assign(d->omega, d->omega + M);
    m->v0.assign(d->v0, d->v0 + n * n);
    m->k.assign(d->k, d->k + (size_t)M * n * n);
    m->degree = D;
    if (poly)
        m->poly.assign(poly->a, poly->a + (size_t)M * (D - 1) * n * n);
    else if (D > 1)
        m->poly.assign((size_t)M * (D - 1) * n * n, 0.0);
    if (bil) {
        m->n_pairs = bil->n_pairs;
        m->pairs.assign(bil->pairs, bil->pairs + 2 * bil->n_pairs);
        m->bpair.assign(bil->b, bil->b + (size_t)bil->n_pairs * n * n);
        m->n_sq = n_sq;
        m->sq_c = sq_c;
        m->sq_lam = sq_lam;
    }
    m->fast2 = (n == 2 && M <= qcl::kMaxFastModes && !bil);
    // energy scale: |V0| plus each mode's coupling over its zero-point-ish length
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i)
        scale += std::fabs(m->v0[i]);
    for (int j = 0; j < M; ++j) {
        const double len = 1.0 / (m->omega[j] * std::sqrt(m->mass[j]));
        double kj = 0.0;
        for (int i = 0; i < n * n; ++i)
            kj += std::fabs(m->k[(size_t)j * n * n + i]);
        scale += kj * len;
        double lk = len;
        for (int k = 2; k <= D; ++k) {
            lk *= len;
            double ak = 0.0;
            for (int i = 0; i < n * n; ++i)
                ak += std::fabs(m->poly[((size_t)j * (D - 1) + (k - 2)) * n * n + i]);
            scale += ak * lk;
        }
    }
    for (int p = 0; p < m->n_pairs; ++p) {
        const int i = m->pairs[2 * p], j = m->pairs[2 * p + 1];
        const double li = 1.0 / (m->omega[i] * std::sqrt(m->mass[i])), lj = 1.0 / (m->omega[j] * std::sqrt(m->mass[j]));
        double bp = 0.0;
        for (int e = 0; e < n * n; ++e)
            bp += std::fabs(m->bpair[(size_t)p * n * n + e]);
        scale += bp * li * lj;
    }
    m->energy_scale = scale > 0.0 ? scale : 1.0;
    // two-state constants (closed-form kernels)
    if (n == 2) {
        m->kq.resize(M);
        m->minv.resize(M);
        m->kbar.resize(M);
        m->dlt.resize(M);
        m->cpl.resize(M);
        for (int j = 0; j < M; ++j) {
            const double *K = &m->k[(size_t)j * 4];
            m->kq[j] = m->mass[j] * m->omega[j] * m->omega[j];
            m->minv[j] = 1.0 / m->mass[j];
            m->kbar[j] = 0.5 * (K[0] + K[3]);
            m->dlt[j] = 0.5 * (K[0] - K[3]);
            m->cpl[j] = K[1];
        }
        m->dlt0 = 0.5 * (m->v0[0] - m->v0[3]);
        m->c0 = m->v0[1];
        if (D > 1) {
            // per mode and power k = 1..4 (zero past the degree): dl, cc and
            // Vbar parts of A_jk, as value and slope coefficients
            m->n2poly.assign((size_t)M * 20, 0.0);
            for (int j = 0; j < M; ++j)
                for (int k = 1; k <= D; ++k) {
                    const double *A = k == 1 ? &m->k[(size_t)j * 4]
                                             : &m->poly[((size_t)j * (D - 1) + (k - 2)) * 4];
                    const double bar = 0.5 * (A[0] + A[3]), dl = 0.5 * (A[0] - A[3]), cc = A[1];
                    double *row = &m->n2poly[(size_t)j * 20];
                    row[0 + k - 1] = dl;
                    row[4 + k - 1] = k * dl;
                    row[8 + k - 1] = cc;
                    row[12 + k - 1] = k * cc;
                    row[16 + k - 1] = k * bar;
                }
        }
    }

    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return device_fail(e, "hipGetDevice");
    }
    std::vector<double> packed(m->v0);
    packed.insert(packed.end(), m->k.begin(), m->k.end());
    m->c64_offset = packed.size();
    if (n == 2) {
        packed.push_back(m->dlt0);
        packed.push_back(m->c0);
        packed.insert(packed.end(), m->dlt.begin(), m->dlt.end());
        packed.insert(packed.end(), m->cpl.begin(), m->cpl.end());
        if (D > 1) {
            m->n2poly64_offset = packed.size();
            packed.push_back(m->dlt0);
            packed.push_back(m->c0);
            for (int part : {0, 8})  // dv, then cv
                for (int j = 0; j < M; ++j)
                    for (int k = 0; k < 4; ++k)
                        packed.push_back(m->n2poly[(size_t)j * 20 + part + k]);
        }
    }
    // general-N tables (factored couplings), binary64 then binary32
    const int T = n * (n + 1) / 2;
    std::vector<double> basis, coef, gen;
    for (int k = 0; k < n; ++k)
        for (int l = k; l < n; ++l)
            gen.push_back(m->v0[k * n + l]);
    if (D == 1) {
        std::vector<double> kmat((size_t)M * T);
        for (int j = 0; j < M; ++j)
            for (int k = 0, s = 0; k < n; ++k)
                for (int l = k; l < n; ++l, ++s)
                    kmat[(size_t)j * T + s] = m->k[(size_t)j * n * n + k * n + l];
        m->rank = factor_couplings(M, T, kmat, basis, coef);
        m->rank_pad = qcl::rank_bucket(m->rank, n);
        if (m->rank_pad == 1) {  // exact zeros off the diagonal: the kernels skip those products
            bool diag = true;
            for (int k = 0, sl = 0; k < n; ++k)
                for (int l = k; l < n; ++l, ++sl)
                    diag = diag && (k == l || m->rank == 0 || basis[sl] == 0.0);
            m->basis_diag = diag;
        }
        const int RB = m->rank_pad;
        // every direction kept: the slot basis (unit matrices), coefficients
        // the slot values themselves; the kernels skip its contractions
        const bool slots = RB == T;
        auto basis_rs = [&](int r, int s) {
            return slots ? (r == s ? 1.0 : 0.0) : (r < m->rank ? basis[(size_t)r * T + s] : 0.0);
        };
        auto coef_jr = [&](int j, int r) {
            return slots ? kmat[(size_t)j * T + r] : (r < m->rank ? coef[(size_t)j * m->rank + r] : 0.0);
        };
        for (int r = 0; r < RB; ++r)
            for (int s = 0; s < T; ++s)
                gen.push_back(basis_rs(r, s));
        for (int j = 0; j < qcl::kMaxModesPad; ++j) {
            const bool real = j < M;
            gen.push_back(real ? m->mass[j] * m->omega[j] * m->omega[j] : 0.0);
            gen.push_back(real ? 1.0 / m->mass[j] : 0.0);
            for (int r = 0; r < RB; ++r)
                gen.push_back(real ? coef_jr(j, r) : 0.0);
            for (int r = 0; r < RB; ++r)
                gen.push_back(real ? coef_jr(j, r) / m->mass[j] : 0.0);
        }
    } else {
        // rows (j, k), k = 1..4: A_j1 = K_j, A_jk from poly, zero past the degree
        std::vector<double> amat((size_t)M * 4 * T, 0.0);
        for (int j = 0; j < M; ++j)
            for (int k = 1; k <= D; ++k) {
                const double *A = k == 1 ? &m->k[(size_t)j * n * n]
                                         : &m->poly[((size_t)j * (D - 1) + (k - 2)) * n * n];
                for (int a = 0, s = 0; a < n; ++a)
                    for (int b = a; b < n; ++b, ++s)
                        amat[((size_t)j * 4 + (k - 1)) * T + s] = A[a * n + b];
            }
        m->rank = factor_couplings(M * 4, T, amat, basis, coef);
        m->rank_pad = T;
        const int RB = T;  // slot basis: the coefficients are the slot values
        for (int r = 0; r < RB; ++r)
            for (int s = 0; s < T; ++s)
                gen.push_back(r == s ? 1.0 : 0.0);
        for (int j = 0; j < qcl::kMaxModesPad; ++j) {
            const bool real = j < M;
            gen.push_back(real ? m->mass[j] * m->omega[j] * m->omega[j] : 0.0);
            gen.push_back(real ? 1.0 / m->mass[j] : 0.0);
            for (int r = 0; r < RB; ++r) {
                double c[4];
                for (int k = 0; k < 4; ++k)
                    c[k] = real ? amat[((size_t)j * 4 + k) * T + r] : 0.0;
                for (int k = 0; k < 4; ++k)
                    gen.push_back(c[k]);
                for (int k = 0; k < 4; ++k)
                    gen.push_back((k + 1) * c[k]);
            }
            if (m->n_pairs > 0)  // coefficients of mode j in the squared combinations (zero past n_sq)
                for (int sq = 0; sq < qcl::sq_pad(m->n_sq); ++sq)
                    gen.push_back(real && sq < m->n_sq ? m->sq_c[(size_t)sq * M + j] : 0.0);
        }
        if (m->n_pairs > 0)  // slot weights lambda [sq][slot]
            for (int sq = 0; sq < qcl::sq_pad(m->n_sq); ++sq)
                for (int r = 0; r < T; ++r)
                    gen.push_back(sq < m->n_sq ? m->sq_lam[(size_t)sq * T + r] : 0.0);
    }
    while (packed.size() % 32)
        packed.push_back(0.0);
    m->gen64_offset = packed.size();
    packed.insert(packed.end(), gen.begin(), gen.end());
    while (packed.size() % 32)
        packed.push_back(0.0);
    m->gen32_byte_offset = packed.size() * sizeof(double);
    std::vector<float> gen32(gen.begin(), gen.end());
    const size_t n32 = (gen32.size() + 1) / 2;  // floats packed two per double slot
    const size_t base = packed.size();
    packed.resize(base + n32, 0.0);
    std::memcpy(packed.data() + base, gen32.data(), gen32.size() * sizeof(float));
    const size_t bytes = sizeof(double) * packed.size();
    e = hipMalloc((void **)&m->d_model, bytes);
    if (e != hipSuccess) {
        delete m;
        return e == hipErrorOutOfMemory ? fail(QCL_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes", bytes)
                                        : device_fail(e, "hipMalloc");
    }
    e = hipMemcpy(m->d_model, packed.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(m->d_model);
        delete m;
        return device_fail(e, "hipMemcpy");
    }
    *out = m;
    return QCL_OK;
}

// A model with a supplied potential (qcl_create_model_source): the source
// is compiled first (no device needed), then loaded on the current device.
qcl_status create_model_source(const qcl_model_desc *d, const qcl_source_desc *src, qcl_model *out)
{
    if (!d || !src || !out)
        return fail(QCL_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const int n = d->n_states, M = d->n_modes;
    if (n < 2 || n > 4)
        return fail(QCL_ERR_INVALID_ARG, "n_states %d outside [2, 4] for a supplied potential", n);
    if (M < 1 || M > QCL_MAX_MODES_SOURCE)
        return fail(QCL_ERR_INVALID_ARG, "n_modes %d outside [1, %d] for a supplied potential", M,
                    QCL_MAX_MODES_SOURCE);
    if (!d->mass || !d->omega)
        return fail(QCL_ERR_INVALID_ARG, "mass or omega is NULL");
    if (!(d->hbar > 0.0) || !std::isfinite(d->hbar))
        return fail(QCL_ERR_INVALID_ARG, "hbar must be finite and > 0");
    if (!finite_all(d->mass, M) || !finite_all(d->omega, M))
        return fail(QCL_ERR_INVALID_ARG, "non-finite model parameter");
    for (int j = 0; j < M; ++j)
        if (!(d->mass[j] > 0.0) || !(d->omega[j] > 0.0))
            return fail(QCL_ERR_INVALID_ARG, "mass and omega must be > 0 (mode %d)", j);
    if (!src->source)
        return fail(QCL_ERR_INVALID_ARG, "source is NULL");
    if (src->n_params < 0 || src->n_params > QCL_MAX_PARAMS)
        return fail(QCL_ERR_INVALID_ARG, "n_params %d outside [0, %d]", src->n_params, QCL_MAX_PARAMS);
    if (src->n_params > 0 && (!src->params || !finite_all(src->params, src->n_params)))
        return fail(QCL_ERR_INVALID_ARG, "params is NULL or not finite");
    qcl_model_s *m = new (std::nothrow) qcl_model_s();
    if (!m)
        return fail(QCL_ERR_OUT_OF_MEMORY, "host allocation failed");
    m->n = n;
    m->m = M;
    m->hbar = d->hbar;
    m->mass.assign(d->mass, d->mass + M);
    m->omega.assign(d->omega, d->omega + M);
    m->v0.assign((size_t)n * n, 0.0);
    m->k.assign((size_t)M * n * n, 0.0);
    m->source = true;
    if (qcl_status st = qcl::user_compile(*m, src->source, src->params, src->n_params)) {
        delete m;
        return st;
    }
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return device_fail(e, "hipGetDevice");
    }
    if (qcl_status st = qcl::user_load(*m)) {
        delete m;
        return st;
    }
    *out = m;
    return QCL_OK;
}

}  // namespace

namespace qcl {

qcl_status set_error(qcl_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

// The batched call with a given workspace.  fixed_workspace: the library's
// own per-device array (qcl_propagate_batch_static): a plan that does not
// fit is reported against its stated limit, and every class runs on the
// caller's stream in turn (no side streams are created).
qcl_status propagate_batch_in(const qcl_batch_item *items, int32_t n_items, void *workspace, size_t workspace_bytes,
                              void *stream, bool fixed_workspace)
{
    BatchPlan plan;
    if (qcl_status st = plan_batch(items, n_items, plan))
        return st;
    if (plan.bytes > 0) {
        if (!workspace || ((uintptr_t)workspace % 256))
            return fail(QCL_ERR_INVALID_ARG, "workspace is NULL or not 256-byte aligned");
        if (workspace_bytes < plan.bytes)
            return fixed_workspace
                       ? fail(QCL_ERR_INVALID_ARG,
                              "this batch needs %zu bytes of descriptors; the static workspace holds %zu "
                              "(QCL_STATIC_WORKSPACE_BYTES): split the batch, or use qcl_propagate_batch",
                              plan.bytes, workspace_bytes)
                       : fail(QCL_ERR_INVALID_ARG, "workspace holds %zu bytes, %zu needed", workspace_bytes,
                              plan.bytes);
    }
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    std::vector<uint64_t> words(plan.bytes / 8, 0);
    for (const BatchClass &c : plan.classes) {
        int64_t tile_begin = 0;
        for (size_t k = 0; k < c.order.size(); ++k) {
            const qcl_batch_item &it = items[c.order[k]];
            qcl::batch_item(*it.model, *it.ens, it.prop, it.partials, tile_begin,
                            (uint8_t *)words.data() + c.offset + k * c.item_bytes);
            tile_begin += qcl::n_tiles(it.ens->n_traj);
        }
    }
    if (plan.bytes > 0) {
        // counters (first word of each class block) are zero in the uploaded image
        hipError_t e = qcl::upload_words(words.data(), words.size(), (uint64_t *)ws, s);
        if (e != hipSuccess)
            return device_fail(e, "batch descriptor upload");
    }
    auto launch_class = [&](const BatchClass &c, hipStream_t on) {
        return qcl::launch_batch(*items[c.order[0]].model, c.prec, c.scheme, c.occ, c.wpc, ws + c.offset,
                                 (int32_t)c.order.size(), c.total_tiles,
                                 (unsigned long long *)(ws + c.counter_offset), on);
    };
    hipError_t e = hipSuccess;
    if (plan.classes.size() == 1 || fixed_workspace) {
        for (const BatchClass &c : plan.classes)
            if (e == hipSuccess)
                e = launch_class(c, s);
    } else if (plan.classes.size() > 1) {
        // heaviest class first, each on the side stream with the least
        // estimated work so far (longest-processing-time order), so the
        // streams finish close together; a class whose last tiles leave
        // CUs idle is overlapped by the classes on the other streams
        std::lock_guard<std::mutex> lock(g_fan_mutex);
        Fan *f = nullptr;
        if ((e = device_fan(f)) != hipSuccess)
            return device_fail(e, "side stream set-up");
        const int used = (int)std::min<size_t>(kSideStreams, plan.classes.size());
        if ((e = hipEventRecord(f->fork, s)) != hipSuccess)
            return device_fail(e, "hipEventRecord");
        for (int k = 0; k < used; ++k)
            if ((e = hipStreamWaitEvent(f->s[k], f->fork, 0)) != hipSuccess)
                return device_fail(e, "hipStreamWaitEvent");
        double load[kSideStreams] = {};
        for (size_t i = 0; i < plan.classes.size() && e == hipSuccess; ++i) {
            int k = 0;
            for (int j = 1; j < used; ++j)
                k = load[j] < load[k] ? j : k;
            load[k] += plan.classes[i].cost;
            e = launch_class(plan.classes[i], f->s[k]);
        }
        // join whatever was launched back into the caller's stream
        for (int k = 0; k < used; ++k) {
            hipError_t ej = hipEventRecord(f->join[k], f->s[k]);
            if (ej == hipSuccess)
                ej = hipStreamWaitEvent(s, f->join[k], 0);
            if (ej != hipSuccess && e == hipSuccess)
                e = ej;
        }
    }
    if (e == hipErrorNotSupported)
        return fail(QCL_ERR_UNSUPPORTED, "no batched kernel for this model class");
    if (e != hipSuccess)
        return device_fail(e, "batched propagate launch");
    for (int32_t i = 0; i < n_items; ++i)
        items[i].ens->step += items[i].prop.n_steps;
    return QCL_OK;
}

}  // namespace qcl

extern "C" {

const char *qcl_last_error(void) { return g_last_error.c_str(); }

qcl_status qcl_create_model(const qcl_model_desc *d, qcl_model *out) { return create_model(d, nullptr, nullptr, out); }

qcl_status qcl_create_model_source(const qcl_model_desc *d, const qcl_source_desc *src, qcl_model *out)
{
    return create_model_source(d, src, out);
}

int32_t qcl_model_is_source(qcl_model m) { return m && m->source ? 1 : 0; }

qcl_status qcl_create_model_poly(const qcl_model_desc *d, const qcl_poly_desc *poly, qcl_model *out)
{
    if (!poly) {
        if (out)
            *out = nullptr;
        return fail(QCL_ERR_INVALID_ARG, "poly is NULL");
    }
    return create_model(d, poly, nullptr, out);
}

qcl_status qcl_create_model_bilinear(const qcl_model_desc *d, const qcl_poly_desc *poly, const qcl_bilinear_desc *bil,
                                     qcl_model *out)
{
    if (!bil) {
        if (out)
            *out = nullptr;
        return fail(QCL_ERR_INVALID_ARG, "bil is NULL");
    }
    return create_model(d, poly, bil, out);
}

int32_t qcl_model_pairs(qcl_model m) { return m ? m->n_pairs : 0; }

int32_t qcl_model_degree(qcl_model m) { return m ? m->degree : 0; }

qcl_status qcl_destroy_model(qcl_model m)
{
    if (!m)
        return QCL_OK;
    if (m->d_model)
        (void)hipFree(m->d_model);
    qcl::user_release(*m);
    delete m;
    return QCL_OK;
}

int32_t qcl_model_states(qcl_model m) { return m ? m->n : 0; }
int32_t qcl_model_modes(qcl_model m) { return m ? m->m : 0; }
int32_t qcl_model_rank(qcl_model m) { return m ? m->rank : 0; }

qcl_status qcl_ensemble_bytes(qcl_model m, int64_t n_traj, int32_t prec, int64_t *ld, size_t *bytes)
{
    if (qcl_status st = check_model(m))
        return st;
    if (!ld || !bytes)
        return fail(QCL_ERR_INVALID_ARG, "NULL output");
    if (n_traj < 0 || n_traj > ((int64_t)1 << 40))
        return fail(QCL_ERR_INVALID_ARG, "n_traj out of range");
    if (prec != QCL_FP64 && prec != QCL_FP32_ACC64)
        return fail(QCL_ERR_INVALID_ARG, "unknown precision %d", prec);
    const int64_t L = leading_dim(n_traj);
    const size_t rs = real_size(prec);
    size_t b = 0;
    b += align256((size_t)m->m * L * rs);          // q
    b += align256((size_t)m->m * L * rs);          // p
    b += align256((size_t)m->n * m->n * L * rs);   // u
    b += align256((size_t)L * 8);                  // w
    b += align256((size_t)L * 8);                  // phase
    b += align256((size_t)L);                      // a
    b += align256((size_t)L);                      // b
    b += align256((size_t)L * 4);                  // flags
    *ld = L;
    *bytes = b;
    return QCL_OK;
}

qcl_status qcl_ensemble_bind(qcl_model m, void *base, int64_t n_traj, int32_t prec, int64_t traj_offset,
                             qcl_ensemble *e)
{
    int64_t L;
    size_t total;
    if (qcl_status st = qcl_ensemble_bytes(m, n_traj, prec, &L, &total))
        return st;
    if (!e || !base)
        return fail(QCL_ERR_INVALID_ARG, "NULL argument");
    if ((uintptr_t)base % 256)
        return fail(QCL_ERR_INVALID_ARG, "base must be 256-byte aligned");
    if (traj_offset < 0)
        return fail(QCL_ERR_INVALID_ARG, "traj_offset < 0");
    const size_t rs = real_size(prec);
    char *c = (char *)base;
    std::memset(e, 0, sizeof(*e));
    e->n_traj = n_traj;
    e->ld = L;
    e->traj_offset = traj_offset;
    e->step = 0;
    e->prec = prec;
    e->q = c; c += align256((size_t)m->m * L * rs);
    e->p = c; c += align256((size_t)m->m * L * rs);
    e->u = c; c += align256((size_t)m->n * m->n * L * rs);
    e->w = (double *)c; c += align256((size_t)L * 8);
    e->phase = (double *)c; c += align256((size_t)L * 8);
    e->a = (uint8_t *)c; c += align256((size_t)L);
    e->b = (uint8_t *)c; c += align256((size_t)L);
    e->flags = (uint32_t *)c;
    return QCL_OK;
}

qcl_status qcl_partials_bytes(qcl_model m, int64_t n_traj, int32_t n_out, size_t *bytes)
{
    if (qcl_status st = check_model(m))
        return st;
    if (!bytes)
        return fail(QCL_ERR_INVALID_ARG, "NULL output");
    if (n_traj < 0 || n_out < 1)
        return fail(QCL_ERR_INVALID_ARG, "n_traj >= 0 and n_out >= 1 required");
    *bytes = (partials_rows(n_traj) * n_out * qcl::tile_values(m->n) + n_out) * sizeof(double);
    return QCL_OK;
}

qcl_status qcl_sample_initial(qcl_model m, const qcl_init_desc *init, uint64_t seed, qcl_ensemble *ens,
                              double *partials, int32_t n_out, void *stream)
{
    if (qcl_status st = check_model(m))
        return st;
    if (qcl_status st = check_ensemble(*m, ens))
        return st;
    if (!init || !init->q0)
        return fail(QCL_ERR_INVALID_ARG, "init or init->q0 is NULL");
    if (!(init->kT >= 0.0) || !std::isfinite(init->kT))
        return fail(QCL_ERR_INVALID_ARG, "kT must be finite and >= 0");
    if (init->state < 0 || init->state >= m->n)
        return fail(QCL_ERR_INVALID_ARG, "initial state %d outside [0, %d)", init->state, m->n);
    if (init->basis != QCL_INIT_DIABATIC && init->basis != QCL_INIT_ADIABATIC)
        return fail(QCL_ERR_INVALID_ARG, "unknown basis %d", init->basis);
    if (!finite_all(init->q0, m->m))
        return fail(QCL_ERR_INVALID_ARG, "non-finite q0");
    if (n_out < 1)
        return fail(QCL_ERR_INVALID_ARG, "n_out must be >= 1");
    if (ens->n_traj > 0 && (!partials || !aligned256(partials)))
        return fail(QCL_ERR_INVALID_ARG, "partials is NULL or not 256-byte aligned");
    qcl::SampleArgs sa{};
    for (int j = 0; j < m->m; ++j) {
        const double w = m->omega[j], ms = m->mass[j], hb = m->hbar;
        const double th = init->kT > 0.0 ? std::tanh(hb * w / (2.0 * init->kT)) : 1.0;
        sa.q0[j] = init->q0[j];
        sa.sq[j] = std::sqrt(hb / (2.0 * ms * w * th));
        sa.sp[j] = std::sqrt(hb * ms * w / (2.0 * th));
    }
    sa.state = init->state;
    sa.basis = init->basis;
    sa.key0 = (uint32_t)seed;
    sa.key1 = (uint32_t)(seed >> 32);
    if (ens->n_traj == 0) {
        ens->step = 0;
        return QCL_OK;
    }
    if (qcl_status st = check_device(*m))
        return st;
    hipError_t e = m->source  ? qcl::launch_user_sample(*m, sa, *ens, partials, n_out, (hipStream_t)stream)
                   : m->fast2 ? qcl::launch_sample_n2(*m, sa, *ens, partials, n_out, (hipStream_t)stream)
                              : qcl::launch_sample_general(*m, sa, *ens, partials, n_out, (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(QCL_ERR_UNSUPPORTED, "no sampling kernel for this model");
    if (e != hipSuccess)
        return device_fail(e, "sample kernel launch");
    ens->step = 0;
    return QCL_OK;
}

qcl_status qcl_propagate(qcl_model m, qcl_ensemble *ens, const qcl_prop_desc *pd, double *partials, void *stream)
{
    if (qcl_status st = check_propagate(m, ens, pd, partials))
        return st;
    if (ens->n_traj == 0 || pd->n_steps == 0) {
        ens->step += pd->n_steps;
        return QCL_OK;
    }
    hipError_t e = m->source  ? qcl::launch_user_propagate(*m, *ens, *pd, partials, (hipStream_t)stream)
                   : m->fast2 ? qcl::launch_propagate_n2(*m, *ens, *pd, partials, (hipStream_t)stream)
                              : qcl::launch_propagate_general(*m, *ens, *pd, partials, (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(QCL_ERR_UNSUPPORTED, "no propagation kernel for this model");
    if (e != hipSuccess)
        return device_fail(e, "propagate kernel launch");
    ens->step += pd->n_steps;
    return QCL_OK;
}

qcl_status qcl_batch_workspace_bytes(const qcl_batch_item *items, int32_t n_items, size_t *bytes)
{
    if (!bytes)
        return fail(QCL_ERR_INVALID_ARG, "bytes is NULL");
    BatchPlan plan;
    if (qcl_status st = plan_batch(items, n_items, plan))
        return st;
    *bytes = plan.bytes;
    return QCL_OK;
}

qcl_status qcl_propagate_batch(const qcl_batch_item *items, int32_t n_items, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    return qcl::propagate_batch_in(items, n_items, workspace, workspace_bytes, stream, false);
}

qcl_status qcl_resample_workspace_bytes(int64_t n_traj, size_t *bytes)
{
    if (!bytes)
        return fail(QCL_ERR_INVALID_ARG, "bytes is NULL");
    if (n_traj < 0 || n_traj >= ((int64_t)1 << 31))
        return fail(QCL_ERR_INVALID_ARG, "resampling needs 0 <= n_traj < 2^31");
    *bytes = n_traj == 0 ? 0 : qcl::resample_layout(n_traj).bytes;
    return QCL_OK;
}

qcl_status qcl_resample(qcl_model m, const qcl_ensemble *src, qcl_ensemble *dst, uint64_t seed, void *workspace,
                        size_t workspace_bytes, void *stream)
{
    if (qcl_status st = check_model(m))
        return st;
    if (qcl_status st = check_ensemble(*m, src))
        return st;
    if (qcl_status st = check_ensemble(*m, dst))
        return st;
    if (src->n_traj != dst->n_traj || src->prec != dst->prec || src->ld != dst->ld ||
        src->traj_offset != dst->traj_offset)
        return fail(QCL_ERR_INVALID_ARG, "src and dst differ in n_traj, precision, ld or traj_offset");
    if (src->n_traj >= ((int64_t)1 << 31))
        return fail(QCL_ERR_INVALID_ARG, "resampling needs n_traj < 2^31");
    if (src->n_traj > 0) {
        const void *a[] = {src->q, src->p, src->u, src->w, src->phase, src->a, src->b, src->flags};
        const void *b[] = {dst->q, dst->p, dst->u, dst->w, dst->phase, dst->a, dst->b, dst->flags};
        for (const void *x : a)
            for (const void *y : b)
                if (x && x == y)
                    return fail(QCL_ERR_INVALID_ARG, "src and dst share an array");
        const size_t need = qcl::resample_layout(src->n_traj).bytes;
        if (!workspace || ((uintptr_t)workspace % 256) || workspace_bytes < need)
            return fail(QCL_ERR_INVALID_ARG, "workspace must be 256-byte aligned and hold %zu bytes", need);
        if (qcl_status st = check_device(*m))
            return st;
        const hipError_t e = qcl::launch_resample(*m, *src, *dst, seed, workspace, (hipStream_t)stream);
        if (e != hipSuccess)
            return device_fail(e, "resample launch");
    }
    dst->step = src->step;
    return QCL_OK;
}

qcl_status qcl_reduce_observables_async(qcl_model m, double *partials, int64_t n_traj, int32_t n_out, double *out,
                                        int64_t *excluded, void *stream)
{
    if (qcl_status st = check_reduce(m, partials, n_traj, n_out, out))
        return st;
    if (excluded && !aligned256(excluded))
        return fail(QCL_ERR_INVALID_ARG, "excluded is not 256-byte aligned");
    hipError_t e = qcl::launch_reduce(m->n, partials, n_traj, n_out, out, excluded, (hipStream_t)stream);
    if (e != hipSuccess)
        return device_fail(e, "reduce kernel launch");
    return QCL_OK;
}

qcl_status qcl_reduce_observables(qcl_model m, double *partials, int64_t n_traj, int32_t n_out, double *out,
                                  void *stream)
{
    if (qcl_status st = check_reduce(m, partials, n_traj, n_out, out))
        return st;
    // the counts go to the slots after the scratch rows of the partials
    int64_t *counts = (int64_t *)(partials + partials_rows(n_traj) * n_out * qcl::tile_values(m->n));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = qcl::launch_reduce(m->n, partials, n_traj, n_out, out, counts, s);
    if (e != hipSuccess)
        return device_fail(e, "reduce kernel launch");
    int64_t worst = 0, worst_bin = -1, first_bin = -1;
    int64_t buf[256];  // counts are read back in chunks: nothing is allocated
    for (int32_t o0 = 0; o0 < n_out; o0 += 256) {
        const int32_t n = std::min<int32_t>(256, n_out - o0);
        if ((e = hipMemcpyAsync(buf, counts + o0, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return device_fail(e, "reading the excluded counts");
        for (int32_t k = 0; k < n; ++k) {
            if (buf[k] > 0 && first_bin < 0)
                first_bin = o0 + k;
            if (buf[k] > worst) {
                worst = buf[k];
                worst_bin = o0 + k;
            }
        }
    }
    if (worst > 0)
        return fail(QCL_ERR_NONFINITE,
                    "%lld of %lld walkers excluded from bin %lld (non-finite weight or phase; first excluded at bin "
                    "%lld); the averages are over the finite walkers, normalised by all %lld",
                    (long long)worst, (long long)n_traj, (long long)worst_bin, (long long)first_bin,
                    (long long)n_traj);
    return QCL_OK;
}

}  // extern "C"
