// Refinement of the HSS solution on the exact kernel (the HSS factorization
// used as a preconditioner, as proposed in Section 6): preconditioned
// conjugate gradients on (K + lambda I) alpha = Y, one independent recurrence
// per right-hand side, kernel products by kernel_matvec, preconditioner solves
// by the ULV factor, stopping on the recomputed true residual.  Also the
// label kernel of prediction (Algorithm 1 step 4; one-vs-all argmax).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace krr {


namespace {

// Per-row problem index of a batch (nullptr: one problem).  Coefficients are
// stored per (problem, right-hand side): coef[p * k + c].
__device__ __forceinline__ int prob_of(const int32_t *pid, int64_t i) { return pid ? pid[i] : 0; }

// r = Y - Kx - lambda x
__global__ void k_residual(const double *__restrict__ Y, const double *__restrict__ Kx, const double *__restrict__ x,
                           const double *__restrict__ lam, const int32_t *__restrict__ pid, int64_t n, int k,
                           double *__restrict__ r) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * k) r[t] = Y[t] - Kx[t] - lam[prob_of(pid, t / k)] * x[t];
}

// y[:, c] = a[p, c] * x[:, c] + b[p, c] * y[:, c]
__global__ void k_axpby(const double *__restrict__ a, const double *__restrict__ x, const double *__restrict__ b,
                        double *__restrict__ y, const int32_t *__restrict__ pid, int64_t n, int k) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int c = (int)(t % k);
    const int64_t ci = (int64_t)prob_of(pid, t / k) * k + c;
    y[t] = a[ci] * x[t] + b[ci] * y[t];
}

// q = Kp + lambda p (in place on Kp)
__global__ void k_add_shift(double *__restrict__ Kp, const double *__restrict__ p, const double *__restrict__ lam,
                            const int32_t *__restrict__ pid, int64_t n, int k) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * k) Kp[t] += lam[prob_of(pid, t / k)] * p[t];
}

// Segmented column dots: out[p * k + c] = sum over rows of problem p of a b
// (one workgroup per (problem, column); rows in order, FP64).
__global__ __launch_bounds__(256) void k_seg_dot(const double *__restrict__ a, const double *__restrict__ b,
                                                 const int64_t *__restrict__ pbeg, int k, double *__restrict__ out) {
    __shared__ double red[4];
    const int p = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    double acc = 0.0;
    for (int64_t i = pbeg[p] + tid; i < pbeg[p + 1]; i += 256) acc += a[i * k + c] * b[i * k + c];
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) out[(int64_t)p * k + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_fill_pid(const int64_t *__restrict__ pbeg, int np, int64_t n, int32_t *__restrict__ pid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = np - 1;  // last p with pbeg[p] <= i
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (pbeg[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    pid[i] = lo;
}

__global__ void k_labels(const double *__restrict__ S, int64_t m, int k, int32_t *__restrict__ lab) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (k == 1) {
        lab[i] = S[i] >= 0.0 ? 1 : -1;
        return;
    }
    int best = 0;
    double bv = S[i * k];
    for (int c = 1; c < k; ++c)
        if (S[i * k + c] > bv) {
            bv = S[i * k + c];
            best = c;
        }
    lab[i] = best;
}

// The problems of a solve: one (plain column dots) or a batch (segmented).
struct Segs {
    int np = 1;
    int64_t n = 0;
    int k = 1;
    DBuf pbeg, pid, lam, coef, out, scratch;

    std::vector<double> dots(const double *a, const double *b, hipStream_t s) {
        const size_t cnt = (size_t)np * k;
        out.reserve(sizeof(double) * cnt);
        if (np == 1) {
            dot_columns(a, b, n, k, out.as<double>(), scratch, s);
        } else {
            k_seg_dot<<<dim3(np, k), 256, 0, s>>>(a, b, pbeg.as<int64_t>(), k, out.as<double>());
            check_launch("k_seg_dot");
        }
        std::vector<double> h(cnt);
        d2h(h.data(), out.as<double>(), cnt, s);
        sync(s);
        return h;
    }
    // y = a x + b y with per-(problem, column) coefficients
    void axpby(const std::vector<double> &a, const double *x, const std::vector<double> &b, double *y, hipStream_t s) {
        const size_t cnt = (size_t)np * k;
        std::vector<double> ab(a);
        ab.insert(ab.end(), b.begin(), b.end());
        coef.reserve(sizeof(double) * 2 * cnt);
        h2d(coef.as<double>(), ab.data(), 2 * cnt, s);
        k_axpby<<<ceil_div(n * k, 256), 256, 0, s>>>(coef.as<double>(), x, coef.as<double>() + cnt, y,
                                                     pid.as<int32_t>(), n, k);
        check_launch("k_axpby");
        sync(s);  // `ab` is released on return
    }
};

}  // namespace

void predict_labels(const double *scores, int64_t m, int k, int32_t *labels, hipStream_t s) {
    if (m == 0) return;
    k_labels<<<ceil_div(m, 256), 256, 0, s>>>(scores, m, k, labels);
    check_launch("k_labels");
}

int refine(const hss_ulv_s *F, int64_t n, const void *Xp, int xprec, int d, double h, double lambda, const double *Y,
           int nrhs, double *alpha, double tol, int max_iter, int mv_prec, int res_prec, hipStream_t s,
           krr_refine_stats *st,
           const Batch *batch, double *relres_all) {
    EventTimer timer(s);
    const int64_t len = n * nrhs;
    Segs sg;
    sg.n = n;
    sg.k = nrhs;
    std::vector<double> lam_h(1, lambda);
    if (batch && batch->np() > 1) {
        sg.np = batch->np();
        lam_h = batch->lam;
        sg.pbeg = upload(batch->pbeg, s);
        sg.pid = dalloc<int32_t>(n);
        k_fill_pid<<<ceil_div(n, 256), 256, 0, s>>>(sg.pbeg.as<int64_t>(), sg.np, n, sg.pid.as<int32_t>());
        check_launch("k_fill_pid");
    } else if (batch) {
        lam_h = batch->lam;
        h = batch->h[0];
        batch = nullptr;
    }
    sg.lam = upload(lam_h, s);
    const int np = sg.np, cnt = np * nrhs;
    DBuf r = dalloc<double>(len), z = dalloc<double>(len), p = dalloc<double>(len), q = dalloc<double>(len);
    // q's rows of problems that the products leave out keep finite values
    KRR_HIP(hipMemsetAsync(q.get(), 0, sizeof(double) * len, s));
    // the inner products leave out problems whose every right-hand side has
    // converged (their step lengths are 0 from then on)
    Batch active;
    if (batch) active = *batch;
    auto precond = [&](const double *in, double *out) {
        if (F)
            ulv_solve(F, in, nrhs, out, s);
        else
            KRR_HIP(hipMemcpyAsync(out, in, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
    };
    int matvecs = 0;
    // The products see the same points and widths throughout, so the
    // negligible tiles of the symmetric product are found once: by the first
    // true residual when it takes that form (recording evaluates every
    // entry), else by the first iteration's product.  The iterations' products
    // skip them; the true residuals that confirm convergence evaluate every
    // entry.
    SymSkip skipmap;
    auto matvec = [&](const double *x, double *out, int prec, const Batch *b, SymSkip *sk) {
        kernel_matvec_impl(Xp, n, Xp, n, d, xprec, h, x, nrhs, 0.0, out, prec, s, b, sk);
        ++matvecs;
    };
    auto true_residual = [&]() {
        matvec(alpha, q.as<double>(), res_prec, batch, skipmap.ready ? nullptr : &skipmap);
        k_residual<<<ceil_div(len, 256), 256, 0, s>>>(Y, q.as<double>(), alpha, sg.lam.as<double>(),
                                                      sg.pid.as<int32_t>(), n, nrhs, r.as<double>());
        check_launch("k_residual");
    };
    std::vector<double> ynorm = sg.dots(Y, Y, s);
    for (auto &v : ynorm) v = std::sqrt(v) > 0 ? std::sqrt(v) : 1.0;
    true_residual();
    std::vector<double> rr = sg.dots(r.as<double>(), r.as<double>(), s);
    auto rel = [&](const std::vector<double> &v) {
        std::vector<double> o(cnt);
        for (int c = 0; c < cnt; ++c) o[c] = std::sqrt(std::max(v[c], 0.0)) / ynorm[c];
        return o;
    };
    auto all_below = [&](const std::vector<double> &v) {
        for (double x : v)
            if (!(x <= tol)) return false;
        return true;
    };
    std::vector<double> relres = rel(rr);
    // The recurrence's residual stops an iteration at inner * tol.  With the
    // true residual formed in the iterations' own precision the two track
    // each other closely (the negligible-tile map drops entries below 2^-32
    // only), so 0.8 leaves a 20% margin; when the true residual is formed in
    // FP64 from FP32 iterations, their gap is the FP32 products' error, and
    // the inner target is halved.
    const double inner = res_prec == mv_prec ? 0.8 : 0.5;
    int it = 0;
    bool converged = all_below(relres);
    while (!converged && it < max_iter) {
        // (re)start: z = M^{-1} r, p = z
        precond(r.as<double>(), z.as<double>());
        KRR_HIP(hipMemcpyAsync(p.get(), z.get(), sizeof(double) * len, hipMemcpyDeviceToDevice, s));
        std::vector<double> rz = sg.dots(r.as<double>(), z.as<double>(), s);
        std::vector<bool> done(cnt);
        for (int c = 0; c < cnt; ++c) done[c] = relres[c] <= tol;
        while (it < max_iter) {
            ++it;
            if (batch) {
                active.skip.assign(np, 0);
                for (int pp = 0; pp < np; ++pp) {
                    bool all = true;
                    for (int c = 0; c < nrhs; ++c) all = all && done[(size_t)pp * nrhs + c];
                    active.skip[pp] = all ? 1 : 0;
                }
            }
            matvec(p.as<double>(), q.as<double>(), mv_prec, batch ? &active : nullptr, &skipmap);
            k_add_shift<<<ceil_div(len, 256), 256, 0, s>>>(q.as<double>(), p.as<double>(), sg.lam.as<double>(),
                                                           sg.pid.as<int32_t>(), n, nrhs);
            check_launch("k_add_shift");
            std::vector<double> pq = sg.dots(p.as<double>(), q.as<double>(), s);
            std::vector<double> a(cnt), one(cnt, 1.0), ma(cnt);
            for (int c = 0; c < cnt; ++c) {
                a[c] = (done[c] || pq[c] <= 0.0) ? 0.0 : rz[c] / pq[c];
                ma[c] = -a[c];
            }
            sg.axpby(a, p.as<double>(), one, alpha, s);         // alpha += a p
            sg.axpby(ma, q.as<double>(), one, r.as<double>(), s); // r -= a q
            rr = sg.dots(r.as<double>(), r.as<double>(), s);
            std::vector<double> rec = rel(rr);
            if (verbose()) {
                double mx = 0;
                for (double v : rec) mx = std::max(mx, v);
                fprintf(stderr, "[krr] refine it=%d relres(recurrence, max)=%.3e\n", it, mx);
            }
            bool stop = true;
            for (int c = 0; c < cnt; ++c) {
                if (rec[c] <= inner * tol) done[c] = true;
                stop = stop && done[c];
            }
            if (stop) break;
            precond(r.as<double>(), z.as<double>());
            std::vector<double> rz2 = sg.dots(r.as<double>(), z.as<double>(), s);
            std::vector<double> beta(cnt);
            for (int c = 0; c < cnt; ++c) {
                beta[c] = (done[c] || rz[c] == 0.0) ? 0.0 : rz2[c] / rz[c];
                rz[c] = rz2[c];
            }
            sg.axpby(one, z.as<double>(), beta, p.as<double>(), s);  // p = z + beta p
        }
        // confirm on the true residual; restart from it if the recurrence drifted
        true_residual();
        rr = sg.dots(r.as<double>(), r.as<double>(), s);
        relres = rel(rr);
        converged = all_below(relres);
        if (verbose()) fprintf(stderr, "[krr] refine it=%d true relres=%.3e\n", it, relres[0]);
    }
    if (relres_all) std::copy(relres.begin(), relres.end(), relres_all);
    if (st) {
        st->iterations = it;
        st->matvecs = matvecs;
        // per right-hand side: the largest relative residual over the problems
        for (int c = 0; c < 64; ++c) {
            double mx = 0.0;
            if (c < nrhs)
                for (int pp = 0; pp < np; ++pp) mx = std::max(mx, relres[(size_t)pp * nrhs + c]);
            st->relres[c] = mx;
        }
        st->t_ms = timer.stop_ms();
    }
    sync(s);
    return converged ? KRR_OK : KRR_E_NOT_CONVERGED;
}

}  // namespace krr
