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

void kernel_matvec_impl(const void *X, int64_t m, const void *Y, int64_t n, int d, int xprec, double h,
                        const double *W, int nrhs, double beta, double *Out, int prec, hipStream_t s);
void dot_columns(const double *a, const double *b, int64_t n, int k, double *out, DBuf &scratch, hipStream_t s);
void ulv_solve(const hss_ulv_s *F, const double *Bin, int nrhs, double *Xout, hipStream_t s);

namespace {

// r = Y - Kx - lambda x
__global__ void k_residual(const double *__restrict__ Y, const double *__restrict__ Kx, const double *__restrict__ x,
                           double lambda, int64_t len, double *__restrict__ r) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) r[t] = Y[t] - Kx[t] - lambda * x[t];
}

// y[:, c] = a[c] * x[:, c] + b[c] * y[:, c]
__global__ void k_axpby(const double *__restrict__ a, const double *__restrict__ x, const double *__restrict__ b,
                        double *__restrict__ y, int64_t n, int k) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int c = (int)(t % k);
    y[t] = a[c] * x[t] + b[c] * y[t];
}

// q = Kp + lambda p (in place on Kp)
__global__ void k_add_shift(double *__restrict__ Kp, const double *__restrict__ p, double lambda, int64_t len) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) Kp[t] += lambda * p[t];
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

void axpby(const std::vector<double> &a, const double *x, const std::vector<double> &b, double *y, int64_t n, int k,
           DBuf &coef, hipStream_t s) {
    std::vector<double> ab(a);
    ab.insert(ab.end(), b.begin(), b.end());
    coef.reserve(sizeof(double) * 2 * k);
    h2d(coef.as<double>(), ab.data(), 2 * k, s);
    k_axpby<<<ceil_div(n * k, 256), 256, 0, s>>>(coef.as<double>(), x, coef.as<double>() + k, y, n, k);
    check_launch("k_axpby");
    sync(s);  // `ab` is released on return
}

std::vector<double> dots(const double *a, const double *b, int64_t n, int k, DBuf &out, DBuf &scratch,
                         hipStream_t s) {
    out.reserve(sizeof(double) * k);
    dot_columns(a, b, n, k, out.as<double>(), scratch, s);
    std::vector<double> h(k);
    d2h(h.data(), out.as<double>(), k, s);
    sync(s);
    return h;
}

}  // namespace

void predict_labels(const double *scores, int64_t m, int k, int32_t *labels, hipStream_t s) {
    if (m == 0) return;
    k_labels<<<ceil_div(m, 256), 256, 0, s>>>(scores, m, k, labels);
    check_launch("k_labels");
}

int refine(const hss_ulv_s *F, int64_t n, const void *Xp, int xprec, int d, double h, double lambda, const double *Y,
           int nrhs, double *alpha, double tol, int max_iter, int mv_prec, hipStream_t s, krr_refine_stats *st) {
    EventTimer timer(s);
    const int64_t len = n * nrhs;
    DBuf r = dalloc<double>(len), z = dalloc<double>(len), p = dalloc<double>(len), q = dalloc<double>(len);
    DBuf dout, scratch, coef;
    auto precond = [&](const double *in, double *out) {
        if (F)
            ulv_solve(F, in, nrhs, out, s);
        else
            KRR_HIP(hipMemcpyAsync(out, in, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
    };
    int matvecs = 0;
    auto true_residual = [&]() {
        kernel_matvec_impl(Xp, n, Xp, n, d, xprec, h, alpha, nrhs, 0.0, q.as<double>(), mv_prec, s);
        ++matvecs;
        k_residual<<<ceil_div(len, 256), 256, 0, s>>>(Y, q.as<double>(), alpha, lambda, len, r.as<double>());
        check_launch("k_residual");
    };
    std::vector<double> ynorm = dots(Y, Y, n, nrhs, dout, scratch, s);
    for (auto &v : ynorm) v = std::sqrt(v) > 0 ? std::sqrt(v) : 1.0;
    true_residual();
    std::vector<double> rr = dots(r.as<double>(), r.as<double>(), n, nrhs, dout, scratch, s);
    auto rel = [&](const std::vector<double> &v) {
        std::vector<double> o(nrhs);
        for (int c = 0; c < nrhs; ++c) o[c] = std::sqrt(std::max(v[c], 0.0)) / ynorm[c];
        return o;
    };
    auto all_below = [&](const std::vector<double> &v) {
        for (double x : v)
            if (!(x <= tol)) return false;
        return true;
    };
    std::vector<double> relres = rel(rr);
    int it = 0;
    bool converged = all_below(relres);
    while (!converged && it < max_iter) {
        // (re)start: z = M^{-1} r, p = z
        precond(r.as<double>(), z.as<double>());
        KRR_HIP(hipMemcpyAsync(p.get(), z.get(), sizeof(double) * len, hipMemcpyDeviceToDevice, s));
        std::vector<double> rz = dots(r.as<double>(), z.as<double>(), n, nrhs, dout, scratch, s);
        std::vector<bool> done(nrhs);
        for (int c = 0; c < nrhs; ++c) done[c] = relres[c] <= tol;
        while (it < max_iter) {
            ++it;
            kernel_matvec_impl(Xp, n, Xp, n, d, xprec, h, p.as<double>(), nrhs, 0.0, q.as<double>(), mv_prec, s);
            ++matvecs;
            k_add_shift<<<ceil_div(len, 256), 256, 0, s>>>(q.as<double>(), p.as<double>(), lambda, len);
            check_launch("k_add_shift");
            std::vector<double> pq = dots(p.as<double>(), q.as<double>(), n, nrhs, dout, scratch, s);
            std::vector<double> a(nrhs), one(nrhs, 1.0), ma(nrhs);
            for (int c = 0; c < nrhs; ++c) {
                a[c] = (done[c] || pq[c] <= 0.0) ? 0.0 : rz[c] / pq[c];
                ma[c] = -a[c];
            }
            axpby(a, p.as<double>(), one, alpha, n, nrhs, coef, s);        // alpha += a p
            axpby(ma, q.as<double>(), one, r.as<double>(), n, nrhs, coef, s); // r -= a q
            rr = dots(r.as<double>(), r.as<double>(), n, nrhs, dout, scratch, s);
            std::vector<double> rec = rel(rr);
            if (verbose()) fprintf(stderr, "[krr] refine it=%d relres(recurrence)=%.3e\n", it, rec[0]);
            bool stop = true;
            for (int c = 0; c < nrhs; ++c) {
                if (rec[c] <= 0.5 * tol) done[c] = true;
                stop = stop && done[c];
            }
            if (stop) break;
            precond(r.as<double>(), z.as<double>());
            std::vector<double> rz2 = dots(r.as<double>(), z.as<double>(), n, nrhs, dout, scratch, s);
            std::vector<double> beta(nrhs);
            for (int c = 0; c < nrhs; ++c) {
                beta[c] = (done[c] || rz[c] == 0.0) ? 0.0 : rz2[c] / rz[c];
                rz[c] = rz2[c];
            }
            axpby(one, z.as<double>(), beta, p.as<double>(), n, nrhs, coef, s);  // p = z + beta p
        }
        // confirm on the true residual; restart from it if the recurrence drifted
        true_residual();
        rr = dots(r.as<double>(), r.as<double>(), n, nrhs, dout, scratch, s);
        relres = rel(rr);
        converged = all_below(relres);
        if (verbose()) fprintf(stderr, "[krr] refine it=%d true relres=%.3e\n", it, relres[0]);
    }
    if (st) {
        st->iterations = it;
        st->matvecs = matvecs;
        for (int c = 0; c < 64; ++c) st->relres[c] = c < nrhs ? relres[c] : 0.0;
        st->t_ms = timer.stop_ms();
    }
    sync(s);
    return converged ? KRR_OK : KRR_E_NOT_CONVERGED;
}

}  // namespace krr
