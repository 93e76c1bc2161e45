// Host-side solver of the per-projection problem as a resumable state
// machine.  It never touches the GPU: it asks for one operation at a time
// (an evaluation of J at a point, a residual of the last evaluated
// projection, a gradient at the last evaluated point) and is fed the
// results.  solve_projection drives one machine synchronously; the serving
// loop drives many, batching the operations of all of them into shared
// launches.  Given the same results, a machine takes the same steps, so a
// request's answer does not depend on what else is in flight.
#pragma once

#include <math.h>
#include <string.h>

#include "pcasolve.h"

namespace pcas {

enum OpKind { OP_EVAL = 0, OP_RESID = 1, OP_GRAD = 2, OP_DONE = 3 };

struct SolveOp {
    OpKind kind = OP_DONE;
    double w[PCAS_MAX_K] = {0};   // OP_EVAL: the point; OP_GRAD: the point (last evaluated)
    bool fixed_ab = false;        // OP_EVAL / OP_RESID: (a, b) = ab instead of Eq. A.1
    double ab[2] = {1.0, 0.0};    // OP_EVAL fixed: (a, b); OP_GRAD: (a, b) of the residual
};

class SolveMachine {
public:
    SolveMachine() = default;

    // ftol: noise-floor threshold (opts.ftol_rel, with < 0 resolved by the
    // caller for the dtype).
    void start(const pcas_opts &o, int K, double ftol, const double *w0) {
        o_ = o;
        K_ = K;
        ftol_ = ftol;
        for (int k = 0; k < K; ++k) w_[k] = w0[k];
        memset(&rep_, 0, sizeof(rep_));
        rep_.locate_iters = -1;
        pc_ = o.method == 0 ? P_START : CG_START;
        run();
    }

    const SolveOp &op() const { return op_; }
    bool done() const { return op_.kind == OP_DONE; }

    // Result of OP_EVAL or OP_RESID.
    void eval_result(double J, double a, double b) {
        rJ_ = J;
        ra_ = a;
        rb_ = b;
        if (op_.kind == OP_EVAL) ++rep_.n_fevals;
        run();
    }
    // Result of OP_GRAD.
    void grad_result(const double *g) {
        for (int k = 0; k < K_; ++k) rg_[k] = g[k];
        ++rep_.n_grads;
        run();
    }

    const double *w() const { return w_; }
    const pcas_report &report() const { return rep_; }

private:
    enum Pc {
        CG_START, CG_AFTER_EVAL0, CG_AFTER_GRAD0, CG_LOOP, CG_LS, CG_AFTER_LS_EVAL, CG_LS_END,
        CG_AFTER_GRAD, CG_FINISH,
        P_START, P_AFTER_EVAL0, P_LOOP, P_AFTER_RESID, P_GRAD, P_AFTER_GRAD, P_LS, P_AFTER_LS,
        P_END, P_AFTER_FINAL,
        FINISHED
    };

    static double dot(const double *a, const double *b, int K) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += a[k] * b[k];
        return s;
    }

    void want_eval(const double *w, bool fixed, double a, double b, Pc next) {
        op_.kind = OP_EVAL;
        for (int k = 0; k < K_; ++k) op_.w[k] = w[k];
        op_.fixed_ab = fixed;
        op_.ab[0] = a;
        op_.ab[1] = b;
        pc_ = next;
    }
    void want_resid(Pc next) {
        op_.kind = OP_RESID;
        op_.fixed_ab = false;
        pc_ = next;
    }
    void want_grad(const double *w, double a, double b, Pc next) {
        op_.kind = OP_GRAD;
        for (int k = 0; k < K_; ++k) op_.w[k] = w[k];
        op_.ab[0] = a;
        op_.ab[1] = b;
        pc_ = next;
    }
    void finish() {
        op_.kind = OP_DONE;
        pc_ = FINISHED;
    }

    // Runs until the next operation is needed (or the solve ends).
    void run() {
        const int K = K_;
        for (;;) {
            switch (pc_) {
            // ---- PR+ nonlinear CG on the reduced objective ----------------
            case CG_START:
                want_eval(w_, false, 1.0, 0.0, CG_AFTER_EVAL0);
                return;
            case CG_AFTER_EVAL0:
                phi_ = rJ_;
                a_ = ra_;
                b_ = rb_;
                want_grad(w_, a_, b_, CG_AFTER_GRAD0);
                return;
            case CG_AFTER_GRAD0:
                for (int k = 0; k < K; ++k) {
                    g_[k] = rg_[k];
                    d_[k] = -g_[k];
                }
                rep_.J0 = phi_;
                g0_ = sqrt(dot(g_, g_, K));
                rep_.gnorm0 = g0_;
                restart_ = first_ = true;
                t_prev_ = gd_prev_ = 0.0;
                it_ = 0;
                rep_.status = PCAS_STOP_MAXITER;
                pc_ = CG_LOOP;
                break;
            case CG_LOOP: {
                if (it_ >= o_.max_iter) {
                    pc_ = CG_FINISH;
                    break;
                }
                const double gn = sqrt(dot(g_, g_, K));
                if (gn <= o_.gtol_rel * g0_ || phi_ == 0.0) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    pc_ = CG_FINISH;
                    break;
                }
                gd_ = dot(g_, d_, K);
                if (gd_ >= 0.0) {
                    for (int k = 0; k < K; ++k) d_[k] = -g_[k];
                    gd_ = -gn * gn;
                    restart_ = true;
                }
                dn_ = sqrt(dot(d_, d_, K));
                t_ = first_ ? o_.mu0 / dn_ : t_prev_ * gd_prev_ / gd_;
                accepted_ = at_noise_ = false;
                bt_ = 0;
                pc_ = CG_LS;
                break;
            }
            case CG_LS:
                if (bt_ >= o_.max_backtracks || t_ * dn_ < o_.xtol) {
                    pc_ = CG_LS_END;
                    break;
                }
                for (int k = 0; k < K; ++k) wt_[k] = w_[k] + t_ * d_[k];
                want_eval(wt_, false, 1.0, 0.0, CG_AFTER_LS_EVAL);
                return;
            case CG_AFTER_LS_EVAL: {
                phi_t_ = rJ_;
                a_t_ = ra_;
                b_t_ = rb_;
                if (phi_t_ <= phi_ + o_.alpha * t_ * gd_) {
                    accepted_ = true;
                    pc_ = CG_LS_END;
                    break;
                }
                if (fabs(phi_t_ - phi_) <= ftol_ * phi_) {   // below the objective's noise
                    at_noise_ = true;
                    pc_ = CG_LS_END;
                    break;
                }
                const double tq = -gd_ * t_ * t_ / (2.0 * (phi_t_ - phi_ - gd_ * t_));
                const double lo = o_.beta_lo * t_, hi = o_.beta * t_;
                t_ = tq < lo ? lo : (tq > hi ? hi : tq);
                ++bt_;
                pc_ = CG_LS;
                break;
            }
            case CG_LS_END:
                if (at_noise_) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    pc_ = CG_FINISH;
                    break;
                }
                if (!accepted_) {
                    if (restart_) {
                        rep_.status = PCAS_STOP_LINESEARCH;
                        pc_ = CG_FINISH;
                        break;
                    }
                    for (int k = 0; k < K; ++k) d_[k] = -g_[k];
                    restart_ = true;
                    pc_ = CG_LOOP;
                    break;
                }
                for (int k = 0; k < K; ++k) w_[k] = wt_[k];
                phi_ = phi_t_;
                a_ = a_t_;
                b_ = b_t_;
                want_grad(w_, a_, b_, CG_AFTER_GRAD);
                return;
            case CG_AFTER_GRAD: {
                double num = 0.0;
                for (int k = 0; k < K; ++k) num += rg_[k] * (rg_[k] - g_[k]);
                double beta_pr = num / dot(g_, g_, K);
                beta_pr = beta_pr > 0.0 ? beta_pr : 0.0;
                for (int k = 0; k < K; ++k) {
                    d_[k] = -rg_[k] + beta_pr * d_[k];
                    g_[k] = rg_[k];
                }
                t_prev_ = t_;
                gd_prev_ = gd_;
                restart_ = false;
                first_ = false;
                ++it_;
                pc_ = CG_LOOP;
                break;
            }
            case CG_FINISH:
                rep_.iters = it_;
                rep_.J = phi_;
                rep_.a = a_;
                rep_.b = b_;
                rep_.gnorm = sqrt(dot(g_, g_, K));
                finish();
                return;

            // ---- the Appendix algorithm: Eq. A.1, Eq. A.2, Armijo -----------
            case P_START:
                want_eval(w_, false, 1.0, 0.0, P_AFTER_EVAL0);   // step 1 at w0
                return;
            case P_AFTER_EVAL0:
                J_ = rJ_;
                a_ = ra_;
                b_ = rb_;
                rep_.J0 = J_;
                rep_.status = PCAS_STOP_MAXITER;
                it_ = 0;
                pc_ = P_LOOP;
                break;
            case P_LOOP:
                if (it_ >= o_.max_iter) {
                    pc_ = P_END;
                    break;
                }
                if (it_ > 0) {
                    want_resid(P_AFTER_RESID);   // step 1 at the accepted point
                    return;
                }
                pc_ = P_GRAD;
                break;
            case P_AFTER_RESID:
                J_ = rJ_;
                a_ = ra_;
                b_ = rb_;
                pc_ = P_GRAD;
                break;
            case P_GRAD:
                rep_.J = J_;
                rep_.a = a_;
                rep_.b = b_;
                want_grad(w_, a_, b_, P_AFTER_GRAD);
                return;
            case P_AFTER_GRAD: {
                const double gn = sqrt(dot(rg_, rg_, K));
                if (it_ == 0) rep_.gnorm0 = gn;
                rep_.gnorm = gn;
                if (gn == 0.0 || J_ == 0.0) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    finish();
                    return;
                }
                gn_ = gn;
                for (int k = 0; k < K; ++k) d_[k] = rg_[k] / gn;   // step 2
                mu_ = o_.mu0;
                pc_ = P_LS;
                break;
            }
            case P_LS:
                for (int k = 0; k < K; ++k) wt_[k] = w_[k] - mu_ * d_[k];
                want_eval(wt_, true, a_, b_, P_AFTER_LS);
                return;
            case P_AFTER_LS:
                if (rJ_ <= J_ - o_.alpha * mu_ * gn_) {
                    for (int k = 0; k < K; ++k) w_[k] = wt_[k];
                    rep_.iters = it_ + 1;
                    ++it_;
                    pc_ = P_LOOP;
                    break;
                }
                mu_ *= o_.beta;
                if (mu_ < o_.mu_min) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    finish();
                    return;
                }
                pc_ = P_LS;
                break;
            case P_END:
                if (o_.max_iter > 0) {
                    want_resid(P_AFTER_FINAL);
                    return;
                }
                finish();
                return;
            case P_AFTER_FINAL:
                rep_.a = ra_;
                rep_.b = rb_;
                rep_.J = rJ_;
                finish();
                return;
            case FINISHED:
                return;
            }
        }
    }

    pcas_opts o_{};
    int K_ = 0;
    double ftol_ = 0.0;
    Pc pc_ = FINISHED;
    SolveOp op_;
    pcas_report rep_{};
    // results of the last operation
    double rJ_ = 0.0, ra_ = 0.0, rb_ = 0.0, rg_[PCAS_MAX_K] = {0};
    // solver state
    double w_[PCAS_MAX_K] = {0}, wt_[PCAS_MAX_K] = {0}, g_[PCAS_MAX_K] = {0}, d_[PCAS_MAX_K] = {0};
    double phi_ = 0.0, a_ = 0.0, b_ = 0.0, phi_t_ = 0.0, a_t_ = 0.0, b_t_ = 0.0;
    double g0_ = 0.0, gd_ = 0.0, dn_ = 0.0, t_ = 0.0, t_prev_ = 0.0, gd_prev_ = 0.0;
    double J_ = 0.0, gn_ = 0.0, mu_ = 0.0;
    bool restart_ = true, first_ = true, accepted_ = false, at_noise_ = false;
    int it_ = 0, bt_ = 0;
};

}  // namespace pcas
