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

// Whether the machine, fed J at an OP_EVAL's point, asks next for the
// gradient there (at that evaluation's own fit and slot), so that a driver
// can start the gradient before J is back.  The machine's own decision is
// made as always from the J it is fed; the rule only restates it:
//   GRAD_ALWAYS     a start or polish evaluation;
//   GRAD_IF_ARMIJO  a line-search trial: J <= thr (accepted), unless extrap
//                   is set and the quadratic through phi(0) = phi,
//                   phi'(0) = gd and phi(t) = J has its minimiser beyond 2 t
//                   (then an extrapolated trial comes first);
//   GRAD_IF_BELOW   an extrapolated trial: J < thr (it is kept);
//   GRAD_NEVER      anything else.
enum { GRAD_NEVER = 0, GRAD_ALWAYS = 1, GRAD_IF_ARMIJO = 2, GRAD_IF_BELOW = 3 };
struct GradRule {
    int mode = GRAD_NEVER;
    int extrap = 0;
    double thr = 0.0, phi = 0.0, gd = 0.0, t = 0.0;
};

// Two projection buffers ("slots") per solve: OP_EVAL writes its projection
// to op.slot, OP_RESID and OP_GRAD read the projection in op.slot.  A line
// search that tries one more point after an accepted one keeps both, so the
// gradient can be taken at whichever of the two it accepts.
struct SolveOp {
    OpKind kind = OP_DONE;
    double w[PCAS_MAX_K] = {0};   // OP_EVAL: the point; OP_GRAD: the point of the slot
    bool fixed_ab = false;        // OP_EVAL / OP_RESID: (a, b) = ab instead of Eq. A.1
    double ab[2] = {1.0, 0.0};    // OP_EVAL fixed: (a, b); OP_GRAD: (a, b) of the residual
    int slot = 0;                 // projection buffer, 0 or 1
    GradRule next_grad;           // OP_EVAL: whether OP_GRAD at this point follows
};

// Relative rounding noise of an evaluated J, the band within which two
// values of J cannot be told apart.  fixed >= 0: that value.  Otherwise a
// model of the projection's rounding: each p_i carries an error of about
// u |p_i| (u the unit roundoff of the evaluation's type), which moves
// J = sum r_i^2 by about 2 u sqrt(sum r_i^2 p_i^2) ~ 2 u sqrt(J sum p_i^2 / M);
// the band is three of those.  At the fitted (a, b), sum p^2 = a^2 sum y^2 +
// 2 a b sum y + M b^2 + J exactly (the fit's normal equations make r
// orthogonal to y and to 1), so the band needs no extra pass.
struct NoiseModel {
    double fixed = -1.0;
    double u = 0.0, M = 1.0, sy = 0.0, syy = 0.0;
    double rel(double J, double a, double b) const {
        if (fixed >= 0.0) return fixed;
        if (!(J > 0.0)) return 0.0;
        const double sp2 = a * a * syy + 2.0 * a * b * sy + M * b * b + J;
        return 6.0 * u * sqrt(fmax(sp2, 0.0) / (M * J));
    }
};

class SolveMachine {
public:
    SolveMachine() = default;

    void start(const pcas_opts &o, int K, const NoiseModel &noise, const double *w0) {
        o_ = o;
        K_ = K;
        noise_ = noise;
        for (int k = 0; k < K; ++k) w_[k] = w0[k];
        memset(&rep_, 0, sizeof(rep_));
        rep_.locate_iters = -1;
        pc_ = o.method == 0 ? P_START : (o.method == 1 ? CG_START : QN_START);
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
    // Result of OP_GRAD; H (K x K, row-major, may be null): the Gauss-Newton
    // matrix of the reduced objective at the same point, which a
    // preconditioned CG (opts.precond) uses.
    void grad_result(const double *g, const double *H = nullptr) {
        for (int k = 0; k < K_; ++k) rg_[k] = g[k];
        rH_ok_ = H != nullptr;
        if (H)
            for (int i = 0; i < K_; ++i)
                for (int j = 0; j < K_; ++j) rH_[i * PCAS_MAX_K + j] = H[i * K_ + j];
        ++rep_.n_grads;
        run();
    }

    const double *w() const { return w_; }
    const pcas_report &report() const { return rep_; }

private:
    enum Pc {
        LS_TRIAL, LS_AFTER_TRIAL, LS_AFTER_EXTRAP,
        CG_START, CG_AFTER_EVAL0, CG_AFTER_GRAD0, CG_LOOP, CG_LS_END, CG_AFTER_GRAD,
        QN_START, QN_AFTER_EVAL0, QN_AFTER_GRAD0, QN_LOOP, QN_LS_END, QN_AFTER_GRAD,
        POLISH, POLISH_AFTER_EVAL, POLISH_AFTER_GRAD, SOLVE_FINISH,
        P_START, P_AFTER_EVAL0, P_LOOP, P_AFTER_RESID, P_GRAD, P_AFTER_GRAD, P_LS, P_AFTER_LS,
        P_END, P_AFTER_FINAL,
        FINISHED
    };

    static double dot(const double *a, const double *b, int K) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += a[k] * b[k];
        return s;
    }

    void want_eval(const double *w, bool fixed, double a, double b, Pc next, int slot = 0,
                   int grad = GRAD_NEVER) {
        op_.kind = OP_EVAL;
        op_.next_grad = GradRule{};
        op_.next_grad.mode = grad;
        for (int k = 0; k < K_; ++k) op_.w[k] = w[k];
        op_.fixed_ab = fixed;
        op_.ab[0] = a;
        op_.ab[1] = b;
        op_.slot = slot;
        pc_ = next;
    }
    void want_resid(Pc next) {
        op_.kind = OP_RESID;
        op_.fixed_ab = false;
        op_.slot = 0;
        pc_ = next;
    }
    void want_grad(const double *w, double a, double b, Pc next, int slot = 0) {
        op_.kind = OP_GRAD;
        for (int k = 0; k < K_; ++k) op_.w[k] = w[k];
        op_.ab[0] = a;
        op_.ab[1] = b;
        op_.slot = slot;
        pc_ = next;
    }
    // The inverse-Hessian estimate's update after an accepted step s with
    // gradient change y: scaled identity (y.s / y.y) at the first usable
    // pair, then the BFGS update expanded for symmetric H; a pair with
    // y.s <= 1e-12 |s| |y| is skipped.
    void hessian_update(double *H, bool &have, const double *sv, const double *yv) {
        const int K = K_;
        const double sy = dot(sv, yv, K), yy = dot(yv, yv, K);
        if (!(sy > 1e-12 * sqrt(dot(sv, sv, K)) * sqrt(yy))) return;
        if (!have) {
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) H[i * PCAS_MAX_K + j] = i == j ? sy / yy : 0.0;
            have = true;
        }
        const double rho = 1.0 / sy;
        double hy[PCAS_MAX_K];
        for (int i = 0; i < K; ++i) {
            double v = 0.0;
            for (int j = 0; j < K; ++j) v += H[i * PCAS_MAX_K + j] * yv[j];
            hy[i] = v;
        }
        const double c = rho + rho * rho * dot(yv, hy, K);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j)
                H[i * PCAS_MAX_K + j] += c * sv[i] * sv[j] - rho * (sv[i] * hy[j] + hy[i] * sv[j]);
    }
    // CG's curvature estimate after an accepted step: (y.y / y.s) I at the
    // first usable pair, then the direct BFGS update
    //   B+ = B - (B s)(B s)^T / (s.B s) + y y^T / (y.s);
    // a pair with y.s <= 1e-12 |s| |y| is skipped.
    void curvature_update(double *B, bool &have, const double *sv, const double *yv) {
        const int K = K_;
        const double sy = dot(sv, yv, K), yy = dot(yv, yv, K);
        if (!(sy > 1e-12 * sqrt(dot(sv, sv, K)) * sqrt(yy))) return;
        if (!have) {
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) B[i * PCAS_MAX_K + j] = i == j ? yy / sy : 0.0;
            have = true;
        }
        double bs[PCAS_MAX_K];
        for (int i = 0; i < K; ++i) {
            double v = 0.0;
            for (int j = 0; j < K; ++j) v += B[i * PCAS_MAX_K + j] * sv[j];
            bs[i] = v;
        }
        const double sbs = dot(sv, bs, K);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j)
                B[i * PCAS_MAX_K + j] += -bs[i] * bs[j] / sbs + yv[i] * yv[j] / sy;
    }
    // z = H^-1 g by the Cholesky factors of H (the preconditioner of CG);
    // false, with z = g, when H is missing or not positive definite.
    bool precondition(const double *H, bool ok, const double *g, double *z) const {
        const int K = K_;
        double L[PCAS_MAX_K * PCAS_MAX_K];
        for (int i = 0; ok && i < K; ++i)
            for (int j = 0; j <= i; ++j) {
                double s = H[i * PCAS_MAX_K + j];
                for (int k = 0; k < j; ++k) s -= L[i * PCAS_MAX_K + k] * L[j * PCAS_MAX_K + k];
                if (i == j) {
                    if (!(s > 0.0)) {
                        ok = false;
                        break;
                    }
                    L[i * PCAS_MAX_K + i] = sqrt(s);
                } else {
                    L[i * PCAS_MAX_K + j] = s / L[j * PCAS_MAX_K + j];
                }
            }
        if (!ok) {
            for (int k = 0; k < K; ++k) z[k] = g[k];
            return false;
        }
        double v[PCAS_MAX_K];
        for (int i = 0; i < K; ++i) {   // L v = g
            double s = g[i];
            for (int k = 0; k < i; ++k) s -= L[i * PCAS_MAX_K + k] * v[k];
            v[i] = s / L[i * PCAS_MAX_K + i];
        }
        for (int i = K - 1; i >= 0; --i) {   // L^T z = v
            double s = v[i];
            for (int k = i + 1; k < K; ++k) s -= L[k * PCAS_MAX_K + i] * z[k];
            z[i] = s / L[i * PCAS_MAX_K + i];
        }
        return true;
    }
    // d.B d (B applied first, then the dot with d).
    double quad_form(const double *B, const double *v) const {
        const int K = K_;
        double bv[PCAS_MAX_K];
        for (int i = 0; i < K; ++i) {
            double s = 0.0;
            for (int j = 0; j < K; ++j) s += B[i * PCAS_MAX_K + j] * v[j];
            bv[i] = s;
        }
        return dot(v, bv, K);
    }
    // A solve that stops at the noise floor (noise or decrement stop, failed
    // search) may take the polish step first.
    void end_at_floor(int status) {
        rep_.status = status;
        pc_ = o_.polish ? POLISH : SOLVE_FINISH;
    }

    // Line search along d_ from w_ (phi_ = J(w_), gd_ = g.d_ < 0, dn_ = ||d_||)
    // with first trial step t_; on return to `ret`, ls_ holds the outcome and,
    // when accepted, wt_ / phi_t_ / a_t_ / b_t_ / t_ the accepted point, whose
    // projection is in slot ls_slot_.
    enum LsOutcome { LS_OK, LS_NOISE, LS_FAIL };
    void line_search(Pc ret) {
        ls_ret_ = ret;
        bt_ = 0;
        pc_ = LS_TRIAL;
    }
    void ls_end(LsOutcome outcome, int slot) {
        ls_ = outcome;
        ls_slot_ = slot;
        pc_ = ls_ret_;
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
            // ---- line search shared by CG and BFGS -----------------------
            // Armijo trials; a rejected trial shrinks t to the minimiser of
            // the quadratic through phi(0), phi'(0), phi(t), kept within
            // [beta_lo t, beta t]; a rejected change below the noise floor
            // ends the solve.  An accepted first trial whose quadratic puts
            // the minimiser beyond 2t is followed by one trial there (capped
            // at ls_extrap t; backtracking alone cannot lengthen a step) and
            // the lower of the two points is kept.
            case LS_TRIAL:
                if (bt_ >= o_.max_backtracks || t_ * dn_ < o_.xtol) {
                    ls_end(LS_FAIL, 0);
                    break;
                }
                for (int k = 0; k < K; ++k) wt_[k] = w_[k] + t_ * d_[k];
                thr_ = phi_ + o_.alpha * t_ * gd_;
                want_eval(wt_, false, 1.0, 0.0, LS_AFTER_TRIAL, 0, GRAD_IF_ARMIJO);
                op_.next_grad.extrap = bt_ == 0 && o_.ls_extrap > 0.0;
                op_.next_grad.thr = thr_;
                op_.next_grad.phi = phi_;
                op_.next_grad.gd = gd_;
                op_.next_grad.t = t_;
                return;
            case LS_AFTER_TRIAL: {
                phi_t_ = rJ_;
                a_t_ = ra_;
                b_t_ = rb_;
                const double tq = -gd_ * t_ * t_ / (2.0 * (phi_t_ - phi_ - gd_ * t_));
                if (phi_t_ <= thr_) {
                    if (bt_ == 0 && o_.ls_extrap > 0.0 && tq > 2.0 * t_) {
                        tx_ = tq < o_.ls_extrap * t_ ? tq : o_.ls_extrap * t_;
                        for (int k = 0; k < K; ++k) wx_[k] = w_[k] + tx_ * d_[k];
                        want_eval(wx_, false, 1.0, 0.0, LS_AFTER_EXTRAP, 1, GRAD_IF_BELOW);
                        op_.next_grad.thr = phi_t_;
                        return;
                    }
                    ls_end(LS_OK, 0);
                    break;
                }
                if (fabs(phi_t_ - phi_) <= nu_ * phi_) {   // below the objective's noise
                    ls_end(LS_NOISE, 0);
                    break;
                }
                const double lo = o_.beta_lo * t_, hi = o_.beta * t_;
                t_ = tq < lo ? lo : (tq > hi ? hi : tq);
                ++bt_;
                pc_ = LS_TRIAL;
                break;
            }
            case LS_AFTER_EXTRAP:
                if (rJ_ < phi_t_) {
                    t_ = tx_;
                    for (int k = 0; k < K; ++k) wt_[k] = wx_[k];
                    phi_t_ = rJ_;
                    a_t_ = ra_;
                    b_t_ = rb_;
                    ls_end(LS_OK, 1);
                } else {
                    ls_end(LS_OK, 0);
                }
                break;

            // ---- PR+ nonlinear CG on the reduced objective ----------------
            // PR+ directions, each searched by the line search above from the
            // minimiser of the quadratic model along d.  The model's
            // curvature is a Hessian estimate B built from the accepted steps
            // by direct BFGS updates (used for step lengths only; the
            // directions stay CG's).  A predicted decrease within the noise
            // floor ends the solve when the model is trusted, as in BFGS.
            // Preconditioned (opts.precond, Nocedal and Wright Sec. 5.1 and
            // the PR+ rule with preconditioned inner products): each gradient
            // comes with the Gauss-Newton matrix H of its point; directions
            // are -z + beta d with z = H^-1 g and beta = max(0, z+.(g+ - g) /
            // (z.g)), and H is the model of the first trial and of the stop.
            case CG_START:
                want_eval(w_, false, 1.0, 0.0, CG_AFTER_EVAL0, 0, GRAD_ALWAYS);
                return;
            case CG_AFTER_EVAL0:
                phi_ = rJ_;
                a_ = ra_;
                b_ = rb_;
                nu_ = noise_.rel(phi_, a_, b_);
                want_grad(w_, a_, b_, CG_AFTER_GRAD0);
                return;
            case CG_AFTER_GRAD0:
                for (int k = 0; k < K; ++k) g_[k] = rg_[k];
                pre_ = o_.precond != 0;
                if (pre_) {
                    memcpy(Hg_, rH_, sizeof(Hg_));
                    have_hg_ = precondition(Hg_, rH_ok_, g_, z_);
                }
                for (int k = 0; k < K; ++k) d_[k] = pre_ ? -z_[k] : -g_[k];
                rep_.J0 = phi_;
                g0_ = sqrt(dot(g_, g_, K));
                rep_.gnorm0 = g0_;
                restart_ = first_ = true;
                t_prev_ = gd_prev_ = 0.0;
                curv_ = 0.0;
                have_hc_ = have_h_ = have_b_ = false;
                last_drop_ = INFINITY;
                last_pred_ = -1.0;
                it_ = 0;
                rep_.status = PCAS_STOP_MAXITER;
                pc_ = CG_LOOP;
                break;
            case CG_LOOP: {
                if (it_ >= o_.max_iter) {
                    pc_ = SOLVE_FINISH;
                    break;
                }
                const double gn = sqrt(dot(g_, g_, K));
                if (gn <= o_.gtol_rel * g0_ || phi_ == 0.0) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    pc_ = SOLVE_FINISH;
                    break;
                }
                gd_ = dot(g_, d_, K);
                if (gd_ >= 0.0) {
                    if (pre_ && have_hg_) {   // restart along the preconditioned gradient
                        for (int k = 0; k < K; ++k) d_[k] = -z_[k];
                        gd_ = -dot(g_, z_, K);
                    } else {
                        for (int k = 0; k < K; ++k) d_[k] = -g_[k];
                        gd_ = -gn * gn;
                    }
                    restart_ = true;
                }
                dn_ = sqrt(dot(d_, d_, K));
                // first trial: the quadratic model's minimiser along d with the
                // curvature estimate B, -(g.d) / (d.B d); before B exists,
                // mu0 / ||d|| first, then with the curvature the last accepted
                // step measured, (s.y) / (s.s)
                {
                    // preconditioned: the Gauss-Newton matrix at this point is the model
                    const double dbd = pre_ && have_hg_ ? quad_form(Hg_, d_)
                                                        : (have_b_ ? quad_form(B_, d_) : 0.0);
                    pred_ = -1.0;
                    if (dbd > 0.0) {
                        t_ = -gd_ / dbd;
                        pred_ = -0.5 * gd_ * t_;
                        // the model's decrease below the noise, and the model
                        // trusted (as in BFGS): stop
                        if (pred_ <= nu_ * phi_ &&
                            (last_drop_ <= nu_ * phi_ ||
                             (0.5 * last_pred_ <= last_drop_ && last_drop_ <= 2.0 * last_pred_))) {
                            end_at_floor(PCAS_STOP_CONVERGED);
                            break;
                        }
                    } else if (first_) {
                        t_ = o_.mu0 / dn_;
                    } else if (curv_ > 0.0) {
                        t_ = -gd_ / (curv_ * dn_ * dn_);
                    } else {
                        t_ = t_prev_ * gd_prev_ / gd_;
                    }
                }
                t0_ = t_;
                line_search(CG_LS_END);
                break;
            }
            case CG_LS_END:
                if (ls_ == LS_NOISE) {
                    end_at_floor(PCAS_STOP_CONVERGED);
                    break;
                }
                if (ls_ == LS_FAIL) {
                    if (restart_) {
                        end_at_floor(PCAS_STOP_LINESEARCH);
                        break;
                    }
                    for (int k = 0; k < K; ++k) d_[k] = -g_[k];
                    restart_ = true;
                    pc_ = CG_LOOP;
                    break;
                }
                for (int k = 0; k < K; ++k) {
                    wprev_[k] = w_[k];
                    w_[k] = wt_[k];
                }
                last_pred_ = t_ == t0_ ? pred_ : -1.0;
                last_drop_ = phi_ - phi_t_;
                phi_ = phi_t_;
                a_ = a_t_;
                b_ = b_t_;
                nu_ = noise_.rel(phi_, a_, b_);
                want_grad(w_, a_, b_, CG_AFTER_GRAD, ls_slot_);
                return;
            case CG_AFTER_GRAD: {
                {
                    double sv[PCAS_MAX_K], yv[PCAS_MAX_K];
                    for (int k = 0; k < K; ++k) {
                        sv[k] = w_[k] - wprev_[k];
                        yv[k] = rg_[k] - g_[k];
                    }
                    const double ss = dot(sv, sv, K);
                    curv_ = ss > 0.0 ? dot(sv, yv, K) / ss : 0.0;
                    curvature_update(B_, have_b_, sv, yv);
                    if (o_.polish) hessian_update(Hc_, have_hc_, sv, yv);   // polish only
                }
                if (pre_) {
                    // preconditioned PR+: z = H^-1 g with the new point's
                    // Gauss-Newton matrix, beta = z+.(g+ - g) / (z.g)
                    double zn[PCAS_MAX_K];
                    const double zg = dot(z_, g_, K);
                    memcpy(Hg_, rH_, sizeof(Hg_));
                    have_hg_ = precondition(Hg_, rH_ok_, rg_, zn);
                    double num = 0.0;
                    for (int k = 0; k < K; ++k) num += zn[k] * (rg_[k] - g_[k]);
                    double beta_pr = zg > 0.0 ? num / zg : 0.0;
                    beta_pr = beta_pr > 0.0 ? beta_pr : 0.0;
                    for (int k = 0; k < K; ++k) {
                        d_[k] = -zn[k] + beta_pr * d_[k];
                        g_[k] = rg_[k];
                        z_[k] = zn[k];
                    }
                } else {
                    double num = 0.0;
                    for (int k = 0; k < K; ++k) num += rg_[k] * (rg_[k] - g_[k]);
                    double beta_pr = num / dot(g_, g_, K);
                    beta_pr = beta_pr > 0.0 ? beta_pr : 0.0;
                    for (int k = 0; k < K; ++k) {
                        d_[k] = -rg_[k] + beta_pr * d_[k];
                        g_[k] = rg_[k];
                    }
                }
                t_prev_ = t_;
                gd_prev_ = gd_;
                restart_ = false;
                first_ = false;
                ++it_;
                pc_ = CG_LOOP;
                break;
            }

            // ---- BFGS on the reduced objective ------------------------------
            // d = -H g with unit first trial; -g with mu0/||g|| while there is
            // no estimate.  H starts as (y.s / y.y) I at the first accepted
            // step, then takes the inverse BFGS update
            //   H+ = (I - rho s y^T) H (I - rho y s^T) + rho s s^T, rho = 1/(y.s),
            // expanded for symmetric H; an update with y.s <= 1e-12 |s| |y| is
            // skipped.  A failed search drops the estimate and retries along
            // -g; a failed search along -g ends the solve.  With an estimate,
            // a predicted decrease g.H g / 2 within the noise floor ends the
            // solve as converged when the model is trusted: the last step's
            // decrease was within the floor too, or (unit step) within a
            // factor 2 of its prediction (H can still underestimate flat
            // directions).
            case QN_START:
                want_eval(w_, false, 1.0, 0.0, QN_AFTER_EVAL0, 0, GRAD_ALWAYS);
                return;
            case QN_AFTER_EVAL0:
                phi_ = rJ_;
                a_ = ra_;
                b_ = rb_;
                nu_ = noise_.rel(phi_, a_, b_);
                want_grad(w_, a_, b_, QN_AFTER_GRAD0);
                return;
            case QN_AFTER_GRAD0:
                for (int k = 0; k < K; ++k) g_[k] = rg_[k];
                rep_.J0 = phi_;
                g0_ = sqrt(dot(g_, g_, K));
                rep_.gnorm0 = g0_;
                have_h_ = have_hc_ = false;
                last_drop_ = INFINITY;
                last_pred_ = -1.0;
                it_ = 0;
                rep_.status = PCAS_STOP_MAXITER;
                pc_ = QN_LOOP;
                break;
            case QN_LOOP: {
                if (it_ >= o_.max_iter) {
                    pc_ = SOLVE_FINISH;
                    break;
                }
                const double gn = sqrt(dot(g_, g_, K));
                if (gn <= o_.gtol_rel * g0_ || phi_ == 0.0) {
                    rep_.status = PCAS_STOP_CONVERGED;
                    pc_ = SOLVE_FINISH;
                    break;
                }
                if (have_h_) {
                    for (int i = 0; i < K; ++i) {
                        double v = 0.0;
                        for (int j = 0; j < K; ++j) v += H_[i * PCAS_MAX_K + j] * g_[j];
                        d_[i] = -v;
                    }
                    gd_ = dot(g_, d_, K);
                    t_ = 1.0;
                    if (gd_ >= 0.0) {
                        have_h_ = false;   // the estimate lost definiteness
                    } else if (-0.5 * gd_ <= nu_ * phi_ &&
                               (last_drop_ <= nu_ * phi_ ||
                                (0.5 * last_pred_ <= last_drop_ && last_drop_ <= 2.0 * last_pred_))) {
                        // the model's predicted decrease g.H g / 2 is below the
                        // noise, and the model is trusted (the last step's
                        // decrease was below the noise, or within a factor 2
                        // of what the model predicted for it)
                        end_at_floor(PCAS_STOP_CONVERGED);
                        break;
                    }
                }
                if (!have_h_) {
                    for (int k = 0; k < K; ++k) d_[k] = -g_[k];
                    gd_ = -gn * gn;
                    t_ = o_.mu0 / gn;
                }
                dn_ = sqrt(dot(d_, d_, K));
                line_search(QN_LS_END);
                break;
            }
            case QN_LS_END:
                if (ls_ == LS_NOISE) {
                    end_at_floor(PCAS_STOP_CONVERGED);
                    break;
                }
                if (ls_ == LS_FAIL) {
                    if (!have_h_) {
                        end_at_floor(PCAS_STOP_LINESEARCH);
                        break;
                    }
                    // keep the estimate for a polish step, then retry along -g
                    memcpy(Hc_, H_, sizeof(H_));
                    have_hc_ = true;
                    have_h_ = false;
                    pc_ = QN_LOOP;
                    break;
                }
                want_grad(wt_, a_t_, b_t_, QN_AFTER_GRAD, ls_slot_);
                return;
            case QN_AFTER_GRAD: {
                double sv[PCAS_MAX_K], yv[PCAS_MAX_K];
                for (int k = 0; k < K; ++k) {
                    sv[k] = wt_[k] - w_[k];
                    yv[k] = rg_[k] - g_[k];
                }
                // the model's decrease at the accepted step, for a unit
                // quasi-Newton step (phi(w + d) ~ phi + g.d - g.d / 2)
                last_pred_ = (have_h_ && t_ == 1.0) ? -0.5 * gd_ : -1.0;
                hessian_update(H_, have_h_, sv, yv);
                last_drop_ = phi_ - phi_t_;
                for (int k = 0; k < K; ++k) {
                    w_[k] = wt_[k];
                    g_[k] = rg_[k];
                }
                phi_ = phi_t_;
                a_ = a_t_;
                b_ = b_t_;
                nu_ = noise_.rel(phi_, a_, b_);
                ++it_;
                pc_ = QN_LOOP;
                break;
            }

            // ---- polish: one step w - H g at the noise floor ----------------
            // H: BFGS's estimate (or its last one), or CG's from its steps.
            // The step is kept if ||g|| drops; the gradient resolves the
            // minimiser far below the noise of J.
            case POLISH: {
                // preconditioned CG: the Gauss-Newton step H^-1 g at the point
                const bool gn = o_.method == 1 && pre_ && have_hg_;
                const double *H = o_.method == 2 && have_h_ ? H_ : (have_hc_ ? Hc_ : nullptr);
                if (!H && !gn) {
                    pc_ = SOLVE_FINISH;
                    break;
                }
                double gd = 0.0;
                for (int i = 0; i < K; ++i) {
                    double v = 0.0;
                    if (gn) {
                        v = z_[i];
                    } else {
                        for (int j = 0; j < K; ++j) v += H[i * PCAS_MAX_K + j] * g_[j];
                    }
                    wx_[i] = w_[i] - v;
                    gd -= g_[i] * v;
                }
                if (!(gd < 0.0)) {
                    pc_ = SOLVE_FINISH;
                    break;
                }
                want_eval(wx_, false, 1.0, 0.0, POLISH_AFTER_EVAL, 1, GRAD_ALWAYS);
                return;
            }
            case POLISH_AFTER_EVAL:
                phi_t_ = rJ_;
                a_t_ = ra_;
                b_t_ = rb_;
                want_grad(wx_, a_t_, b_t_, POLISH_AFTER_GRAD, 1);
                return;
            case POLISH_AFTER_GRAD:
                if (dot(rg_, rg_, K) < dot(g_, g_, K)) {
                    for (int k = 0; k < K; ++k) {
                        w_[k] = wx_[k];
                        g_[k] = rg_[k];
                    }
                    phi_ = phi_t_;
                    a_ = a_t_;
                    b_ = b_t_;
                }
                pc_ = SOLVE_FINISH;
                break;

            case SOLVE_FINISH:
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
    NoiseModel noise_;
    double nu_ = 0.0;   // noise band of J at the current point (relative)
    Pc pc_ = FINISHED;
    SolveOp op_;
    pcas_report rep_{};
    // results of the last operation
    double rJ_ = 0.0, ra_ = 0.0, rb_ = 0.0, rg_[PCAS_MAX_K] = {0};
    double rH_[PCAS_MAX_K * PCAS_MAX_K] = {0};   // Gauss-Newton matrix with rg_ (row-major)
    bool rH_ok_ = false;
    // solver state
    double w_[PCAS_MAX_K] = {0}, wt_[PCAS_MAX_K] = {0}, wx_[PCAS_MAX_K] = {0};
    double wprev_[PCAS_MAX_K] = {0};
    double g_[PCAS_MAX_K] = {0}, d_[PCAS_MAX_K] = {0};
    double H_[PCAS_MAX_K * PCAS_MAX_K] = {0};   // BFGS inverse-Hessian estimate (row-major)
    double B_[PCAS_MAX_K * PCAS_MAX_K] = {0};   // CG: Hessian (curvature) estimate (row-major)
    double Hc_[PCAS_MAX_K * PCAS_MAX_K] = {0};  // estimate kept for the polish step
    // preconditioned CG: the Gauss-Newton matrix at w_ and z = H^-1 g there
    double Hg_[PCAS_MAX_K * PCAS_MAX_K] = {0}, z_[PCAS_MAX_K] = {0};
    bool pre_ = false, have_hg_ = false;
    double phi_ = 0.0, a_ = 0.0, b_ = 0.0, phi_t_ = 0.0, a_t_ = 0.0, b_t_ = 0.0;
    double g0_ = 0.0, gd_ = 0.0, dn_ = 0.0, t_ = 0.0, tx_ = 0.0, t_prev_ = 0.0, gd_prev_ = 0.0;
    double thr_ = 0.0;    // Armijo threshold of the current trial
    double curv_ = 0.0;   // CG: (s.y) / (s.s) of the last accepted step
    double t0_ = 0.0, pred_ = -1.0;   // CG: first trial step, the model's decrease for it
    double last_drop_ = 0.0;   // CG, BFGS: J decrease of the last accepted step
    double last_pred_ = -1.0;  // CG, BFGS: the model's prediction of it (< 0: none)
    double J_ = 0.0, gn_ = 0.0, mu_ = 0.0;
    bool restart_ = true, first_ = true, have_h_ = false, have_hc_ = false, have_b_ = false;
    int it_ = 0, bt_ = 0, ls_slot_ = 0;
    LsOutcome ls_ = LS_FAIL;
    Pc ls_ret_ = FINISHED;
};

}  // namespace pcas
