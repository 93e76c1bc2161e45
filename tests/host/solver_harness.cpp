// CPU harness for the host-side solver state machine: drives one
// SolveMachine with callbacks in place of GPU evaluations, so its iterates
// can be compared with an independent implementation on the CPU.  Test
// infrastructure only; built with g++ by the host-logic tests.
#include "solver.h"

extern "C" {

// J, (a, b) at w; the callee records which point now occupies `slot`.
typedef double (*harness_eval_fn)(const double *w, int slot, int fixed_ab, const double *ab,
                                  double *a, double *b);
// g at w from the projection in `slot` (the callee checks that slot holds w).
typedef void (*harness_grad_fn)(const double *w, int slot, double a, double b, double *g);

int harness_solve(const pcas_opts *opts, int K, double ftol, const double *w0,
                  harness_eval_fn ev, harness_grad_fn gr, double *w_out, pcas_report *rep) {
    pcas::SolveMachine m;
    pcas::NoiseModel noise;
    noise.fixed = ftol;
    m.start(*opts, K, noise, w0);
    int guard = 0;
    while (!m.done()) {
        if (++guard > 100000) return -1;
        const pcas::SolveOp &op = m.op();
        if (op.kind == pcas::OP_EVAL || op.kind == pcas::OP_RESID) {
            double a = 1.0, b = 0.0;
            const double J = ev(op.kind == pcas::OP_EVAL ? op.w : nullptr, op.slot,
                                op.fixed_ab ? 1 : 0, op.ab, &a, &b);
            m.eval_result(J, a, b);
        } else {
            double g[PCAS_MAX_K];
            gr(op.w, op.slot, op.ab[0], op.ab[1], g);
            m.grad_result(g);
        }
    }
    for (int k = 0; k < K; ++k) w_out[k] = m.w()[k];
    *rep = m.report();
    return 0;
}

// The same drive, reporting for every OP_EVAL the gradient rule the machine
// stated with it, the J it was fed, and whether the machine's next request
// was the gradient at that very point, fit and slot.
typedef void (*harness_rule_fn)(int mode, int extrap, double thr, double phi, double gd, double t,
                                double J, int grad_next);

int harness_solve_rules(const pcas_opts *opts, int K, double ftol, const double *w0,
                        harness_eval_fn ev, harness_grad_fn gr, harness_rule_fn rule,
                        double *w_out, pcas_report *rep) {
    pcas::SolveMachine m;
    pcas::NoiseModel noise;
    noise.fixed = ftol;
    m.start(*opts, K, noise, w0);
    int guard = 0;
    while (!m.done()) {
        if (++guard > 100000) return -1;
        const pcas::SolveOp op = m.op();   // a copy: the machine moves on
        if (op.kind == pcas::OP_EVAL || op.kind == pcas::OP_RESID) {
            double a = 1.0, b = 0.0;
            const double J = ev(op.kind == pcas::OP_EVAL ? op.w : nullptr, op.slot,
                                op.fixed_ab ? 1 : 0, op.ab, &a, &b);
            m.eval_result(J, a, b);
            if (op.kind == pcas::OP_EVAL) {
                const pcas::SolveOp &nx = m.op();
                const int next = nx.kind == pcas::OP_GRAD && nx.slot == op.slot &&
                                 !memcmp(nx.w, op.w, K * sizeof(double)) &&
                                 !memcmp(&nx.ab[0], &a, sizeof(a)) && !memcmp(&nx.ab[1], &b, sizeof(b));
                const pcas::GradRule &r = op.next_grad;
                rule(r.mode, r.extrap, r.thr, r.phi, r.gd, r.t, J, next);
            }
        } else {
            double g[PCAS_MAX_K];
            gr(op.w, op.slot, op.ab[0], op.ab[1], g);
            m.grad_result(g);
        }
    }
    for (int k = 0; k < K; ++k) w_out[k] = m.w()[k];
    *rep = m.report();
    return 0;
}

// The same drive with a gradient callback that may also return the
// Gauss-Newton matrix at the point (K x K, row-major; return value 1 when
// it did), for the preconditioned CG.
typedef int (*harness_grad_gn_fn)(const double *w, int slot, double a, double b, double *g,
                                  double *H);

int harness_solve_gn(const pcas_opts *opts, int K, double ftol, const double *w0,
                     harness_eval_fn ev, harness_grad_gn_fn gr, double *w_out, pcas_report *rep) {
    pcas::SolveMachine m;
    pcas::NoiseModel noise;
    noise.fixed = ftol;
    m.start(*opts, K, noise, w0);
    int guard = 0;
    while (!m.done()) {
        if (++guard > 100000) return -1;
        const pcas::SolveOp &op = m.op();
        if (op.kind == pcas::OP_EVAL || op.kind == pcas::OP_RESID) {
            double a = 1.0, b = 0.0;
            const double J = ev(op.kind == pcas::OP_EVAL ? op.w : nullptr, op.slot,
                                op.fixed_ab ? 1 : 0, op.ab, &a, &b);
            m.eval_result(J, a, b);
        } else {
            double g[PCAS_MAX_K], H[PCAS_MAX_K * PCAS_MAX_K];
            const int have = gr(op.w, op.slot, op.ab[0], op.ab[1], g, H);
            m.grad_result(g, have ? H : nullptr);
        }
    }
    for (int k = 0; k < K; ++k) w_out[k] = m.w()[k];
    *rep = m.report();
    return 0;
}

// The solver's noise band at one point (the rounding model, or `fixed`).
double harness_noise_rel(double fixed, double u, double M, double sy, double syy, double J,
                         double a, double b) {
    pcas::NoiseModel n;
    n.fixed = fixed;
    n.u = u;
    n.M = M;
    n.sy = sy;
    n.syy = syy;
    return n.rel(J, a, b);
}

}  // extern "C"
