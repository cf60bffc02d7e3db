/*
 * FP64 CPU oracle for the batched rigid-body step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct definitions of what one physics substep computes.  The
 * paper specifies the physics only by its interface (section "Architecture": static model,
 * time-varying per-world state with a leading world dimension, per-world field expansion;
 * section "Manager-Based API", pipeline step "Simulate": d physics substeps per env step
 * with controls held).  The contents of a substep follow MuJoCo's published formulation,
 * written from the mathematics:
 *   - forward kinematics of a tree of bodies with free and hinge joints;
 *   - joint-space inertia M as the sum over bodies of m Jp'Jp + Jr' I Jr (definition of
 *     kinetic energy), plus joint armature;
 *   - bias forces c(q, v) (Coriolis, centrifugal, gravity) as the Jacobian-transpose sum of
 *     each body's Newton-Euler bias wrench (Featherstone 2008, ch. 5, with gravity applied
 *     as a base acceleration);
 *   - brute-force primitive collision against planes;
 *   - soft contact constraints with a pyramidal friction cone, impedance and reference
 *     acceleration (Todorov 2014; MuJoCo "Computation" chapter);
 *   - the primal Newton method with exact line search on the convex constraint cost;
 *   - semi-implicit Euler integration with exponential-map quaternion update.
 * Every stage uses dense matrices and Cholesky factorisations; nothing is blocked, fused
 * or reordered beyond these definitions.
 */
#include "rbo.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

thread_local std::string g_err;
int fail(const std::string& s) {
    g_err = s;
    return -1;
}

// ------------------------------------------------------------------------------------
// small 3-D helpers (row-major 3x3 matrices, quaternions (w, x, y, z), Hamilton product)
// ------------------------------------------------------------------------------------
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* o) {
    double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
inline void matvec3(const double* R, const double* v, double* o) {
    double t[3];
    for (int i = 0; i < 3; i++) t[i] = R[3 * i] * v[0] + R[3 * i + 1] * v[1] + R[3 * i + 2] * v[2];
    o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
inline void matmul3(const double* A, const double* B, double* O) {
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    std::memcpy(O, t, sizeof t);
}
inline void quatmul(const double* a, const double* b, double* o) {
    double t[4] = {a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                   a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                   a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                   a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]};
    o[0] = t[0]; o[1] = t[1]; o[2] = t[2]; o[3] = t[3];
}
inline void quatnormalize(double* q) {
    double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) q[i] /= n;
}
inline void quat2mat(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
// rotation vector (axis times angle, angle in [0, pi)) of a rotation matrix E: the angle from the
// trace, the axis from the skew part E - E' = 2 sin(angle) [axis]x
inline void rotvec(const double* E, double* th) {
    double c = std::min(std::max((E[0] + E[4] + E[8] - 1) / 2, -1.0), 1.0);
    double ang = std::acos(c);
    double w[3] = {E[7] - E[5], E[2] - E[6], E[3] - E[1]};
    double f = ang < 1e-6 ? 0.5 + ang * ang / 12 : ang / (2 * std::sin(ang));
    for (int i = 0; i < 3; i++) th[i] = f * w[i];
}
inline void axisangle2quat(const double* u, double theta, double* q) {
    double s = std::sin(theta / 2);
    q[0] = std::cos(theta / 2); q[1] = s * u[0]; q[2] = s * u[1]; q[3] = s * u[2];
}

// ------------------------------------------------------------------------------------
// model and per-world data
// ------------------------------------------------------------------------------------
struct Model {
    int nbody = 0, njnt = 0, ngeom = 0, nu = 0, nq = 0, nv = 0;
    std::vector<int> parent, body_jnt;
    std::vector<double> bpos, bquat, ipos, iquat, mass, inertia;
    std::vector<int> jtype, jbody, jqadr, jdadr;
    std::vector<double> jpos, jaxis, jarm;
    std::vector<double> jrange;   // [njnt, 2]
    std::vector<char> jlimited;   // hinge with lower < upper
    int nlim = 0;
    std::vector<double> jdamp;    // hinge damping
    int ndamp = 0;
    std::vector<int> gtype, gbody, gcontype, gconaff, gcondim;
    int hf_nrow = 0, hf_ncol = 0;
    std::vector<double> hf;   // height grid [hf_nrow, hf_ncol]
    int neq = 0;
    std::vector<int> eqtype, eqbody;           // equality constraints: connect / weld, the moving body
    std::vector<double> eqanchor, eqtarget;    // [neq, 3] anchor (body frame), [neq, 7] world point + quat
    std::vector<double> gpos, gquat, gsize, gfric, gmargin;
    std::vector<double> gfric_spin, gfric_roll;   // torsional, rolling friction (condim 4, 6)
    std::vector<int> atype, ajoint;
    std::vector<double> akp, akd, agear;
    std::vector<int> movable;  // body has a joint on its path to the world
    std::vector<int> dof_depth;    // dofs on the dof's chain from the root, itself included
    std::vector<int> body_cdepth;  // dofs on the body's chain from the root
    double dt = 0.005;
    int K = 1;
    double grav[3] = {0, 0, -9.81};
    int iters = 4;
    double tol = 1e-8;
    int cone = 0;             // 0 pyramidal, 1 elliptic friction cones
    double impratio = 1.0;    // elliptic cones: ratio of frictional to normal impedance
    double solref[2] = {0.02, 1.0};
    double solimp[5] = {0.9, 0.95, 0.001, 0.5, 2.0};
    bool fr_pw = false, ms_pw = false;
    int maxcon = 0, npair = 0;
    int maxconrows = 0;   // rows of maxcon contacts: 1 (condim 1) or 2 (condim - 1) per contact
    double meaninertia = 1.0;
    int mode = 0;
};

struct Contact {
    int g1, g2, feature, b1, b2;
    int dim;   // 1: frictionless (one normal row), 3, 4, 6: pyramidal friction, 2 (dim - 1) rows
    double dist, pos[3], frame[9], mu, mu_spin, mu_roll;
};

struct Data {
    const Model* m;
    std::vector<double> q, v, ctrl, aws;
    double fr = 1.0;
    std::vector<double> ms;  // mass scale per body
    // kinematics
    std::vector<double> xpos, xquat, xmat, com, Iw, mb, janchor, jaxw, gx, gR;
    // dynamics
    std::vector<double> M, c, tau, a0;
    // constraints
    std::vector<Contact> con;
    int nrows = 0;
    std::vector<int> crow;   // first row of each contact
    std::vector<double> J, aref, D, Ahat, efc_force, a, cforce;
    std::vector<double> aint;   // acceleration the integrator applies (a, or its damped correction)
    int niter = 0;
    bool itercap = false;   // the Newton loop used every iteration without meeting a tolerance
    double cost = 0;
    // work record of the substep (for the work and operation-count outputs)
    std::vector<int> row_id;        // per row: 4 c + e (pyramid row e of contact c), 256 + dof (limit),
                                    // 512 + 6 q + k (row k of equality q)
    std::vector<char> bilat;        // per row: bilateral (equality rows: active on both sides)
    std::vector<char> ell;          // per row: one of an elliptic contact's rows (costed per contact)
    std::vector<int> ell_row0;      // per elliptic contact: its first row (normal, t1, t2, spin, roll)
    std::vector<int> ell_dim;       // per elliptic contact: its rows (its condim: 3, 4 or 6)
    std::vector<double> ell_mu;     // per elliptic contact: cone slope mu / sqrt(impratio)
    std::vector<int> row_nnz;       // per row: non-zero Jacobian entries (the dofs it touches)
    int segments = 0;               // quadratic pieces the line searches examined
    int active_final = 0;           // rows active at the solution
    uint32_t fp[RBO_FPITER] = {};   // active-set fingerprint before each of the first Newton updates
    std::vector<std::vector<int>> act_iter;   // rows active when each Newton Hessian was formed

    explicit Data(const Model* mm) : m(mm) {
        int nb = m->nbody, nv = m->nv, nj = m->njnt, ng = m->ngeom;
        q.assign(m->nq, 0); v.assign(nv, 0); ctrl.assign(m->nu, 0); aws.assign(nv, 0);
        ms.assign(nb, 1.0);
        xpos.assign(3 * nb, 0); xquat.assign(4 * nb, 0); xmat.assign(9 * nb, 0); com.assign(3 * nb, 0);
        Iw.assign(9 * nb, 0); mb.assign(nb, 0);
        janchor.assign(3 * nj, 0); jaxw.assign(3 * nj, 0);
        gx.assign(3 * ng, 0); gR.assign(9 * ng, 0);
        M.assign(nv * nv, 0); c.assign(nv, 0); tau.assign(nv, 0); a0.assign(nv, 0); a.assign(nv, 0);
        aint.assign(nv, 0);
    }
};

// ------------------------------------------------------------------------------------
// forward kinematics: body frames, centres of mass, world inertias, joint axes, geom poses
// ------------------------------------------------------------------------------------
void kinematics(const Model& m, Data& d) {
    for (int i = 0; i < 3; i++) d.xpos[i] = 0;
    double qid[4] = {1, 0, 0, 0};
    std::memcpy(&d.xquat[0], qid, sizeof qid);
    quat2mat(qid, &d.xmat[0]);
    for (int b = 1; b < m.nbody; b++) {
        int p = m.parent[b];
        double x0[3], q0[4], R0[9];
        matvec3(&d.xmat[9 * p], &m.bpos[3 * b], x0);
        for (int i = 0; i < 3; i++) x0[i] += d.xpos[3 * p + i];
        quatmul(&d.xquat[4 * p], &m.bquat[4 * b], q0);
        int j = m.body_jnt[b];
        double* xb = &d.xpos[3 * b];
        double* qb = &d.xquat[4 * b];
        if (j < 0) {
            std::memcpy(xb, x0, 3 * sizeof(double));
            std::memcpy(qb, q0, 4 * sizeof(double));
        } else if (m.jtype[j] == RBO_JNT_FREE) {
            int a = m.jqadr[j];
            for (int i = 0; i < 3; i++) xb[i] = d.q[a + i];
            for (int i = 0; i < 4; i++) qb[i] = d.q[a + 3 + i];
            quatnormalize(qb);
            std::memcpy(&d.janchor[3 * j], xb, 3 * sizeof(double));
        } else {
            quat2mat(q0, R0);
            double o[3], u[3], qr[4], Rb[9], off[3];
            matvec3(R0, &m.jpos[3 * j], o);
            for (int i = 0; i < 3; i++) o[i] += x0[i];
            matvec3(R0, &m.jaxis[3 * j], u);
            axisangle2quat(u, d.q[m.jqadr[j]], qr);
            quatmul(qr, q0, qb);
            quat2mat(qb, Rb);
            matvec3(Rb, &m.jpos[3 * j], off);
            for (int i = 0; i < 3; i++) xb[i] = o[i] - off[i];
            std::memcpy(&d.janchor[3 * j], o, sizeof o);
            std::memcpy(&d.jaxw[3 * j], u, sizeof u);
        }
        quat2mat(qb, &d.xmat[9 * b]);
    }
    // centres of mass, masses and world-frame rotational inertias about the COM
    for (int b = 0; b < m.nbody; b++) {
        const double* R = &d.xmat[9 * b];
        double off[3];
        matvec3(R, &m.ipos[3 * b], off);
        for (int i = 0; i < 3; i++) d.com[3 * b + i] = d.xpos[3 * b + i] + off[i];
        double s = d.ms[b];
        d.mb[b] = s * m.mass[b];
        double Ri[9], RR[9];
        quat2mat(&m.iquat[4 * b], Ri);
        matmul3(R, Ri, RR);
        // I = RR diag(s*inertia) RR'
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) {
                double acc = 0;
                for (int l = 0; l < 3; l++) acc += RR[3 * i + l] * s * m.inertia[3 * b + l] * RR[3 * k + l];
                d.Iw[9 * b + 3 * i + k] = acc;
            }
    }
    for (int g = 0; g < m.ngeom; g++) {
        int b = m.gbody[g];
        double off[3], Rg[9];
        matvec3(&d.xmat[9 * b], &m.gpos[3 * g], off);
        for (int i = 0; i < 3; i++) d.gx[3 * g + i] = d.xpos[3 * b + i] + off[i];
        quat2mat(&m.gquat[4 * g], Rg);
        matmul3(&d.xmat[9 * b], Rg, &d.gR[9 * g]);
    }
}

// Point Jacobians of world point p attached to body b: jacp, jacr are [3, nv] row-major.
void jacobian(const Model& m, const Data& d, int b, const double* p, double* jacp, double* jacr) {
    int nv = m.nv;
    std::fill(jacp, jacp + 3 * nv, 0.0);
    std::fill(jacr, jacr + 3 * nv, 0.0);
    for (int bb = b; bb > 0; bb = m.parent[bb]) {
        int j = m.body_jnt[bb];
        if (j < 0) continue;
        int k = m.jdadr[j];
        if (m.jtype[j] == RBO_JNT_HINGE) {
            const double* u = &d.jaxw[3 * j];
            double r[3], w[3];
            for (int i = 0; i < 3; i++) r[i] = p[i] - d.janchor[3 * j + i];
            cross3(u, r, w);
            for (int i = 0; i < 3; i++) {
                jacr[i * nv + k] = u[i];
                jacp[i * nv + k] = w[i];
            }
        } else {
            const double* R = &d.xmat[9 * bb];
            double r[3];
            for (int i = 0; i < 3; i++) r[i] = p[i] - d.xpos[3 * bb + i];
            for (int a = 0; a < 3; a++) {
                jacp[a * nv + k + a] = 1.0;
                double e[3] = {R[a], R[3 + a], R[6 + a]};  // body axis a in world
                double w[3];
                cross3(e, r, w);
                for (int i = 0; i < 3; i++) {
                    jacr[i * nv + k + 3 + a] = e[i];
                    jacp[i * nv + k + 3 + a] = w[i];
                }
            }
        }
    }
}

// M = sum_b m_b Jp(b, com_b)' Jp(b, com_b) + Jr(b)' I_b Jr(b) + diag(armature)
void mass_matrix(const Model& m, Data& d) {
    int nv = m.nv;
    std::fill(d.M.begin(), d.M.end(), 0.0);
    std::vector<double> jp(3 * nv), jr(3 * nv), IJ(3 * nv);
    for (int b = 1; b < m.nbody; b++) {
        jacobian(m, d, b, &d.com[3 * b], jp.data(), jr.data());
        const double* I = &d.Iw[9 * b];
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < nv; k++) IJ[i * nv + k] = I[3 * i] * jr[k] + I[3 * i + 1] * jr[nv + k] + I[3 * i + 2] * jr[2 * nv + k];
        for (int r = 0; r < nv; r++)
            for (int s = 0; s < nv; s++) {
                double acc = 0;
                for (int i = 0; i < 3; i++) acc += d.mb[b] * jp[i * nv + r] * jp[i * nv + s] + jr[i * nv + r] * IJ[i * nv + s];
                d.M[r * nv + s] += acc;
            }
    }
    for (int j = 0; j < m.njnt; j++)
        if (m.jtype[j] == RBO_JNT_HINGE) d.M[m.jdadr[j] * (nv + 1)] += m.jarm[j];
}

// c(q, v): bias accelerations of every body with qacc = 0 and the world accelerating
// upward at -gravity, turned into bias wrenches and projected with Jacobian transposes.
void bias_forces(const Model& m, Data& d) {
    int nv = m.nv, nb = m.nbody;
    std::vector<double> w(3 * nb, 0.0), al(3 * nb, 0.0), ac(3 * nb, 0.0);
    for (int i = 0; i < 3; i++) ac[i] = -m.grav[i];
    std::fill(d.c.begin(), d.c.end(), 0.0);
    std::vector<double> jp(3 * nv), jr(3 * nv);
    for (int b = 1; b < nb; b++) {
        int p = m.parent[b], j = m.body_jnt[b];
        double* wb = &w[3 * b];
        double* ab = &al[3 * b];
        double* acb = &ac[3 * b];
        const double* cb = &d.com[3 * b];
        const double* cp = &d.com[3 * p];
        if (j >= 0 && m.jtype[j] == RBO_JNT_FREE) {
            double wl[3] = {d.v[m.jdadr[j] + 3], d.v[m.jdadr[j] + 4], d.v[m.jdadr[j] + 5]};
            matvec3(&d.xmat[9 * b], wl, wb);
            ab[0] = ab[1] = ab[2] = 0;
            double r[3], t[3], t2[3];
            for (int i = 0; i < 3; i++) r[i] = cb[i] - d.xpos[3 * b + i];
            cross3(wb, r, t);
            cross3(wb, t, t2);
            for (int i = 0; i < 3; i++) acb[i] = -m.grav[i] + t2[i];
        } else {
            const double* wp = &w[3 * p];
            const double* ap = &al[3 * p];
            // the point o about which the body moves relative to its parent
            double o[3];
            double qd = 0, u[3] = {0, 0, 0};
            if (j >= 0) {
                std::memcpy(o, &d.janchor[3 * j], sizeof o);
                std::memcpy(u, &d.jaxw[3 * j], sizeof u);
                qd = d.v[m.jdadr[j]];
            } else {
                std::memcpy(o, cb, sizeof o);
            }
            double uq[3] = {u[0] * qd, u[1] * qd, u[2] * qd}, t[3];
            for (int i = 0; i < 3; i++) wb[i] = wp[i] + uq[i];
            cross3(wp, uq, t);
            for (int i = 0; i < 3; i++) ab[i] = ap[i] + t[i];
            // acceleration of o as a point of the parent
            double r[3], t1[3], t2[3], t3[3], ao[3];
            for (int i = 0; i < 3; i++) r[i] = o[i] - cp[i];
            cross3(ap, r, t1);
            cross3(wp, r, t2);
            cross3(wp, t2, t3);
            for (int i = 0; i < 3; i++) ao[i] = ac[3 * p + i] + t1[i] + t3[i];
            // acceleration of this body's COM
            for (int i = 0; i < 3; i++) r[i] = cb[i] - o[i];
            cross3(ab, r, t1);
            cross3(wb, r, t2);
            cross3(wb, t2, t3);
            for (int i = 0; i < 3; i++) acb[i] = ao[i] + t1[i] + t3[i];
        }
        // bias wrench of the body and its projection
        double f[3], n[3], Iw[3], Ia[3], wIw[3];
        for (int i = 0; i < 3; i++) f[i] = d.mb[b] * acb[i];
        matvec3(&d.Iw[9 * b], wb, Iw);
        matvec3(&d.Iw[9 * b], ab, Ia);
        cross3(wb, Iw, wIw);
        for (int i = 0; i < 3; i++) n[i] = Ia[i] + wIw[i];
        jacobian(m, d, b, cb, jp.data(), jr.data());
        for (int k = 0; k < nv; k++)
            for (int i = 0; i < 3; i++) d.c[k] += jp[i * nv + k] * f[i] + jr[i * nv + k] * n[i];
    }
}

void actuation(const Model& m, Data& d) {
    std::fill(d.tau.begin(), d.tau.end(), 0.0);
    for (int u = 0; u < m.nu; u++) {
        int j = m.ajoint[u];
        int k = m.jdadr[j], a = m.jqadr[j];
        if (m.atype[u] == RBO_ACT_POSITION)
            d.tau[k] += m.akp[u] * (d.ctrl[u] - d.q[a]) - m.akd[u] * d.v[k];
        else
            d.tau[k] += m.agear[u] * d.ctrl[u];
    }
}

// passive joint damping: -damping * qvel on each damped hinge, added to the applied forces
void passive(const Model& m, Data& d) {
    for (int j = 0; j < m.njnt; j++)
        if (m.jdamp[j] > 0) d.tau[m.jdadr[j]] -= m.jdamp[j] * d.v[m.jdadr[j]];
}

// dense Cholesky A = L L' (lower); returns false if not positive definite
bool cholesky(const std::vector<double>& A, int n, std::vector<double>& L) {
    L.assign(n * n, 0.0);
    for (int j = 0; j < n; j++) {
        double s = A[j * n + j];
        for (int k = 0; k < j; k++) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0)) return false;
        L[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; i++) {
            double t = A[i * n + j];
            for (int k = 0; k < j; k++) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    return true;
}
void chol_solve(const std::vector<double>& L, int n, const double* b, double* x) {
    std::vector<double> y(n);
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < n; k++) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

// ------------------------------------------------------------------------------------
// collision: brute force over geom pairs
// ------------------------------------------------------------------------------------
bool pair_allowed(const Model& m, int g1, int g2) {
    int b1 = m.gbody[g1], b2 = m.gbody[g2];
    if (b1 == b2) return false;
    if ((m.parent[b1] == b2 && b2 != 0) || (m.parent[b2] == b1 && b1 != 0)) return false;
    if (((m.gcontype[g1] & m.gconaff[g2]) | (m.gcontype[g2] & m.gconaff[g1])) == 0) return false;
    if (!m.movable[b1] && !m.movable[b2]) return false;
    return true;
}

int pair_capacity(int t1, int t2) {
    if (t1 == RBO_GEOM_PLANE && t2 == RBO_GEOM_SPHERE) return 1;
    if (t1 == RBO_GEOM_PLANE && t2 == RBO_GEOM_CAPSULE) return 2;
    if (t1 == RBO_GEOM_PLANE && t2 == RBO_GEOM_BOX) return 8;
    if (t1 == RBO_GEOM_BOX && t2 == RBO_GEOM_BOX) return 8;
    if (t1 == RBO_GEOM_SPHERE && t2 == RBO_GEOM_BOX) return 1;
    if (t1 == RBO_GEOM_CAPSULE && t2 == RBO_GEOM_BOX) return 2;
    if ((t1 == RBO_GEOM_SPHERE || t1 == RBO_GEOM_CAPSULE) && (t2 == RBO_GEOM_SPHERE || t2 == RBO_GEOM_CAPSULE)) return 1;
    if (t2 == RBO_GEOM_HFIELD) return t1 == RBO_GEOM_SPHERE ? 1 : t1 == RBO_GEOM_CAPSULE ? 2 : t1 == RBO_GEOM_BOX ? 8 : -1;
    return -1;
}

// tangent frame: t1 = normalise(e_k - (e_k.n) n), k = argmin |n_k| (lowest on ties); t2 = n x t1
void contact_frame(const double* n, double* frame) {
    int k = 0;
    for (int i = 1; i < 3; i++)
        if (std::fabs(n[i]) < std::fabs(n[k])) k = i;
    double t1[3] = {0, 0, 0};
    t1[k] = 1.0;
    double dn = t1[k] * n[k];
    for (int i = 0; i < 3; i++) t1[i] -= dn * n[i];
    double l = std::sqrt(dot3(t1, t1));
    for (int i = 0; i < 3; i++) t1[i] /= l;
    double t2[3];
    cross3(n, t1, t2);
    for (int i = 0; i < 3; i++) {
        frame[i] = n[i];
        frame[3 + i] = t1[i];
        frame[6 + i] = t2[i];
    }
}

void add_contact(const Model& m, Data& d, int g1, int g2, int feature, double dist, const double* pos,
                 const double* n) {
    Contact c;
    c.g1 = g1; c.g2 = g2; c.feature = feature; c.dist = dist;
    c.b1 = m.gbody[g1]; c.b2 = m.gbody[g2];
    std::memcpy(c.pos, pos, 3 * sizeof(double));
    contact_frame(n, c.frame);
    c.dim = std::max(m.gcondim[g1], m.gcondim[g2]);
    c.mu = c.dim == 1 ? 0.0 : (m.fr_pw ? d.fr : std::max(m.gfric[g1], m.gfric[g2]));
    c.mu_spin = c.dim >= 4 ? std::max(m.gfric_spin[g1], m.gfric_spin[g2]) : 0.0;
    c.mu_roll = c.dim >= 6 ? std::max(m.gfric_roll[g1], m.gfric_roll[g2]) : 0.0;
    d.con.push_back(c);
}

// Box-box by the separating-axis test (Ericson 2004, ch. 4.4 and 5.2): overlaps along the 6
// face normals and the 9 edge-edge cross products; the axis of least overlap (earlier axes
// win unless a later one is smaller by more than 1e-5 (1 + overlap)) gives the normal from
// g1 to g2.  Face axis: the incident face (most anti-parallel to the reference face) is
// clipped against the reference face's four side planes and every clipped point below the
// reference face is a contact, midway between the point and the face.  Edge axis: one
// contact midway between the closest points of the two supporting edges, depth -overlap.
void box_box(const Model& m, Data& d, int g1, int g2, double margin) {
    const double* cA = &d.gx[3 * g1];
    const double* cB = &d.gx[3 * g2];
    const double* RA = &d.gR[9 * g1];
    const double* RB = &d.gR[9 * g2];
    const double* hA = &m.gsize[3 * g1];
    const double* hB = &m.gsize[3 * g2];
    double aA[3][3], aB[3][3], dc[3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) {
            aA[i][k] = RA[3 * k + i];  // column i of the rotation = box axis i
            aB[i][k] = RB[3 * k + i];
        }
    for (int k = 0; k < 3; k++) dc[k] = cB[k] - cA[k];
    int best = -1;
    double best_ov = 0, best_ax[3] = {0, 0, 0};
    for (int ax = 0; ax < 15; ax++) {
        double L[3];
        if (ax < 3) {
            for (int k = 0; k < 3; k++) L[k] = aA[ax][k];
        } else if (ax < 6) {
            for (int k = 0; k < 3; k++) L[k] = aB[ax - 3][k];
        } else {
            int i = (ax - 6) / 3, j = (ax - 6) % 3;
            cross3(aA[i], aB[j], L);
            double n = std::sqrt(dot3(L, L));
            if (n < 1e-6) continue;
            for (int k = 0; k < 3; k++) L[k] /= n;
        }
        double rA = 0, rB = 0;
        for (int i = 0; i < 3; i++) {
            rA += hA[i] * std::fabs(dot3(L, aA[i]));
            rB += hB[i] * std::fabs(dot3(L, aB[i]));
        }
        double ov = rA + rB - std::fabs(dot3(L, dc));
        if (-ov >= margin) return;  // separated along this axis
        if (best < 0 || ov < best_ov - 1e-5 * (1 + std::fabs(best_ov))) {
            best = ax;
            best_ov = ov;
            for (int k = 0; k < 3; k++) best_ax[k] = L[k];
        }
    }
    if (best < 0) return;
    double n[3];
    double sgn = dot3(best_ax, dc) < 0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; k++) n[k] = sgn * best_ax[k];
    if (best < 6) {
        bool refA = best < 3;
        int rax = refA ? best : best - 3;
        const double* cR = refA ? cA : cB;
        const double* hR = refA ? hA : hB;
        double (*aR)[3] = refA ? aA : aB;
        const double* cI = refA ? cB : cA;
        const double* hI = refA ? hB : hA;
        double (*aI)[3] = refA ? aB : aA;
        double nr[3];  // outward normal of the reference face
        for (int k = 0; k < 3; k++) nr[k] = refA ? n[k] : -n[k];
        double pR[3];
        for (int k = 0; k < 3; k++) pR[k] = cR[k] + hR[rax] * nr[k];
        int u = (rax + 1) % 3, v = (rax + 2) % 3;
        if (u > v) std::swap(u, v);
        // incident face: most anti-parallel to the reference normal (lowest axis on ties)
        int ia = 0;
        double bestdot = -1;
        for (int j = 0; j < 3; j++) {
            double a = std::fabs(dot3(aI[j], nr));
            if (a > bestdot + 1e-12) { bestdot = a; ia = j; }
        }
        double s = dot3(aI[ia], nr) > 0 ? -1.0 : 1.0;
        int p = (ia + 1) % 3, q = (ia + 2) % 3;
        if (p > q) std::swap(p, q);
        double fc[3];
        for (int k = 0; k < 3; k++) fc[k] = cI[k] + s * hI[ia] * aI[ia][k];
        const double sp[4] = {1, -1, -1, 1}, sq[4] = {1, 1, -1, -1};
        std::vector<std::array<double, 3>> poly(4);
        for (int c = 0; c < 4; c++)
            for (int k = 0; k < 3; k++) poly[c][k] = fc[k] + sp[c] * hI[p] * aI[p][k] + sq[c] * hI[q] * aI[q][k];
        // Sutherland-Hodgman against (x.u <= hu), (-x.u <= hu), (x.v <= hv), (-x.v <= hv), x = point - pR
        for (int plane = 0; plane < 4; plane++) {
            const double* dir = plane < 2 ? aR[u] : aR[v];
            double ext = plane < 2 ? hR[u] : hR[v];
            double sg = (plane % 2 == 0) ? 1.0 : -1.0;
            std::vector<std::array<double, 3>> out;
            size_t np = poly.size();
            for (size_t i = 0; i < np; i++) {
                const auto& P = poly[i];
                const auto& Q = poly[(i + 1) % np];
                double x[3], y[3];
                for (int k = 0; k < 3; k++) { x[k] = P[k] - pR[k]; y[k] = Q[k] - pR[k]; }
                double fp = sg * dot3(x, dir) - ext, fq = sg * dot3(y, dir) - ext;
                if (fp <= 0) out.push_back(P);
                if ((fp < 0 && fq > 0) || (fp > 0 && fq < 0)) {
                    double t = fp / (fp - fq);
                    std::array<double, 3> I;
                    for (int k = 0; k < 3; k++) I[k] = P[k] + t * (Q[k] - P[k]);
                    out.push_back(I);
                }
            }
            poly.swap(out);
            if (poly.empty()) return;
        }
        int feat = 0;
        for (const auto& P : poly) {
            double x[3];
            for (int k = 0; k < 3; k++) x[k] = P[k] - pR[k];
            double dist = dot3(x, nr);
            if (dist < margin && feat < 8) {
                double pos[3];
                for (int k = 0; k < 3; k++) pos[k] = P[k] - nr[k] * dist / 2;
                add_contact(m, d, g1, g2, feat, dist, pos, n);
            }
            feat++;
        }
    } else {
        int i = (best - 6) / 3, j = (best - 6) % 3;
        double PA[3], PB[3];
        for (int k = 0; k < 3; k++) { PA[k] = cA[k]; PB[k] = cB[k]; }
        for (int a = 0; a < 3; a++) {
            if (a != i) {
                double sa = dot3(n, aA[a]) >= 0 ? 1.0 : -1.0;
                for (int k = 0; k < 3; k++) PA[k] += sa * hA[a] * aA[a][k];
            }
            if (a != j) {
                double sb = dot3(n, aB[a]) >= 0 ? -1.0 : 1.0;
                for (int k = 0; k < 3; k++) PB[k] += sb * hB[a] * aB[a][k];
            }
        }
        // closest points of PA + t aA_i (|t| <= hA_i) and PB + w aB_j (|w| <= hB_j)
        double r[3];
        for (int k = 0; k < 3; k++) r[k] = PA[k] - PB[k];
        double b = dot3(aA[i], aB[j]), c = dot3(aA[i], r), f = dot3(aB[j], r);
        double den = 1 - b * b;
        double t = den > 1e-12 ? (b * f - c) / den : 0.0;
        t = std::min(std::max(t, -hA[i]), hA[i]);
        double w = b * t + f;
        if (w < -hB[j] || w > hB[j]) {
            w = std::min(std::max(w, -hB[j]), hB[j]);
            t = std::min(std::max(b * w - c, -hA[i]), hA[i]);
        }
        double pos[3];
        for (int k = 0; k < 3; k++) pos[k] = 0.5 * (PA[k] + t * aA[i][k] + PB[k] + w * aB[j][k]);
        add_contact(m, d, g1, g2, 0, -best_ov, pos, n);
    }
}

// A sphere (centre c, radius r) of geom g1 against box g2: the closest point of the box to c (the centre
// clamped to the box in the box frame); when c lies inside the box, the nearest face instead
// (least depth h_i - |p_i|, lowest axis on ties, towards the side of p_i, + at 0).  Signed
// distance = |c - closest| - r outside, -(depth + r) inside; normal from the sphere towards
// the box; the contact point lies halfway between the sphere's surface and the box's.
void sphere_at_box(const Model& m, Data& d, int g1, int g2, int feature, const double* c, double r, double margin) {
    const double* x = &d.gx[3 * g2];
    const double* R = &d.gR[9 * g2];
    const double* h = &m.gsize[3 * g2];
    double rel[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]}, p[3];
    for (int i = 0; i < 3; i++) p[i] = R[i] * rel[0] + R[3 + i] * rel[1] + R[6 + i] * rel[2];   // R' rel
    double q[3];
    bool inside = true;
    for (int i = 0; i < 3; i++) {
        q[i] = std::min(std::max(p[i], -h[i]), h[i]);
        if (q[i] != p[i]) inside = false;
    }
    double nl[3] = {0, 0, 0}, dist;   // nl: box towards sphere, box frame
    if (!inside) {
        double df[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
        double len = std::sqrt(dot3(df, df));
        for (int i = 0; i < 3; i++) nl[i] = df[i] / len;
        dist = len - r;
    } else {
        int k = 0;
        for (int i = 1; i < 3; i++)
            if (h[i] - std::fabs(p[i]) < h[k] - std::fabs(p[k])) k = i;
        nl[k] = p[k] < 0 ? -1.0 : 1.0;
        dist = -(h[k] - std::fabs(p[k]) + r);
    }
    if (!(dist < margin)) return;
    double nw[3];
    matvec3(R, nl, nw);
    double n[3] = {-nw[0], -nw[1], -nw[2]}, pos[3];
    for (int i = 0; i < 3; i++) pos[i] = c[i] - nw[i] * (r + dist / 2);
    add_contact(m, d, g1, g2, feature, dist, pos, n);
}

void sphere_box(const Model& m, Data& d, int g1, int g2, double margin) {
    sphere_at_box(m, d, g1, g2, 0, &d.gx[3 * g1], m.gsize[3 * g1], margin);
}

// Capsule g1 against box g2, as against a plane: the spheres of radius r at the capsule's two
// segment ends (feature 0 at -z, 1 at +z of the capsule frame), each against the box by the
// sphere rule above.
// Closest points of segments [p1, q1] and [p2, q2] (Ericson, Real-Time Collision Detection,
// section 5.1.9): the parameters s, t in [0, 1] minimising the distance, with nearly parallel
// segments (a e - b^2 <= 1e-6 a e) taking s = 0.
void closest_segments(const double* p1, const double* q1, const double* p2, const double* q2, double* c1,
                      double* c2) {
    double d1[3], d2[3], r[3];
    for (int i = 0; i < 3; i++) {
        d1[i] = q1[i] - p1[i];
        d2[i] = q2[i] - p2[i];
        r[i] = p1[i] - p2[i];
    }
    const double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    auto clamp01 = [](double x) { return std::min(std::max(x, 0.0), 1.0); };
    double s = 0, t = 0;
    if (a <= 1e-12 && e <= 1e-12) {
        s = t = 0;
    } else if (a <= 1e-12) {
        t = clamp01(f / e);
    } else {
        const double c = dot3(d1, r);
        if (e <= 1e-12) {
            s = clamp01(-c / a);
        } else {
            const double b = dot3(d1, d2), den = a * e - b * b;
            s = den > 1e-6 * a * e ? clamp01((b * f - c * e) / den) : 0.0;
            t = (b * s + f) / e;
            if (t < 0) {
                t = 0;
                s = clamp01(-c / a);
            } else if (t > 1) {
                t = 1;
                s = clamp01((b - c) / a);
            }
        }
    }
    for (int i = 0; i < 3; i++) {
        c1[i] = p1[i] + d1[i] * s;
        c2[i] = p2[i] + d2[i] * t;
    }
}

// Spheres and capsules against each other: a capsule is its segment (local z, half-length
// size[1]) swept by its radius, a sphere a point swept by its radius; the contact joins the
// closest points c1 (on g1) and c2 (on g2): distance |c2 - c1| - r1 - r2, normal from c1 to c2
// (+z when they coincide), point halfway between the surfaces, feature 0.
void round_pair(const Model& m, Data& d, int g1, int g2, double margin) {
    double p[2][3], q[2][3];
    for (int k = 0; k < 2; k++) {
        const int g = k == 0 ? g1 : g2;
        const double* x = &d.gx[3 * g];
        const double* R = &d.gR[9 * g];
        const double h = m.gtype[g] == RBO_GEOM_CAPSULE ? m.gsize[3 * g + 1] : 0.0;
        for (int i = 0; i < 3; i++) {
            p[k][i] = x[i] - h * R[3 * i + 2];
            q[k][i] = x[i] + h * R[3 * i + 2];
        }
    }
    double c1[3], c2[3];
    closest_segments(p[0], q[0], p[1], q[1], c1, c2);
    const double r1 = m.gsize[3 * g1], r2 = m.gsize[3 * g2];
    double n[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
    const double len = std::sqrt(dot3(n, n));
    if (len > 0) {
        for (int i = 0; i < 3; i++) n[i] /= len;
    } else {
        n[0] = 0; n[1] = 0; n[2] = 1;
    }
    const double dist = len - r1 - r2;
    if (dist >= margin) return;
    double pos[3];
    for (int i = 0; i < 3; i++) pos[i] = c1[i] + n[i] * (r1 + 0.5 * dist);
    add_contact(m, d, g1, g2, 0, dist, pos, n);
}

void capsule_box(const Model& m, Data& d, int g1, int g2, double margin) {
    const double* x = &d.gx[3 * g1];
    const double* R = &d.gR[9 * g1];
    const double r = m.gsize[3 * g1], h = m.gsize[3 * g1 + 1];
    for (int f = 0; f < 2; f++) {
        const double sgn = f == 0 ? -1.0 : 1.0;
        double e[3];
        for (int i = 0; i < 3; i++) e[i] = x[i] + sgn * h * R[3 * i + 2];
        sphere_at_box(m, d, g1, g2, f, e, r, margin);
    }
}

// The plane of the height-field triangle under world point e (by its local x, y): outward
// (local +z side) unit normal n and vertex p0, world frame; false when e lies outside the grid.
bool hfield_plane(const Model& m, const Data& d, int g, const double* e, double* n, double* p0) {
    const double* x = &d.gx[3 * g];
    const double* R = &d.gR[9 * g];
    const double sx = m.gsize[3 * g], sy = m.gsize[3 * g + 1];
    const double rel[3] = {e[0] - x[0], e[1] - x[1], e[2] - x[2]};
    const double lx = R[0] * rel[0] + R[3] * rel[1] + R[6] * rel[2];
    const double ly = R[1] * rel[0] + R[4] * rel[1] + R[7] * rel[2];
    const int nr = m.hf_nrow, nc = m.hf_ncol;
    const double u = (lx + sx) / (2 * sx) * (nc - 1), v = (ly + sy) / (2 * sy) * (nr - 1);
    if (!(u >= 0 && u <= nc - 1 && v >= 0 && v <= nr - 1)) return false;
    const int j = std::min((int)std::floor(u), nc - 2), i = std::min((int)std::floor(v), nr - 2);
    auto vert = [&](int a, int b, double* P) {
        P[0] = -sx + 2 * sx * b / (nc - 1);
        P[1] = -sy + 2 * sy * a / (nr - 1);
        P[2] = m.hf[(size_t)a * nc + b];
    };
    double P0[3], P1[3], P2[3];
    vert(i, j, P0);
    if (u - j >= v - i) {
        vert(i, j + 1, P1);
        vert(i + 1, j + 1, P2);
    } else {
        vert(i + 1, j + 1, P1);
        vert(i + 1, j, P2);
    }
    const double a[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    const double b[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    double nl[3];
    cross3(a, b, nl);
    const double len = std::sqrt(dot3(nl, nl));
    for (int k = 0; k < 3; k++) nl[k] /= len;
    matvec3(R, nl, n);
    double pw[3];
    matvec3(R, P0, pw);
    for (int k = 0; k < 3; k++) p0[k] = x[k] + pw[k];
    return true;
}

// Height field g1 against sphere, capsule or box g2, as against a plane candidate by candidate
// (sphere centre, capsule ends 0 / 1, box vertices by sign bits): each candidate point is
// tested against the plane of the triangle under it (hfield_plane); candidates outside the
// grid make no contact.  Normal from the height field towards g2.
void hfield_pair(const Model& m, Data& d, int g1, int g2, double margin) {
    const double* x = &d.gx[3 * g2];
    const double* R = &d.gR[9 * g2];
    const double* sz = &m.gsize[3 * g2];
    const int t2 = m.gtype[g2];
    const int ncand = t2 == RBO_GEOM_SPHERE ? 1 : t2 == RBO_GEOM_CAPSULE ? 2 : 8;
    for (int k = 0; k < ncand; k++) {
        double e[3], rad = 0;
        if (t2 == RBO_GEOM_SPHERE) {
            for (int i = 0; i < 3; i++) e[i] = x[i];
            rad = sz[0];
        } else if (t2 == RBO_GEOM_CAPSULE) {
            const double sgn = k == 0 ? -1.0 : 1.0;
            for (int i = 0; i < 3; i++) e[i] = x[i] + sgn * sz[1] * R[3 * i + 2];
            rad = sz[0];
        } else {
            const double loc[3] = {(k & 4) ? sz[0] : -sz[0], (k & 2) ? sz[1] : -sz[1], (k & 1) ? sz[2] : -sz[2]};
            matvec3(R, loc, e);
            for (int i = 0; i < 3; i++) e[i] += x[i];
        }
        double n[3], p0[3];
        if (!hfield_plane(m, d, g1, e, n, p0)) continue;
        const double r[3] = {e[0] - p0[0], e[1] - p0[1], e[2] - p0[2]};
        const double dist = dot3(n, r) - rad;
        if (dist < margin) {
            double pos[3];
            for (int i = 0; i < 3; i++) pos[i] = e[i] - n[i] * (rad + dist / 2);
            add_contact(m, d, g1, g2, k, dist, pos, n);
        }
    }
}

void collide(const Model& m, Data& d) {
    d.con.clear();
    for (int ga = 0; ga < m.ngeom; ga++)
        for (int gb = ga + 1; gb < m.ngeom; gb++) {
            if (!pair_allowed(m, ga, gb)) continue;
            int g1 = ga, g2 = gb;
            if (m.gtype[g2] < m.gtype[g1]) std::swap(g1, g2);
            int t1 = m.gtype[g1], t2 = m.gtype[g2];
            double margin = std::max(m.gmargin[g1], m.gmargin[g2]);
            if (t1 == RBO_GEOM_BOX && t2 == RBO_GEOM_BOX) {
                box_box(m, d, g1, g2, margin);
                continue;
            }
            if (t1 == RBO_GEOM_SPHERE && t2 == RBO_GEOM_BOX) {
                sphere_box(m, d, g1, g2, margin);
                continue;
            }
            if (t1 == RBO_GEOM_CAPSULE && t2 == RBO_GEOM_BOX) {
                capsule_box(m, d, g1, g2, margin);
                continue;
            }
            if ((t1 == RBO_GEOM_SPHERE || t1 == RBO_GEOM_CAPSULE) && (t2 == RBO_GEOM_SPHERE || t2 == RBO_GEOM_CAPSULE)) {
                round_pair(m, d, g1, g2, margin);
                continue;
            }
            if (t2 == RBO_GEOM_HFIELD) {
                hfield_pair(m, d, g2, g1, margin);   // the height field first, as a plane
                continue;
            }
            if (t1 != RBO_GEOM_PLANE) continue;  // other pairs were rejected at creation
            const double* Rp = &d.gR[9 * g1];
            double n[3] = {Rp[2], Rp[5], Rp[8]};  // plane normal = plane's local +z
            const double* p0 = &d.gx[3 * g1];
            const double* x = &d.gx[3 * g2];
            const double* R = &d.gR[9 * g2];
            const double* sz = &m.gsize[3 * g2];
            if (t2 == RBO_GEOM_SPHERE) {
                double r[3] = {x[0] - p0[0], x[1] - p0[1], x[2] - p0[2]};
                double dist = dot3(n, r) - sz[0];
                if (dist < margin) {
                    double pos[3];
                    for (int i = 0; i < 3; i++) pos[i] = x[i] - n[i] * (sz[0] + dist / 2);
                    add_contact(m, d, g1, g2, 0, dist, pos, n);
                }
            } else if (t2 == RBO_GEOM_CAPSULE) {
                for (int f = 0; f < 2; f++) {
                    double sgn = f == 0 ? -1.0 : 1.0, e[3], r[3];
                    for (int i = 0; i < 3; i++) e[i] = x[i] + sgn * sz[1] * R[3 * i + 2];
                    for (int i = 0; i < 3; i++) r[i] = e[i] - p0[i];
                    double dist = dot3(n, r) - sz[0];
                    if (dist < margin) {
                        double pos[3];
                        for (int i = 0; i < 3; i++) pos[i] = e[i] - n[i] * (sz[0] + dist / 2);
                        add_contact(m, d, g1, g2, f, dist, pos, n);
                    }
                }
            } else if (t2 == RBO_GEOM_BOX) {
                for (int k = 0; k < 8; k++) {
                    double loc[3] = {(k & 4) ? sz[0] : -sz[0], (k & 2) ? sz[1] : -sz[1], (k & 1) ? sz[2] : -sz[2]};
                    double vk[3], r[3];
                    matvec3(R, loc, vk);
                    for (int i = 0; i < 3; i++) vk[i] += x[i];
                    for (int i = 0; i < 3; i++) r[i] = vk[i] - p0[i];
                    double dist = dot3(n, r);
                    if (dist < margin) {
                        double pos[3];
                        for (int i = 0; i < 3; i++) pos[i] = vk[i] - n[i] * dist / 2;
                        add_contact(m, d, g1, g2, k, dist, pos, n);
                    }
                }
            }
        }
    std::sort(d.con.begin(), d.con.end(), [](const Contact& a, const Contact& b) {
        if (a.g1 != b.g1) return a.g1 < b.g1;
        if (a.g2 != b.g2) return a.g2 < b.g2;
        return a.feature < b.feature;
    });
}

// ------------------------------------------------------------------------------------
// soft constraints: pyramidal rows, impedance, reference acceleration, regulariser
// ------------------------------------------------------------------------------------
double impedance(const Model& m, double r) {
    double dmin = m.solimp[0], dmax = m.solimp[1], width = m.solimp[2], mid = m.solimp[3], p = m.solimp[4];
    double x = std::min(std::fabs(r) / width, 1.0);
    double y;
    if (x <= mid)
        y = std::pow(x, p) / std::pow(mid, p - 1);
    else
        y = 1 - std::pow(1 - x, p) / std::pow(1 - mid, p - 1);
    double imp = dmin + y * (dmax - dmin);
    return std::min(std::max(imp, 1e-4), 0.9999);
}

// Rows of the soft constraints, contacts first (4 pyramid rows each, or the normal row alone for
// a frictionless contact, in contact order), then
// joint limits in joint order.  A limited hinge whose angle lies below its lower bound (or
// above its upper bound) contributes one frictionless unilateral row with Jacobian +e_i
// (-e_i) on its dof and distance q - lower (upper - q); limits use the same solref/solimp as
// contacts and no margin.
void make_rows(const Model& m, Data& d, const std::vector<double>& LM) {
    int nv = m.nv, nc = (int)d.con.size();
    // limit rows: (dof, sign, distance)
    std::vector<int> ldof;
    std::vector<double> lsgn, ldist;
    for (int j = 0; j < m.njnt; j++) {
        if (!m.jlimited[j]) continue;
        double q = d.q[m.jqadr[j]];
        double lo = q - m.jrange[2 * j], hi = m.jrange[2 * j + 1] - q;
        if (lo < 0) { ldof.push_back(m.jdadr[j]); lsgn.push_back(1.0); ldist.push_back(lo); }
        if (hi < 0) { ldof.push_back(m.jdadr[j]); lsgn.push_back(-1.0); ldist.push_back(hi); }
    }
    const int nl = (int)ldof.size();
    d.crow.assign(nc, 0);
    int nr = 0;
    for (int ci = 0; ci < nc; ci++) {
        d.crow[ci] = nr;
        nr += d.con[ci].dim == 1 ? 1 : (m.cone == 1 ? d.con[ci].dim : 2 * (d.con[ci].dim - 1));
    }
    int ne = 0;
    for (int q = 0; q < m.neq; q++) ne += m.eqtype[q] == RBO_EQ_WELD ? 6 : 3;
    d.nrows = nr + nl + ne;
    d.bilat.assign(d.nrows, 0);
    d.ell.assign(d.nrows, 0);
    d.ell_row0.clear();
    d.ell_dim.clear();
    d.ell_mu.clear();
    d.J.assign((size_t)d.nrows * nv, 0.0);
    d.row_id.assign(d.nrows, 0);
    d.row_nnz.assign(d.nrows, 0);
    d.aref.assign(d.nrows, 0.0);
    d.D.assign(d.nrows, 0.0);
    d.Ahat.assign(d.nrows, 0.0);
    double dmax = std::min(std::max(m.solimp[1], 1e-4), 0.9999);
    double tc = std::max(m.solref[0], 2 * m.dt), zeta = m.solref[1];
    double bcoef = 2.0 / (dmax * tc);
    double kcoef = 1.0 / (dmax * dmax * tc * tc * zeta * zeta);
    std::vector<double> jp1(3 * nv), jr1(3 * nv), jp2(3 * nv), jr2(3 * nv), Jc(6 * nv), x(nv);
    // reference acceleration and regulariser of row `row` (Jacobian already in place)
    auto finish_row = [&](int row, double rdist) {
        const double* Je = &d.J[(size_t)row * nv];
        for (int k = 0; k < nv; k++) d.row_nnz[row] += Je[k] != 0.0;
        double imp = impedance(m, rdist);
        double vel = 0;
        for (int k = 0; k < nv; k++) vel += Je[k] * d.v[k];
        chol_solve(LM, nv, Je, x.data());
        double A = 0;
        for (int k = 0; k < nv; k++) A += Je[k] * x[k];
        d.Ahat[row] = A;
        d.aref[row] = -bcoef * vel - kcoef * imp * rdist;
        double R = std::max(1e-15, (1 - imp) / imp * A);
        d.D[row] = 1.0 / R;
    };
    for (int ci = 0; ci < nc; ci++) {
        const Contact& c = d.con[ci];
        jacobian(m, d, c.b2, c.pos, jp2.data(), jr2.data());
        jacobian(m, d, c.b1, c.pos, jp1.data(), jr1.data());
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < nv; k++) {
                double acc = 0;
                for (int i = 0; i < 3; i++) acc += c.frame[3 * r + i] * (jp2[i * nv + k] - jp1[i * nv + k]);
                Jc[r * nv + k] = acc;
            }
        // torsional (about the normal) and rolling (about the tangents) rows: the frame's
        // components of the relative angular velocity, rows 3..5 of Jc
        if (c.dim >= 4)
            for (int r = 0; r < 3; r++)
                for (int k = 0; k < nv; k++) {
                    double acc = 0;
                    for (int i = 0; i < 3; i++) acc += c.frame[3 * r + i] * (jr2[i * nv + k] - jr1[i * nv + k]);
                    Jc[(3 + r) * nv + k] = acc;
                }
        double rdist = c.dist - std::max(m.gmargin[c.g1], m.gmargin[c.g2]);
        if (m.cone == 1 && c.dim >= 3) {
            // elliptic cone: the frame rows themselves (normal, t1, t2, then with condim 4 the
            // spin about n, with condim 6 also the rolling about t1 and t2); the normal row takes
            // the distance reference, the others none.  The cone is
            // {f : sum_i (f_i / mu_i)^2 <= f_n^2} with mu_i = mu on the tangents, mu_spin on the
            // spin and mu_roll on the rolling rows; friction row i's regulariser is
            // R_n mu^2 / (mu_i^2 impratio), which makes the cone circular in the rows' D-scaled
            // coordinates, of slope mu / sqrt(impratio) (for the tangents R_n / impratio)
            for (int e = 0; e < c.dim; e++) {
                int row = d.crow[ci] + e;
                std::copy(&Jc[e * nv], &Jc[e * nv] + nv, &d.J[(size_t)row * nv]);
                d.row_id[row] = e < 4 ? 4 * ci + e : 1024 + 6 * ci + (e - 4);
                d.ell[row] = 1;
                finish_row(row, e == 0 ? rdist : 0.0);
                if (e == 1 || e == 2) d.D[row] = d.D[d.crow[ci]] * m.impratio;
                if (e >= 3) {
                    const double r = c.mu > 0 ? (e == 3 ? c.mu_spin : c.mu_roll) / c.mu : 0.0;
                    d.D[row] = d.D[d.crow[ci]] * m.impratio * r * r;
                }
            }
            d.ell_row0.push_back(d.crow[ci]);
            d.ell_dim.push_back(c.dim);
            d.ell_mu.push_back(c.mu / std::sqrt(m.impratio));
            continue;
        }
        // pyramid row pairs J_n +- mu_d J_d over the friction directions d: sliding t1, t2
        // (mu), then spin about n (mu_spin), then rolling about t1, t2 (mu_roll)
        const int nrow_c = c.dim == 1 ? 1 : 2 * (c.dim - 1);
        for (int e = 0; e < nrow_c; e++) {
            int row = d.crow[ci] + e;
            int dir = e / 2;   // 0 t1, 1 t2, 2 spin, 3 roll t1, 4 roll t2
            int t = dir < 2 ? 1 + dir : dir + 1;
            double mu = dir < 2 ? c.mu : (dir == 2 ? c.mu_spin : c.mu_roll);
            double sgn = (e % 2 == 0) ? 1.0 : -1.0;
            double* Je = &d.J[(size_t)row * nv];
            for (int k = 0; k < nv; k++) Je[k] = Jc[k] + sgn * mu * Jc[t * nv + k];
            d.row_id[row] = e < 4 ? 4 * ci + e : 1024 + 6 * ci + (e - 4);
            finish_row(row, rdist);
        }
    }
    for (int l = 0; l < nl; l++) {
        int row = nr + l;
        d.J[(size_t)row * nv + ldof[l]] = lsgn[l];
        d.row_id[row] = 256 + ldof[l];
        finish_row(row, ldist[l]);
    }
    // equality rows: the anchor's world offset from its target (x, y, z), then for a weld the
    // rotation vector of R_body R_target' (x, y, z), each against the point or angular Jacobian
    int row = nr + nl;
    for (int q = 0; q < m.neq; q++) {
        const int b = m.eqbody[q];
        const double* R = &d.xmat[9 * b];
        double c[3];
        matvec3(R, &m.eqanchor[3 * q], c);
        for (int i = 0; i < 3; i++) c[i] += d.xpos[3 * b + i];
        jacobian(m, d, b, c, jp1.data(), jr1.data());
        const double* tgt = &m.eqtarget[7 * q];
        for (int k = 0; k < 3; k++, row++) {
            std::copy(&jp1[k * nv], &jp1[k * nv] + nv, &d.J[(size_t)row * nv]);
            d.row_id[row] = 512 + 6 * q + k;
            d.bilat[row] = 1;
            finish_row(row, c[k] - tgt[k]);
        }
        if (m.eqtype[q] != RBO_EQ_WELD) continue;
        double Rt[9], E[9];
        quat2mat(&tgt[3], Rt);
        for (int i = 0; i < 3; i++)   // E = R Rt'
            for (int j = 0; j < 3; j++) E[3 * i + j] = R[3 * i] * Rt[3 * j] + R[3 * i + 1] * Rt[3 * j + 1] + R[3 * i + 2] * Rt[3 * j + 2];
        double th[3];
        rotvec(E, th);
        for (int k = 0; k < 3; k++, row++) {
            std::copy(&jr1[k * nv], &jr1[k * nv] + nv, &d.J[(size_t)row * nv]);
            d.row_id[row] = 512 + 6 * q + 3 + k;
            d.bilat[row] = 1;
            finish_row(row, th[k]);
        }
    }
}

// ------------------------------------------------------------------------------------
// Soft elliptic cone of one contact.  The contact's force is the projection of -D jar onto the
// friction cone in the metric of the regulariser R = D^-1; with x = sqrt(D) jar the cone is the
// circular one of slope mu (mu the contact's scaled slope), and the cost is half the squared
// norm of the projection of -x onto it:
//   top zone, mu |x_t| <= x_n (separating): 0;
//   bottom zone, |x_t| <= -mu x_n (inside the cone): |x|^2 / 2 (every row active);
//   middle zone: (mu |x_t| - x_n)^2 / (2 (1 + mu^2)) (the force on the cone's surface).
// The contact has n = 3, 4 or 6 rows (normal first, x_t the rest).  Returns the zone (0 top, 1
// middle, 2 bottom); g = ds/djar [n], h = d2s/djar2 (n x n, row-major).
// ------------------------------------------------------------------------------------
int ell_eval(const double* jar, const double* D, double mu, int n, double* s, double* g, double* h) {
    double sq[6] = {0, 0, 0, 0, 0, 0}, x[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < n; a++) {
        sq[a] = std::sqrt(D[a]);
        x[a] = sq[a] * jar[a];
    }
    double T2 = 0;
    for (int a = 1; a < n; a++) T2 += x[a] * x[a];
    const double N = x[0], T = std::sqrt(T2);
    std::fill(g, g + n, 0.0);
    std::fill(h, h + n * n, 0.0);
    *s = 0;
    if (mu * T <= N) return 0;
    if (T <= -mu * N) {
        *s = 0.5 * (N * N + T2);
        for (int a = 0; a < n; a++) {
            g[a] = D[a] * jar[a];
            h[(n + 1) * a] = D[a];
        }
        return 2;
    }
    const double c = 1.0 / (1.0 + mu * mu), hh = mu * T - N;
    double u[6] = {0, 0, 0, 0, 0, 0}, w[6] = {-1.0, 0, 0, 0, 0, 0};   // w: gradient of hh in x
    for (int a = 1; a < n; a++) {
        u[a] = x[a] / T;
        w[a] = mu * u[a];
    }
    *s = 0.5 * c * hh * hh;
    for (int a = 0; a < n; a++) {
        g[a] = sq[a] * c * hh * w[a];
        for (int b = 0; b < n; b++) {
            // c (w w' + hh mu / T (I - u u') on the tangential block)
            double hx = w[a] * w[b];
            if (a > 0 && b > 0) hx += hh * mu / T * ((a == b ? 1.0 : 0.0) - u[a] * u[b]);
            h[n * a + b] = sq[a] * sq[b] * c * hx;
        }
    }
    return 1;
}

// ------------------------------------------------------------------------------------
// primal Newton solver on f(a) = 0.5 (a-a0)'M(a-a0) + sum_e 0.5 D_e min(J_e a - aref_e, 0)^2
// (bilateral rows: the whole residual; elliptic contacts: their cone cost above)
// ------------------------------------------------------------------------------------
double constraint_cost(const Data& d, const std::vector<double>& jar) {
    double f = 0;
    for (int e = 0; e < d.nrows; e++)
        if (!d.ell[e] && (jar[e] < 0 || d.bilat[e])) f += 0.5 * d.D[e] * jar[e] * jar[e];
    for (size_t k = 0; k < d.ell_row0.size(); k++) {
        const int r0 = d.ell_row0[k];
        double sc, g[6], h[36];
        ell_eval(&jar[r0], &d.D[r0], d.ell_mu[k], d.ell_dim[k], &sc, g, h);
        f += sc;
    }
    return f;
}

std::vector<double> residuals(const Model& m, const Data& d, const double* a) {
    std::vector<double> jar(d.nrows);
    for (int e = 0; e < d.nrows; e++) {
        double t = -d.aref[e];
        for (int k = 0; k < m.nv; k++) t += d.J[(size_t)e * m.nv + k] * a[k];
        jar[e] = t;
    }
    return jar;
}

double cost(const Model& m, const Data& d, const double* a) {
    int nv = m.nv;
    double f = 0;
    for (int r = 0; r < nv; r++)
        for (int s = 0; s < nv; s++) f += 0.5 * (a[r] - d.a0[r]) * d.M[r * nv + s] * (a[s] - d.a0[s]);
    return f + constraint_cost(d, residuals(m, d, a));
}

// exact minimiser over alpha >= 0 of the convex piecewise quadratic phi(alpha) = f(a + alpha p)
double line_search(const Model& m, const Data& d, const std::vector<double>& jar, const std::vector<double>& p,
                   int* nseg) {
    int nv = m.nv, nr = d.nrows;
    bool any = false;
    for (int k = 0; k < nv; k++) any |= (p[k] != 0);
    if (!any) return 0.0;
    std::vector<double> s(nr, 0.0), Mp(nv, 0.0);
    for (int e = 0; e < nr; e++)
        for (int k = 0; k < nv; k++) s[e] += d.J[(size_t)e * nv + k] * p[k];
    for (int r = 0; r < nv; r++)
        for (int k = 0; k < nv; k++) Mp[r] += d.M[r * nv + k] * p[k];
    double A0 = 0, B0 = 0;
    for (int k = 0; k < nv; k++) {
        A0 += p[k] * Mp[k];
        B0 += (d.a[k] - d.a0[k]) * Mp[k];
    }
    // breakpoints where a row switches on or off, in ascending order
    std::vector<std::pair<double, int>> bp;
    for (int e = 0; e < nr; e++)
        if (s[e] != 0 && !d.bilat[e]) {
            double al = -jar[e] / s[e];
            if (al > 0) bp.push_back({al, e});
        }
    std::sort(bp.begin(), bp.end());
    // rows active just to the right of alpha = 0
    std::vector<char> act(nr);
    for (int e = 0; e < nr; e++) act[e] = d.bilat[e] || (jar[e] < 0) || (jar[e] == 0 && s[e] < 0);
    size_t i = 0;
    while (true) {
        if (nseg) ++*nseg;
        double A = A0, B = B0;
        for (int e = 0; e < nr; e++)
            if (act[e]) {
                A += d.D[e] * s[e] * s[e];
                B += d.D[e] * s[e] * jar[e];
            }
        double root = -B / A;
        if (i == bp.size() || root <= bp[i].first) return std::max(root, 0.0);
        double here = bp[i].first;
        while (i < bp.size() && bp[i].first == here) {
            act[bp[i].second] = s[bp[i].second] < 0;  // s < 0: switches on; s > 0: switches off
            i++;
        }
    }
}

// Minimiser over alpha >= 0 of phi(alpha) = f(a + alpha p) when elliptic contacts make phi
// convex and continuously differentiable but not piecewise quadratic: Newton's method on
// phi'(alpha) = 0 safeguarded by the bracket [lo, hi] of a sign change (bisection when a Newton
// step leaves it), from alpha = 0, until |phi'| <= 1e-13 |phi'(0)| or the bracket closes.
double line_search_smooth(const Model& m, const Data& d, const std::vector<double>& jar,
                          const std::vector<double>& p, int* nseg) {
    int nv = m.nv, nr = d.nrows;
    std::vector<double> s(nr, 0.0), Mp(nv, 0.0);
    for (int e = 0; e < nr; e++)
        for (int k = 0; k < nv; k++) s[e] += d.J[(size_t)e * nv + k] * p[k];
    for (int r = 0; r < nv; r++)
        for (int k = 0; k < nv; k++) Mp[r] += d.M[r * nv + k] * p[k];
    double A0 = 0, B0 = 0;
    for (int k = 0; k < nv; k++) {
        A0 += p[k] * Mp[k];
        B0 += (d.a[k] - d.a0[k]) * Mp[k];
    }
    if (!(A0 > 0)) return 0.0;
    // phi'(alpha) and phi''(alpha) (the right derivative at zone changes)
    auto dphi = [&](double al, double* d2) {
        double d1 = al * A0 + B0;
        *d2 = A0;
        for (int e = 0; e < nr; e++) {
            if (d.ell[e]) continue;
            const double j = jar[e] + al * s[e];
            if (j < 0 || (j == 0 && s[e] < 0) || d.bilat[e]) {
                d1 += d.D[e] * s[e] * j;
                *d2 += d.D[e] * s[e] * s[e];
            }
        }
        for (size_t k = 0; k < d.ell_row0.size(); k++) {
            const int r0 = d.ell_row0[k], n = d.ell_dim[k];
            double j[6], sc, g[6], h[36];
            for (int a = 0; a < n; a++) j[a] = jar[r0 + a] + al * s[r0 + a];
            ell_eval(j, &d.D[r0], d.ell_mu[k], n, &sc, g, h);
            for (int a = 0; a < n; a++) {
                d1 += g[a] * s[r0 + a];
                for (int b = 0; b < n; b++) *d2 += s[r0 + a] * h[n * a + b] * s[r0 + b];
            }
        }
        return d1;
    };
    double d2, d1 = dphi(0.0, &d2);
    if (!(d1 < 0)) return 0.0;
    const double tolg = 1e-13 * std::fabs(d1);
    double lo = 0, hi = INFINITY, al = 0;
    for (int k = 0; k < 100; k++) {
        if (nseg) ++*nseg;
        if (std::fabs(d1) <= tolg) break;
        if (d1 < 0) lo = al; else hi = al;
        if (std::isfinite(hi) && hi - lo <= 1e-15 * hi) break;
        double nxt = al - d1 / d2;
        if (!(nxt > lo && nxt < hi)) nxt = std::isfinite(hi) ? 0.5 * (lo + hi) : 2 * std::max(lo, 1.0);
        al = nxt;
        d1 = dphi(al, &d2);
    }
    return al;
}

void newton(const Model& m, Data& d) {
    int nv = m.nv, nr = d.nrows;
    int maxiter = m.mode == 1 ? 100 : m.iters;
    double tol = m.mode == 1 ? 1e-12 : m.tol;
    double scale = m.meaninertia * nv;
    d.niter = 0;
    d.itercap = false;
    d.a = d.a0;
    d.segments = 0;
    d.active_final = 0;
    std::fill(d.fp, d.fp + RBO_FPITER, 0u);
    d.act_iter.clear();
    if (nr == 0) {
        d.efc_force.assign(0, 0.0);
        d.cost = 0;
        return;
    }
    if (cost(m, d, d.aws.data()) < cost(m, d, d.a0.data())) d.a = d.aws;
    std::vector<double> jar(nr), g(nv), H(nv * nv), LH, p(nv), anew(nv);
    bool stopped = false;
    for (int it = 0; it < maxiter; it++) {
        for (int e = 0; e < nr; e++) {
            double t = -d.aref[e];
            for (int k = 0; k < nv; k++) t += d.J[(size_t)e * nv + k] * d.a[k];
            jar[e] = t;
        }
        for (int r = 0; r < nv; r++) {
            double t = 0;
            for (int k = 0; k < nv; k++) t += d.M[r * nv + k] * (d.a[k] - d.a0[k]);
            g[r] = t;
        }
        H = d.M;
        for (int e = 0; e < nr; e++) {
            if (d.ell[e] || (!(jar[e] < 0) && !d.bilat[e])) continue;
            const double* Je = &d.J[(size_t)e * nv];
            for (int r = 0; r < nv; r++) {
                g[r] += d.D[e] * jar[e] * Je[r];
                for (int k = 0; k < nv; k++) H[r * nv + k] += d.D[e] * Je[r] * Je[k];
            }
        }
        // elliptic contacts: J_c' ds/djar and J_c' h J_c over their rows
        std::vector<int> ell_zone(d.ell_row0.size());
        for (size_t c = 0; c < d.ell_row0.size(); c++) {
            const int r0 = d.ell_row0[c], n = d.ell_dim[c];
            double sc, ge[6], he[36];
            ell_zone[c] = ell_eval(&jar[r0], &d.D[r0], d.ell_mu[c], n, &sc, ge, he);
            for (int a = 0; a < n; a++) {
                const double* Ja = &d.J[(size_t)(r0 + a) * nv];
                for (int r = 0; r < nv; r++) g[r] += ge[a] * Ja[r];
                for (int b = 0; b < n; b++) {
                    const double* Jb = &d.J[(size_t)(r0 + b) * nv];
                    if (he[n * a + b] == 0) continue;
                    for (int r = 0; r < nv; r++)
                        for (int k = 0; k < nv; k++) H[r * nv + k] += he[n * a + b] * Ja[r] * Jb[k];
                }
            }
        }
        double gn = 0;
        for (int k = 0; k < nv; k++) gn += g[k] * g[k];
        if (std::sqrt(gn) / scale < tol) { stopped = true; break; }
        // record the active set this update is built from
        // (an elliptic contact's rows are active unless it is in its top zone; inside the cone
        // they enter the fingerprint as 2048 + id, so that its zone is recorded too)
        std::vector<int> act;
        uint32_t fp = 0;
        auto ell_zone_of = [&](int e) {
            for (size_t c = 0; c < d.ell_row0.size(); c++)
                if (e >= d.ell_row0[c] && e < d.ell_row0[c] + d.ell_dim[c]) return ell_zone[c];
            return 0;
        };
        for (int e = 0; e < nr; e++) {
            const int zone = d.ell[e] ? ell_zone_of(e) : 0;
            if (d.ell[e] ? zone != 0 : (jar[e] < 0 || d.bilat[e])) {
                act.push_back(e);
                fp += ((uint32_t)d.row_id[e] + (zone == 2 ? 2048u : 0u) + 1u) * 2654435761u;
            }
        }
        if (it < RBO_FPITER) d.fp[it] = fp;
        d.act_iter.push_back(act);
        if (!cholesky(H, nv, LH)) { stopped = true; break; }
        std::vector<double> ng(nv);
        for (int k = 0; k < nv; k++) ng[k] = -g[k];
        chol_solve(LH, nv, ng.data(), p.data());
        double alpha = d.ell_row0.empty() ? line_search(m, d, jar, p, &d.segments)
                                          : line_search_smooth(m, d, jar, p, &d.segments);
        double fold = cost(m, d, d.a.data());
        for (int k = 0; k < nv; k++) anew[k] = d.a[k] + alpha * p[k];
        double fnew = cost(m, d, anew.data());
        d.a = anew;
        d.niter = it + 1;
        // (the converged mode stops on the gradient alone: with elliptic cones the cost is not
        // piecewise quadratic, and a small improvement does not yet mean a small gradient)
        if (m.mode != 1 && (fold - fnew) / scale < tol) { stopped = true; break; }
    }
    d.itercap = !stopped && maxiter > 0;
    d.cost = cost(m, d, d.a.data());
    d.efc_force.assign(nr, 0.0);
    const std::vector<double> jf = residuals(m, d, d.a.data());
    for (int e = 0; e < nr; e++) {
        if (d.ell[e]) continue;
        const double t = jf[e];
        d.efc_force[e] = -d.D[e] * (d.bilat[e] ? t : std::min(t, 0.0));
        d.active_final += t < 0 || d.bilat[e];
    }
    for (size_t c = 0; c < d.ell_row0.size(); c++) {
        const int r0 = d.ell_row0[c], n = d.ell_dim[c];
        double sc, ge[6], he[36];
        const int zone = ell_eval(&jf[r0], &d.D[r0], d.ell_mu[c], n, &sc, ge, he);
        for (int a = 0; a < n; a++) d.efc_force[r0 + a] = -ge[a];
        d.active_final += zone != 0 ? n : 0;
    }
}

// ------------------------------------------------------------------------------------
// operation counts of one substep (work outputs; a multiply-add counts 2).  Unit costs of the
// small kernels used throughout: 3x3 matrix-vector 15, 3x3 matrix product 45, quaternion
// product 28, quaternion to matrix 39, cross product 9, dot product 5, spatial inertia times
// motion vector 45, spatial cross product 30, spatial dot product 11.
// ------------------------------------------------------------------------------------
enum { ST_KIN, ST_DYN, ST_FAC, ST_COL, ST_ROW, ST_NEWTON, ST_INT };

double chol_ops(int n) {   // cholesky(): per column j, 2j + 1 for the diagonal, 2j + 1 per row below
    double f = 0;
    for (int j = 0; j < n; j++) f += 2.0 * j + 1 + (double)(n - 1 - j) * (2.0 * j + 1);
    return f;
}

// primitive tests of the collision pairs (plane-sphere, plane-capsule ends, plane-box vertices,
// sphere-box closest point, box-box separating axes and clipping) and per contact its frame
double collision_ops(const Model& m, const Data& d) {
    double f = 0;
    for (int a = 0; a < m.ngeom; a++)
        for (int b = a + 1; b < m.ngeom; b++) {
            if (!pair_allowed(m, a, b)) continue;
            int t1 = std::min(m.gtype[a], m.gtype[b]), t2 = std::max(m.gtype[a], m.gtype[b]);
            if (t2 == RBO_GEOM_HFIELD) f += (t1 == RBO_GEOM_SPHERE ? 1 : t1 == RBO_GEOM_CAPSULE ? 2 : 8) * 90;
            else if (t1 == RBO_GEOM_PLANE) f += t2 == RBO_GEOM_SPHERE ? 20 : (t2 == RBO_GEOM_CAPSULE ? 60 : 8 * 25);
            else if (t1 == RBO_GEOM_SPHERE) f += 80;
            else if (t1 == RBO_GEOM_CAPSULE) f += 2 * 80 + 12;
            else f += 15 * 40 + 300;
        }
    return f + 25.0 * d.con.size();
}

void count_ops(const Model& m, const Data& d, double* plain, double* tree) {
    const int nv = m.nv, nb = m.nbody, nr = d.nrows, nc = (int)d.con.size();
    int nh = 0, nf = 0;
    for (int j = 0; j < m.njnt; j++) (m.jtype[j] == RBO_JNT_HINGE ? nh : nf)++;
    double nM = 0, sumcd = 0, ldl = 0;
    for (int i = 0; i < nv; i++) {
        nM += m.dof_depth[i];
        ldl += (double)(m.dof_depth[i] - 1) * m.dof_depth[i] + m.dof_depth[i];
    }
    for (int b = 1; b < nb; b++) sumcd += m.body_cdepth[b];
    const double tsolve = 4 * (nM - nv) + nv, symmul = 4 * nM - 2 * nv, bmot = 12 * sumcd;
    // stage 0, kinematics (one body at a time in either formulation): parent composition, the
    // hinge's anchored rotation or the free joint's normalisation, rotation matrix; per body the
    // centre of mass, mass and world inertia; per geom its pose
    double kin = 46.0 * (nb - 1) + 163.0 * nh + 12.0 * nf + 39.0 * (nb - 1) + 211.0 * nb + 102.0 * m.ngeom;
    plain[ST_KIN] += kin;
    tree[ST_KIN] += kin;
    // stage 1: plain -- per body its Jacobians (12 per hinge, 30 per free joint on the chain),
    // m Jp'Jp + Jr' I Jr over all dof pairs, the bias wrench and its projection
    double jac = 0;
    for (int b = 1; b < nb; b++)
        for (int bb = b; bb > 0; bb = m.parent[bb])
            if (m.body_jnt[bb] >= 0) jac += m.jtype[m.body_jnt[bb]] == RBO_JNT_HINGE ? 12 : 30;
    plain[ST_DYN] += 2 * jac + (nb - 1) * (15.0 * nv + 16.0 * nv * nv + 12.0 * nv + 45) + 90.0 * nh + 39.0 * nf + nh;
    // tree: spatial inertias about a common origin, motion subspaces, recursive Newton-Euler
    // (forward velocities and accelerations, body forces, backward sums, projection) and the
    // composite-rigid-body rows M_ij = S_j . (Ic_i S_i) over each dof's chain
    double crba = 0;
    for (int i = 0; i < nv; i++) crba += 45 + 11.0 * m.dof_depth[i] + 1;
    tree[ST_DYN] += 33.0 * (nb - 1) + 42.0 * nh + 27.0 * nf + 54.0 * nh + 198.0 * nf + 126.0 * (nb - 1) + 16.0 * (nb - 1) +
                    11.0 * nv + crba;
    // stage 2: factorisation of M and a0 = M^-1 (tau - c)
    plain[ST_FAC] += chol_ops(nv) + 2.0 * nv * nv + nv;
    tree[ST_FAC] += ldl + tsolve + nv;
    // stage 3: collision
    const double col = collision_ops(m, d);
    plain[ST_COL] += col;
    tree[ST_COL] += col;
    // stage 4: constraint rows.  plain: per contact two point Jacobians and the frame product, per
    // row its Jacobian, velocity, A-hat by a dense solve, impedance, aref and D.  tree: per
    // contact the point-velocity Jacobian over the dofs it touches (27 per dof), the 3x3 block of
    // J M^-1 J' by three half-solves over the chain, the pyramid combinations; per limit row one
    // half-solve
    double rows_plain = 0, rows_tree = 0;
    for (int ci = 0; ci < nc; ci++) {
        const Contact& c = d.con[ci];
        double jc = 0;
        for (int body : {c.b1, c.b2})
            for (int bb = body; bb > 0; bb = m.parent[bb])
                if (m.body_jnt[bb] >= 0) jc += m.jtype[m.body_jnt[bb]] == RBO_JNT_HINGE ? 12 : 30;
        rows_plain += jc + 27.0 * nv;
        const double dd = d.row_nnz[d.crow[ci]];
        rows_tree += 27 * dd + 3 * dd * (dd - 1) + 16 * dd + 24 + 15 + 44 + 20;
    }
    for (int e = 0; e < nr; e++) {
        rows_plain += (d.row_id[e] >= 256 ? 4.0 * nv : 7.0 * nv) + 2.0 * nv * nv + 26;
        if (d.row_id[e] >= 256) rows_tree += d.row_nnz[e] * (d.row_nnz[e] - 1.0) + 3.0 * d.row_nnz[e] + 26;
    }
    plain[ST_ROW] += rows_plain;
    tree[ST_ROW] += rows_tree;
    // stage 5: Newton.  plain: costs, residuals, gradient and Hessian over all dofs, dense
    // Cholesky and solves, the line search's products and segments.  tree: body motions and
    // packed products through the tree, per active row its gradient and Hessian entries over
    // the dofs it touches, the no-fill-in L'DL and its solves, per segment the active rows' sums
    if (nr > 0) {
        const double cost = 6.0 * nv * nv + nr * (2.0 * nv + 5);
        const int nit = (int)d.act_iter.size();
        double pl = 3 * cost + nr * (2.0 * nv + 3);
        double tr = 2 * bmot + 2 * 20.0 * nc + 8.0 * nr + symmul + 4.0 * nv;
        for (int it = 0; it < nit; it++) {
            pl += nr * 2.0 * nv + 3.0 * nv * nv + 2.0 * nv + chol_ops(nv) + nv + 2.0 * nv * nv;   // jar, g, |g|, H, p
            pl += nr * 2.0 * nv + 2.0 * nv * nv + 5.0 * nv + nr + 2.0 * nv + 2 * cost;             // line search, update
            double hess = 0;
            for (int e : d.act_iter[it]) {
                pl += 3.0 * nv + 3.0 * nv * nv;
                const double dd = d.row_nnz[e];
                hess += 4 * dd + dd * (dd + 1);
            }
            double jrows = 0;
            for (int ci = 0; ci < nc; ci++) jrows += 27.0 * d.row_nnz[d.crow[ci]];
            tr += jrows + hess + nM + 2.0 * nv + ldl + tsolve;                     // gradient, Hessian, p
            tr += symmul + bmot + 20.0 * nc + 4.0 * nv + nr + 6.0 * nv + 6.0 * nr;  // line search, update
        }
        // every examined segment sums the active rows' quadratic coefficients
        pl += d.segments * (6.0 * nr + 2);
        tr += d.segments * (6.0 * nr + 2);
        plain[ST_NEWTON] += pl;
        tree[ST_NEWTON] += tr;
    }
    // stage 6: semi-implicit Euler
    const double integ = 2.0 * nv + 2.0 * nh + 64.0 * nf;
    plain[ST_INT] += integ;
    tree[ST_INT] += integ;
}

// ------------------------------------------------------------------------------------
// one substep without integration: actuation, kinematics, dynamics, collision, solve
// ------------------------------------------------------------------------------------
void forward(const Model& m, Data& d) {
    actuation(m, d);
    passive(m, d);
    kinematics(m, d);
    mass_matrix(m, d);
    bias_forces(m, d);
    std::vector<double> LM;
    if (!cholesky(d.M, m.nv, LM)) {
        std::fill(d.a0.begin(), d.a0.end(), NAN);
        d.a = d.a0;
        d.con.clear();
        d.nrows = 0;
        return;
    }
    std::vector<double> rhs(m.nv);
    for (int k = 0; k < m.nv; k++) rhs[k] = d.tau[k] - d.c[k];
    chol_solve(LM, m.nv, rhs.data(), d.a0.data());
    collide(m, d);
    make_rows(m, d, LM);
    newton(m, d);
    d.cforce.assign(3 * d.con.size(), 0.0);
    for (size_t ci = 0; ci < d.con.size(); ci++) {
        const double* f = &d.efc_force[d.crow[ci]];
        double mu = d.con[ci].mu;
        if (d.con[ci].dim == 1) {
            d.cforce[3 * ci] = f[0];
            continue;
        }
        if (m.cone == 1) {   // elliptic: the rows' forces are the frame components
            for (int a = 0; a < 3; a++) d.cforce[3 * ci + a] = f[a];
            continue;
        }
        // every pyramid row carries the normal direction once
        double fn = 0;
        for (int e = 0; e < 2 * (d.con[ci].dim - 1); e++) fn += f[e];
        d.cforce[3 * ci] = fn;
        d.cforce[3 * ci + 1] = mu * (f[0] - f[1]);
        d.cforce[3 * ci + 2] = mu * (f[2] - f[3]);
    }
    // Damping integrated implicitly: the step applies a_int = (M + dt B)^-1 M a, B the diagonal
    // of joint dampings -- the damping force taken at the end-of-step velocity, to first order
    // (M a is the total force the solution carries: applied, passive, bias and constraint)
    d.aint = d.a;
    if (m.ndamp > 0) {
        const int nv = m.nv;
        std::vector<double> H = d.M, LH, Ma(nv, 0.0);
        for (int j = 0; j < m.njnt; j++)
            if (m.jdamp[j] > 0) H[m.jdadr[j] * (nv + 1)] += m.dt * m.jdamp[j];
        for (int r = 0; r < nv; r++)
            for (int k = 0; k < nv; k++) Ma[r] += d.M[r * nv + k] * d.a[k];
        if (cholesky(H, nv, LH)) chol_solve(LH, nv, Ma.data(), d.aint.data());
        else std::fill(d.aint.begin(), d.aint.end(), NAN);
    }
}

// semi-implicit Euler: v' = v + dt a; hinge q' = q + dt v'; free pos += dt v'_lin,
// quat' = normalise(quat * exp(dt w'_local / 2))
void integrate(const Model& m, const double* q, const double* v, const double* a, double* qo, double* vo) {
    double dt = m.dt;
    for (int k = 0; k < m.nv; k++) vo[k] = v[k] + dt * a[k];
    for (int j = 0; j < m.njnt; j++) {
        int qa = m.jqadr[j], da = m.jdadr[j];
        if (m.jtype[j] == RBO_JNT_HINGE) {
            qo[qa] = q[qa] + dt * vo[da];
        } else {
            for (int i = 0; i < 3; i++) qo[qa + i] = q[qa + i] + dt * vo[da + i];
            double th[3] = {dt * vo[da + 3], dt * vo[da + 4], dt * vo[da + 5]};
            double ang = std::sqrt(dot3(th, th));
            double dq[4] = {1, 0, 0, 0};
            if (ang > 0) {
                double u[3] = {th[0] / ang, th[1] / ang, th[2] / ang};
                axisangle2quat(u, ang, dq);
            }
            double qq[4];
            quatmul(&q[qa + 3], dq, qq);
            quatnormalize(qq);
            for (int i = 0; i < 4; i++) qo[qa + 3 + i] = qq[i];
        }
    }
}

bool all_finite(const double* x, int n) {
    for (int i = 0; i < n; i++)
        if (!std::isfinite(x[i])) return false;
    return true;
}

void load_world(const Model& m, Data& d, const double* q, const double* v, const double* ctrl, const double* aws,
                const double* fr, const double* ms) {
    std::copy(q, q + m.nq, d.q.begin());
    std::copy(v, v + m.nv, d.v.begin());
    if (m.nu) std::copy(ctrl, ctrl + m.nu, d.ctrl.begin());
    if (aws)
        std::copy(aws, aws + m.nv, d.aws.begin());
    else
        std::fill(d.aws.begin(), d.aws.end(), 0.0);
    d.fr = fr ? *fr : 1.0;
    if (ms && m.ms_pw)
        std::copy(ms, ms + m.nbody, d.ms.begin());
    else
        std::fill(d.ms.begin(), d.ms.end(), 1.0);
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================
extern "C" {

const char* rbo_last_error(void) { return g_err.c_str(); }

int rbo_model_create(const rbo_desc* dsc, void** out) {
    if (!dsc || !out) return fail("null argument");
    Model* m = new Model();
    Model& M = *m;
    M.nbody = dsc->nbody; M.njnt = dsc->njnt; M.ngeom = dsc->ngeom; M.nu = dsc->nu;
    int nb = M.nbody, nj = M.njnt, ng = M.ngeom, nu = M.nu;
    auto bad = [&](const std::string& s) { delete m; return fail(s); };
    if (nb < 1 || nj < 0 || ng < 0 || nu < 0) return bad("bad sizes");
    M.parent.assign(dsc->body_parent, dsc->body_parent + nb);
    M.bpos.assign(dsc->body_pos, dsc->body_pos + 3 * nb);
    M.bquat.assign(dsc->body_quat, dsc->body_quat + 4 * nb);
    M.ipos.assign(dsc->body_ipos, dsc->body_ipos + 3 * nb);
    M.iquat.assign(dsc->body_iquat, dsc->body_iquat + 4 * nb);
    M.mass.assign(dsc->body_mass, dsc->body_mass + nb);
    M.inertia.assign(dsc->body_inertia, dsc->body_inertia + 3 * nb);
    for (int b = 1; b < nb; b++)
        if (M.parent[b] < 0 || M.parent[b] >= b) return bad("body parent must precede the body");
    M.body_jnt.assign(nb, -1);
    if (nj) {
        M.jtype.assign(dsc->jnt_type, dsc->jnt_type + nj);
        M.jbody.assign(dsc->jnt_body, dsc->jnt_body + nj);
        M.jpos.assign(dsc->jnt_pos, dsc->jnt_pos + 3 * nj);
        M.jaxis.assign(dsc->jnt_axis, dsc->jnt_axis + 3 * nj);
        M.jarm.assign(dsc->jnt_armature, dsc->jnt_armature + nj);
    }
    M.jrange.assign(2 * nj, 0.0);
    if (dsc->jnt_range) M.jrange.assign(dsc->jnt_range, dsc->jnt_range + 2 * nj);
    M.jlimited.assign(nj, 0);
    M.nlim = 0;
    M.jdamp.assign(nj, 0.0);
    if (dsc->jnt_damping) M.jdamp.assign(dsc->jnt_damping, dsc->jnt_damping + nj);
    M.ndamp = 0;
    for (int j = 0; j < nj; j++) {
        if (!(std::isfinite(M.jdamp[j]) && M.jdamp[j] >= 0)) return bad("joint damping must be finite and >= 0");
        M.ndamp += M.jdamp[j] > 0;
    }
    M.jqadr.assign(nj, 0); M.jdadr.assign(nj, 0);
    // joints must be listed in body order so dof order follows body order
    int qa = 0, da = 0, lastb = 0;
    for (int j = 0; j < nj; j++) {
        int b = M.jbody[j];
        if (b <= 0 || b >= nb) return bad("joint on invalid body");
        if (M.body_jnt[b] >= 0) return bad("more than one joint on a body");
        if (b < lastb) return bad("joints must be listed in body order");
        lastb = b;
        M.body_jnt[b] = j;
        M.jqadr[j] = qa; M.jdadr[j] = da;
        if (M.jtype[j] == RBO_JNT_FREE) {
            if (M.parent[b] != 0) return bad("free joint must be on a child of the world");
            qa += 7; da += 6;
            if (M.jrange[2 * j] != M.jrange[2 * j + 1]) return bad("free joints take no range");
            if (M.jdamp[j] != 0) return bad("free joints take no damping");
        } else if (M.jtype[j] == RBO_JNT_HINGE) {
            qa += 1; da += 1;
            const double lo = M.jrange[2 * j], hi = M.jrange[2 * j + 1];
            if (!(std::isfinite(lo) && std::isfinite(hi)) || lo > hi) return bad("joint range must be finite with lower <= upper");
            M.jlimited[j] = lo < hi;
            M.nlim += M.jlimited[j];
            double* ax = &M.jaxis[3 * j];
            double n = std::sqrt(dot3(ax, ax));
            if (!(n > 0)) return bad("zero hinge axis");
            for (int i = 0; i < 3; i++) ax[i] /= n;
        } else {
            return bad("unknown joint type");
        }
    }
    M.nq = qa; M.nv = da;
    for (int b = 0; b < nb; b++) {
        double* q = &M.bquat[4 * b];
        double nrm = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (std::fabs(nrm - 1) > 1e-6) return bad("body quaternion not unit");
        if (b > 0 && !(M.mass[b] > 0)) return bad("non-positive body mass");
        const double* I = &M.inertia[3 * b];
        if (b > 0 && (I[0] + I[1] < I[2] * (1 - 1e-12) || I[1] + I[2] < I[0] * (1 - 1e-12) || I[0] + I[2] < I[1] * (1 - 1e-12) ||
                      !(I[0] > 0 && I[1] > 0 && I[2] > 0)))
            return bad("inertia violates the triangle inequality");
    }
    M.movable.assign(nb, 0);
    for (int b = 1; b < nb; b++) M.movable[b] = M.movable[M.parent[b]] || M.body_jnt[b] >= 0;
    M.body_cdepth.assign(nb, 0);
    M.dof_depth.assign(M.nv, 0);
    for (int b = 1; b < nb; b++) {
        int e = M.body_cdepth[M.parent[b]];
        int j = M.body_jnt[b];
        if (j >= 0) {
            int nd = M.jtype[j] == RBO_JNT_FREE ? 6 : 1;
            for (int k = 0; k < nd; k++) M.dof_depth[M.jdadr[j] + k] = e + k + 1;
            e += nd;
        }
        M.body_cdepth[b] = e;
    }
    if (ng) {
        M.gtype.assign(dsc->geom_type, dsc->geom_type + ng);
        M.gbody.assign(dsc->geom_body, dsc->geom_body + ng);
        M.gcontype.assign(dsc->geom_contype, dsc->geom_contype + ng);
        M.gconaff.assign(dsc->geom_conaffinity, dsc->geom_conaffinity + ng);
        M.gpos.assign(dsc->geom_pos, dsc->geom_pos + 3 * ng);
        M.gquat.assign(dsc->geom_quat, dsc->geom_quat + 4 * ng);
        M.gsize.assign(dsc->geom_size, dsc->geom_size + 3 * ng);
        M.gfric.assign(dsc->geom_friction, dsc->geom_friction + ng);
        M.gmargin.assign(dsc->geom_margin, dsc->geom_margin + ng);
    }
    M.gcondim.assign(ng, 3);
    if (dsc->geom_condim) M.gcondim.assign(dsc->geom_condim, dsc->geom_condim + ng);
    for (int g = 0; g < ng; g++)
        if (M.gcondim[g] != 1 && M.gcondim[g] != 3 && M.gcondim[g] != 4 && M.gcondim[g] != 6)
            return bad("geom condim must be 1, 3, 4 or 6");
    M.gfric_spin.assign(ng, 0.005);
    M.gfric_roll.assign(ng, 0.0001);
    if (dsc->geom_friction_spin) M.gfric_spin.assign(dsc->geom_friction_spin, dsc->geom_friction_spin + ng);
    if (dsc->geom_friction_roll) M.gfric_roll.assign(dsc->geom_friction_roll, dsc->geom_friction_roll + ng);
    for (int g = 0; g < ng; g++)
        if (!(M.gfric_spin[g] >= 0 && M.gfric_roll[g] >= 0 && std::isfinite(M.gfric_spin[g]) &&
              std::isfinite(M.gfric_roll[g])))
            return bad("torsional and rolling friction must be finite and >= 0");
    bool any_hf = false;
    for (int g = 0; g < ng; g++) {
        if (M.gtype[g] < 0 || M.gtype[g] > 4) return bad("unknown geom type");
        if (M.gbody[g] < 0 || M.gbody[g] >= nb) return bad("geom on invalid body");
        if (M.gtype[g] == RBO_GEOM_PLANE && M.movable[M.gbody[g]]) return bad("planes must be static");
        if (M.gtype[g] == RBO_GEOM_HFIELD) {
            if (M.movable[M.gbody[g]]) return bad("height fields must be static");
            if (!(M.gsize[3 * g] > 0 && M.gsize[3 * g + 1] > 0)) return bad("height field extents must be positive");
            any_hf = true;
        }
    }
    if (any_hf) {
        if (dsc->hfield_nrow < 2 || dsc->hfield_ncol < 2 || !dsc->hfield_data) return bad("height field grid missing");
        M.hf_nrow = dsc->hfield_nrow;
        M.hf_ncol = dsc->hfield_ncol;
        M.hf.assign(dsc->hfield_data, dsc->hfield_data + (size_t)M.hf_nrow * M.hf_ncol);
        for (double h : M.hf)
            if (!std::isfinite(h)) return bad("height field heights must be finite");
    }
    M.neq = dsc->neq;
    if (M.neq < 0 || (M.neq > 0 && (!dsc->eq_type || !dsc->eq_body || !dsc->eq_anchor || !dsc->eq_target)))
        return bad("equality constraints missing");
    for (int q = 0; q < M.neq; q++) {
        const int t = dsc->eq_type[q], b = dsc->eq_body[q];
        if (t != RBO_EQ_CONNECT && t != RBO_EQ_WELD) return bad("unknown equality type");
        if (b <= 0 || b >= nb || !M.movable[b]) return bad("an equality constraint needs a moving body");
        const double* tq = dsc->eq_target + 7 * q + 3;
        if (t == RBO_EQ_WELD && std::fabs(std::sqrt(tq[0] * tq[0] + tq[1] * tq[1] + tq[2] * tq[2] + tq[3] * tq[3]) - 1) > 1e-6)
            return bad("weld target quaternion not unit");
        for (int i = 0; i < 10; i++)
            if (!std::isfinite(i < 3 ? dsc->eq_anchor[3 * q + i] : dsc->eq_target[7 * q + i - 3]))
                return bad("equality constraint values must be finite");
    }
    M.eqtype.assign(dsc->eq_type, dsc->eq_type + M.neq);
    M.eqbody.assign(dsc->eq_body, dsc->eq_body + M.neq);
    M.eqanchor.assign(dsc->eq_anchor, dsc->eq_anchor + 3 * M.neq);
    M.eqtarget.assign(dsc->eq_target, dsc->eq_target + 7 * M.neq);
    M.maxcon = 0; M.npair = 0; M.maxconrows = 0;
    for (int a = 0; a < ng; a++)
        for (int b = a + 1; b < ng; b++) {
            if (!pair_allowed(M, a, b)) continue;
            int t1 = std::min(M.gtype[a], M.gtype[b]), t2 = std::max(M.gtype[a], M.gtype[b]);
            int cap = pair_capacity(t1, t2);
            if (cap < 0) return bad("unsupported collision pair type");
            M.maxcon += cap;
            const int dim = std::max(M.gcondim[a], M.gcondim[b]);
            M.maxconrows += cap * (dim == 1 ? 1 : 2 * (dim - 1));
            M.npair++;
        }
    if (nu) {
        M.atype.assign(dsc->act_type, dsc->act_type + nu);
        M.ajoint.assign(dsc->act_joint, dsc->act_joint + nu);
        M.akp.assign(dsc->act_kp, dsc->act_kp + nu);
        M.akd.assign(dsc->act_kd, dsc->act_kd + nu);
        M.agear.assign(dsc->act_gear, dsc->act_gear + nu);
    }
    for (int u = 0; u < nu; u++) {
        if (M.ajoint[u] < 0 || M.ajoint[u] >= nj) return bad("actuator on invalid joint");
        if (M.jtype[M.ajoint[u]] != RBO_JNT_HINGE) return bad("actuators drive hinge joints only");
        if (M.atype[u] != RBO_ACT_POSITION && M.atype[u] != RBO_ACT_MOTOR) return bad("unknown actuator type");
    }
    M.dt = dsc->timestep; M.K = dsc->nsubsteps;
    for (int i = 0; i < 3; i++) M.grav[i] = dsc->gravity[i];
    M.iters = dsc->iterations; M.tol = dsc->tolerance;
    for (int i = 0; i < 2; i++) M.solref[i] = dsc->solref[i];
    for (int i = 0; i < 5; i++) M.solimp[i] = dsc->solimp[i];
    M.fr_pw = dsc->friction_per_world != 0;
    M.ms_pw = dsc->mass_scale_per_world != 0;
    if (!(M.dt > 0) || M.K < 1 || M.iters < 0) return bad("bad options");
    M.cone = dsc->cone;
    M.impratio = dsc->impratio;
    if (M.cone != 0 && M.cone != 1) return bad("cone must be pyramidal (0) or elliptic (1)");
    if (!(M.impratio > 0) || !std::isfinite(M.impratio)) return bad("impratio must be positive");
    if (M.cone == 1)
        for (int g = 0; g < ng; g++)
            if (M.gcondim[g] != 1 && M.gcondim[g] != 3 && M.gcondim[g] != 4 && M.gcondim[g] != 6)
                return bad("elliptic cones take condim 1, 3, 4 or 6");
    // mean diagonal inertia at the reference configuration (free joints at their body pose)
    if (M.nv > 0) {
        Data d(&M);
        for (int j = 0; j < nj; j++) {
            if (M.jtype[j] == RBO_JNT_FREE) {
                int b = M.jbody[j];
                for (int i = 0; i < 3; i++) d.q[M.jqadr[j] + i] = M.bpos[3 * b + i];
                for (int i = 0; i < 4; i++) d.q[M.jqadr[j] + 3 + i] = M.bquat[4 * b + i];
            }
        }
        kinematics(M, d);
        mass_matrix(M, d);
        double tr = 0;
        for (int k = 0; k < M.nv; k++) tr += d.M[k * (M.nv + 1)];
        M.meaninertia = tr / M.nv;
    }
    *out = m;
    return 0;
}

void rbo_model_destroy(void* m) { delete static_cast<Model*>(m); }

int rbo_model_info(const void* mp, rbo_info* out) {
    if (!mp || !out) return fail("null argument");
    const Model& m = *static_cast<const Model*>(mp);
    out->nq = m.nq; out->nv = m.nv; out->nu = m.nu; out->nbody = m.nbody; out->ngeom = m.ngeom;
    int neqrows = 0;
    for (int q = 0; q < m.neq; q++) neqrows += m.eqtype[q] == RBO_EQ_WELD ? 6 : 3;
    out->maxcon = m.maxcon; out->maxrows = m.maxconrows + m.nlim + neqrows; out->npair = m.npair;
    out->meaninertia = m.meaninertia;
    return 0;
}

int rbo_set_mode(void* mp, int32_t mode) {
    if (!mp || (mode != 0 && mode != 1)) return fail("bad mode");
    static_cast<Model*>(mp)->mode = mode;
    return 0;
}

int rbo_forward(const void* mp, const double* qpos, const double* qvel, const double* ctrl, const double* qacc_ws,
                const double* friction, const double* mass_scale, rbo_taps* t) {
    if (!mp || !qpos || !qvel) return fail("null argument");
    const Model& m = *static_cast<const Model*>(mp);
    Data d(&m);
    std::vector<double> zero(m.nu, 0.0);
    load_world(m, d, qpos, qvel, ctrl ? ctrl : zero.data(), qacc_ws, friction, mass_scale);
    forward(m, d);
    if (!t) return 0;
    int nb = m.nbody, ng = m.ngeom, nc = (int)d.con.size();
    auto put = [](double* dst, const std::vector<double>& src) {
        if (dst) std::copy(src.begin(), src.end(), dst);
    };
    put(t->xpos, d.xpos); put(t->xquat, d.xquat); put(t->xmat, d.xmat); put(t->com, d.com);
    put(t->gpos, d.gx); put(t->gmat, d.gR);
    put(t->M, d.M); put(t->bias, d.c); put(t->tau, d.tau); put(t->a0, d.a0);
    put(t->qacc, d.a);
    (void)nb; (void)ng;
    if (t->ncon) *t->ncon = nc;
    for (int ci = 0; ci < nc; ci++) {
        const Contact& c = d.con[ci];
        if (t->geom) { t->geom[2 * ci] = c.g1; t->geom[2 * ci + 1] = c.g2; }
        if (t->feature) t->feature[ci] = c.feature;
        if (t->dist) t->dist[ci] = c.dist;
        if (t->pos) std::copy(c.pos, c.pos + 3, t->pos + 3 * ci);
        if (t->frame) std::copy(c.frame, c.frame + 9, t->frame + 9 * ci);
        if (t->mu) t->mu[ci] = c.mu;
        if (t->cforce) std::copy(&d.cforce[3 * ci], &d.cforce[3 * ci] + 3, t->cforce + 3 * ci);
    }
    put(t->J, d.J); put(t->aref, d.aref); put(t->D, d.D); put(t->Ahat, d.Ahat); put(t->efc_force, d.efc_force);
    if (t->niter) *t->niter = d.niter;
    if (t->cost) *t->cost = d.cost;
    if (t->nrows) *t->nrows = d.nrows;
    return 0;
}

int rbo_step(const void* mp, int32_t n, const double* ctrl, double* qpos, double* qvel, double* qacc_ws,
             const double* friction, const double* mass_scale, uint32_t* status, rbo_contacts* out, int32_t nthreads) {
    return rbo_step_work(mp, n, ctrl, qpos, qvel, qacc_ws, friction, mass_scale, status, out, nullptr, nullptr,
                         nthreads);
}

int rbo_step_work(const void* mp, int32_t n, const double* ctrl, double* qpos, double* qvel, double* qacc_ws,
                  const double* friction, const double* mass_scale, uint32_t* status, rbo_contacts* out, int32_t* sub,
                  double* ops, int32_t nthreads) {
    return rbo_step_fields(mp, n, ctrl, qpos, qvel, qacc_ws, friction, mass_scale, nullptr, status, out, sub, ops,
                           nthreads);
}

int rbo_step_fields(const void* mp, int32_t n, const double* ctrl, double* qpos, double* qvel, double* qacc_ws,
                    const double* friction, const double* mass_scale, const rbo_fields* fields, uint32_t* status,
                    rbo_contacts* out, int32_t* sub, double* ops, int32_t nthreads) {
    if (!mp || n < 0 || !qpos || !qvel || !qacc_ws || !status) return fail("null argument");
    const Model& m0 = *static_cast<const Model*>(mp);
    if (m0.nu && !ctrl) return fail("ctrl required");
    const bool expanded = fields && (fields->geom_size || fields->body_pos || fields->act_kp || fields->act_kd);
#ifdef _OPENMP
    // no more threads than chunks of worlds: a one-world call runs on the calling thread
    int nt = std::max(1, std::min(nthreads > 0 ? nthreads : omp_get_max_threads(), (n + 3) / 4));
#pragma omp parallel num_threads(nt)
#endif
    {
        // a world with expanded fields runs a copy of the model with those fields replaced by its
        // own values (the paper's per-world model fields: section "Architecture", paragraph on the
        // GPU physics backend, and section "Manager-Based API", paragraph "Event manager")
        Model mw = expanded ? m0 : Model();
        const Model& m = expanded ? mw : m0;
        Data d(&m);
        std::vector<double> q1(m.nq), v1(m.nv);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int w = 0; w < n; w++) {
            if (expanded) {
                if (fields->geom_size)
                    std::copy(fields->geom_size + (size_t)w * 3 * m0.ngeom, fields->geom_size + (size_t)(w + 1) * 3 * m0.ngeom,
                              mw.gsize.begin());
                if (fields->body_pos)
                    std::copy(fields->body_pos + (size_t)w * 3 * m0.nbody, fields->body_pos + (size_t)(w + 1) * 3 * m0.nbody,
                              mw.bpos.begin());
                if (fields->act_kp)
                    std::copy(fields->act_kp + (size_t)w * m0.nu, fields->act_kp + (size_t)(w + 1) * m0.nu, mw.akp.begin());
                if (fields->act_kd)
                    std::copy(fields->act_kd + (size_t)w * m0.nu, fields->act_kd + (size_t)(w + 1) * m0.nu, mw.akd.begin());
            }
            double* q = qpos + (size_t)w * m.nq;
            double* v = qvel + (size_t)w * m.nv;
            double* aws = qacc_ws + (size_t)w * m.nv;
            const double* u = m.nu ? ctrl + (size_t)w * m.nu : nullptr;
            const double* fr = friction ? friction + w : nullptr;
            const double* ms = mass_scale ? mass_scale + (size_t)w * m.nbody : nullptr;
            int ncon = 0;
            status[w] &= ~2u;
            int32_t* sw = sub ? sub + (size_t)w * m.K * RBO_SUBCOLS : nullptr;
            double* ow = ops ? ops + (size_t)w * 2 * RBO_NSTAGE : nullptr;
            if (sw) std::fill(sw, sw + m.K * RBO_SUBCOLS, 0);
            if (ow) std::fill(ow, ow + 2 * RBO_NSTAGE, 0.0);
            if (!(status[w] & 1u)) {
                for (int k = 0; k < m.K; k++) {
                    load_world(m, d, q, v, u, aws, fr, ms);
                    forward(m, d);
                    if (d.itercap) status[w] |= 2u;
                    if (sw) {
                        int32_t* r = sw + k * RBO_SUBCOLS;
                        r[0] = (int32_t)d.con.size();
                        r[1] = d.nrows;
                        r[2] = d.niter;
                        r[3] = d.active_final;
                        r[4] = d.segments;
                        for (int i = 0; i < RBO_FPITER; i++) r[5 + i] = (int32_t)d.fp[i];
                    }
                    if (ow) count_ops(m, d, ow, ow + RBO_NSTAGE);
                    integrate(m, q, v, d.aint.data(), q1.data(), v1.data());
                    if (!all_finite(q1.data(), m.nq) || !all_finite(v1.data(), m.nv) || !all_finite(d.aint.data(), m.nv)) {
                        status[w] |= 1u;
                        ncon = 0;
                        break;
                    }
                    std::copy(q1.begin(), q1.end(), q);
                    std::copy(v1.begin(), v1.end(), v);
                    std::copy(d.a.begin(), d.a.end(), aws);
                    ncon = (int)d.con.size();
                }
            }
            if (out) {
                if (out->ncon) out->ncon[w] = ncon;
                size_t base = (size_t)w * m.maxcon;
                for (int ci = 0; ci < ncon; ci++) {
                    const Contact& c = d.con[ci];
                    if (out->geom) { out->geom[2 * (base + ci)] = c.g1; out->geom[2 * (base + ci) + 1] = c.g2; }
                    if (out->feature) out->feature[base + ci] = c.feature;
                    if (out->dist) out->dist[base + ci] = c.dist;
                    if (out->pos) std::copy(c.pos, c.pos + 3, out->pos + 3 * (base + ci));
                    if (out->frame) std::copy(c.frame, c.frame + 9, out->frame + 9 * (base + ci));
                    if (out->force) std::copy(&d.cforce[3 * ci], &d.cforce[3 * ci] + 3, out->force + 3 * (base + ci));
                }
            }
        }
    }
    return 0;
}

int rbo_line_search(const void* mp, const double* qpos, const double* qvel, const double* ctrl, const double* qacc_ws,
                    const double* friction, const double* mass_scale, const double* a, const double* p, double* cost_out,
                    double* alpha_out) {
    if (!mp || !qpos || !qvel || !a || !p) return fail("null argument");
    const Model& m = *static_cast<const Model*>(mp);
    Data d(&m);
    std::vector<double> zero(m.nu, 0.0);
    load_world(m, d, qpos, qvel, ctrl ? ctrl : zero.data(), qacc_ws, friction, mass_scale);
    forward(m, d);
    std::copy(a, a + m.nv, d.a.begin());
    if (cost_out) *cost_out = cost(m, d, d.a.data());
    if (alpha_out) {
        std::vector<double> jar(d.nrows), pv(p, p + m.nv);
        for (int e = 0; e < d.nrows; e++) {
            double t = -d.aref[e];
            for (int k = 0; k < m.nv; k++) t += d.J[(size_t)e * m.nv + k] * d.a[k];
            jar[e] = t;
        }
        *alpha_out = line_search(m, d, jar, pv, nullptr);
    }
    return 0;
}

int rbo_energy(const void* mp, const double* qpos, const double* qvel, const double* mass_scale, double* kin,
               double* pot) {
    if (!mp || !qpos || !qvel) return fail("null argument");
    const Model& m = *static_cast<const Model*>(mp);
    Data d(&m);
    std::vector<double> zero(m.nu, 0.0);
    load_world(m, d, qpos, qvel, zero.data(), nullptr, nullptr, mass_scale);
    kinematics(m, d);
    mass_matrix(m, d);
    double T = 0, V = 0;
    for (int r = 0; r < m.nv; r++)
        for (int s = 0; s < m.nv; s++) T += 0.5 * d.v[r] * d.M[r * m.nv + s] * d.v[s];
    for (int b = 1; b < m.nbody; b++) V -= d.mb[b] * dot3(m.grav, &d.com[3 * b]);
    if (kin) *kin = T;
    if (pot) *pot = V;
    return 0;
}

int rbo_jacobian(const void* mp, const double* qpos, int32_t body, const double* p, double* jacp, double* jacr) {
    if (!mp || !qpos || !p || !jacp || !jacr) return fail("null argument");
    const Model& m = *static_cast<const Model*>(mp);
    if (body < 0 || body >= m.nbody) return fail("bad body");
    Data d(&m);
    std::copy(qpos, qpos + m.nq, d.q.begin());
    kinematics(m, d);
    jacobian(m, d, body, p, jacp, jacr);
    return 0;
}

int rbo_integrate(const void* mp, const double* qpos, const double* qvel, const double* qacc, double* qo, double* vo) {
    if (!mp || !qpos || !qvel || !qacc || !qo || !vo) return fail("null argument");
    integrate(*static_cast<const Model*>(mp), qpos, qvel, qacc, qo, vo);
    return 0;
}

}  // extern "C"
