/*
 * FP64 CPU oracle for the batched rigid-body physics step -- TEST INFRASTRUCTURE ONLY.
 *
 * This library is the plain, slow, obviously-correct reference that the HIP path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never calls it.  It shares no code with the HIP library.
 *
 * The paper (section "Architecture", paragraph on the GPU physics backend) describes the
 * physics only through its interface: a static model, a per-world time-varying state with
 * a leading world dimension, model fields shared or expanded per world, and a step that
 * advances every world (decimated into physics substeps, section "Manager-Based API",
 * pipeline step "Simulate").  Everything inside the step follows the published MuJoCo
 * formulation written from the mathematics (rigid-body kinematics and dynamics after
 * Featherstone 2008; soft constraints and the Newton solver after Todorov 2014).
 *
 * Plain definitions, not fast algorithms: M is the Jacobian sum, c the Jacobian-transpose
 * Newton-Euler sum, all solves dense Cholesky, collision brute force over geom pairs.
 *
 * All arrays are host memory, row-major, float64, owned by the caller.
 * Functions return 0 on success, negative on error (message via rbo_last_error()).
 */
#ifndef RBO_H
#define RBO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { RBO_GEOM_PLANE = 0, RBO_GEOM_SPHERE = 1, RBO_GEOM_CAPSULE = 2, RBO_GEOM_BOX = 3, RBO_GEOM_HFIELD = 4 };
enum { RBO_JNT_FREE = 0, RBO_JNT_HINGE = 1 };
enum { RBO_ACT_POSITION = 0, RBO_ACT_MOTOR = 1 };
enum { RBO_EQ_CONNECT = 0, RBO_EQ_WELD = 1 };

typedef struct rbo_desc {
    int32_t nbody, njnt, ngeom, nu;
    /* bodies [nbody]; body 0 is the world */
    const int32_t* body_parent;
    const double *body_pos, *body_quat, *body_ipos, *body_iquat, *body_mass, *body_inertia;
    /* joints [njnt] */
    const int32_t *jnt_type, *jnt_body;
    const double *jnt_pos, *jnt_axis, *jnt_armature;
    /* geoms [ngeom] */
    const int32_t *geom_type, *geom_body, *geom_contype, *geom_conaffinity;
    const double *geom_pos, *geom_quat, *geom_size, *geom_friction, *geom_margin;
    /* actuators [nu] */
    const int32_t *act_type, *act_joint;
    const double *act_kp, *act_kd, *act_gear;
    /* options */
    double timestep;
    int32_t nsubsteps;
    double gravity[3];
    int32_t iterations;
    double tolerance;
    double solref[2];
    double solimp[5];
    int32_t friction_per_world, mass_scale_per_world;
    /* joint ranges [njnt, 2] (lower, upper), or NULL: a hinge is limited when lower < upper;
       free joints take no range (both entries equal) */
    const double* jnt_range;
    /* joint damping [njnt] (>= 0, hinges only), or NULL: a passive torque -damping * qvel,
       integrated implicitly (see rbo_step) */
    const double* jnt_damping;
    /* geom contact dimensionality [ngeom] (1 frictionless, 3 pyramidal sliding friction, 4 with
       torsional friction, 6 with torsional and rolling friction), or NULL for 3 everywhere; a
       pair takes the larger of its two geoms' */
    const int32_t* geom_condim;
    /* height grid of the model's height-field geoms (type RBO_GEOM_HFIELD, static; a geom's
       size[0], size[1] are the grid's half extents along its local x and y): hfield_nrow rows
       along y by hfield_ncol columns along x (both >= 2), heights [nrow, ncol] along local z;
       sample (i, j) sits at x = -sx + 2 sx j / (ncol - 1), y = -sy + 2 sy i / (nrow - 1).  Each
       cell is split along its diagonal from sample (i, j) to (i + 1, j + 1) into the triangles
       {(i, j), (i, j + 1), (i + 1, j + 1)} and {(i, j), (i + 1, j + 1), (i + 1, j)}.  NULL with
       0 rows when the model has no height field. */
    int32_t hfield_nrow, hfield_ncol;
    const double* hfield_data;
    /* equality constraints [neq] between a moving body and the world: eq_type 0 = connect (the
       point eq_anchor [neq, 3] of body eq_body, in its frame, held at the world point
       eq_target[0..3)), 1 = weld (that, and the body's orientation held at the unit quaternion
       eq_target[3..7)); eq_target [neq, 7].  Each gives 3 (connect) or 6 (weld) bilateral soft
       rows after the contact and limit rows: world x, y, z components of the anchor's offset
       from the target, then of the rotation vector of R_body R_target', each with its own
       impedance, the contacts' solref / solimp and exact A-hat. */
    int32_t neq;
    const int32_t *eq_type, *eq_body;
    const double *eq_anchor, *eq_target;
    /* torsional and rolling friction coefficients [ngeom] (>= 0), or NULL for 0.005 and 0.0001;
       a pair takes the larger of its two geoms' and uses them when its condim is 4 or 6 */
    const double *geom_friction_spin, *geom_friction_roll;
    /* friction cones: 0 pyramidal (2 (condim - 1) rows per contact), 1 elliptic (condim 1 or 3:
       the frame rows themselves, costed per contact by the soft elliptic cone, the tangential
       rows' regulariser the normal row's divided by impratio > 0) */
    int32_t cone;
    double impratio;
} rbo_desc;

typedef struct rbo_info {
    int32_t nq, nv, nu, nbody, ngeom, maxcon, maxrows, npair;
    double meaninertia;
} rbo_info;

/* Contact list of one world, capacity maxcon (any pointer may be NULL). */
typedef struct rbo_contacts {
    int32_t* ncon;        /* [n] */
    int32_t* geom;        /* [n, maxcon, 2] */
    int32_t* feature;     /* [n, maxcon] */
    double* dist;         /* [n, maxcon] */
    double* pos;          /* [n, maxcon, 3] */
    double* frame;        /* [n, maxcon, 9] rows: normal, t1, t2 */
    double* force;        /* [n, maxcon, 3] (f_n, f_t1, f_t2) */
} rbo_contacts;

/* Stage taps of one substep for one world (any pointer may be NULL). */
typedef struct rbo_taps {
    double *xpos, *xquat, *xmat, *com;          /* [nbody,3] [nbody,4] [nbody,9] [nbody,3] */
    double *gpos, *gmat;                        /* [ngeom,3] [ngeom,9] */
    double *M, *bias, *tau, *a0;                /* [nv,nv] [nv] [nv] [nv] */
    int32_t* ncon;                              /* [1] */
    int32_t *geom, *feature;                    /* [maxcon,2] [maxcon] */
    double *dist, *pos, *frame, *mu;            /* [maxcon] [maxcon,3] [maxcon,9] [maxcon] */
    double *J, *aref, *D, *Ahat, *efc_force;    /* [maxrows,nv] [maxrows] x4 */
    double *qacc, *cforce;                      /* [nv] [maxcon,3] */
    int32_t* niter;                             /* [1] Newton iterations run */
    double* cost;                               /* [1] final cost f(qacc) */
    int32_t* nrows;                             /* [1] constraint rows: 4 per contact, limits, equalities */
} rbo_taps;

/* Work outputs of rbo_step_work.
 *
 * Per substep s < K of each world, RBO_SUBCOLS int32 ([n, K, RBO_SUBCOLS]):
 *   0 contacts, 1 constraint rows, 2 Newton updates made, 3 rows active at the solution,
 *   4 line-search segments examined (quadratic pieces whose minimiser was tried),
 *   5 .. 5 + RBO_FPITER - 1: fingerprint of the active set each of the first RBO_FPITER Newton
 *   updates was built from (0 past the last update).  The fingerprint of a set A of rows is
 *   sum over e in A of (id_e + 1) * 2654435761 mod 2^32, with id = 4 c + e for pyramid row e of
 *   contact c (a frictionless contact's one row has e = 0), 256 + dof for a joint-limit row and
 *   512 + 6 q + k for row k of equality q (bilateral rows are always active).
 *
 * Per world, 2 x RBO_NSTAGE doubles ([n, 2, RBO_NSTAGE]), summed over the K substeps: arithmetic
 * operations (a multiply-add counts 2) of the stages kinematics, inertia and bias forces,
 * factorisation and smooth acceleration, collision, constraint rows, Newton solve, integration;
 * row 0 as this oracle's plain definitions perform them (dense Jacobian sums, dense Cholesky,
 * brute-force pairs), row 1 for the recursive tree-sparse formulation of the same quantities
 * (composite-rigid-body inertia, recursive Newton-Euler, no-fill-in L'DL over the dof tree,
 * Jacobian rows over the dofs they touch, Hessian updates over those dofs), evaluated on this
 * oracle's own contacts, rows, active sets, iterations and line-search segments. */
#define RBO_FPITER 4
#define RBO_SUBCOLS (5 + RBO_FPITER)
#define RBO_NSTAGE 7

const char* rbo_last_error(void);
int rbo_model_create(const rbo_desc* d, void** out);
void rbo_model_destroy(void* m);
int rbo_model_info(const void* m, rbo_info* out);

/* mode: 0 = mirror (model iterations/tolerance), 1 = converged (100 iterations, tol 1e-12). */
int rbo_set_mode(void* m, int32_t mode);

/* One substep for one world from (qpos, qvel, ctrl, qacc_ws); fills taps; does not integrate. */
int rbo_forward(const void* m, const double* qpos, const double* qvel, const double* ctrl,
                const double* qacc_ws, const double* friction, const double* mass_scale, rbo_taps* taps);

/* n env steps of K substeps each (OpenMP over worlds, nthreads <= 0 -> all cores).
 * qpos [n,nq], qvel [n,nv], qacc_ws [n,nv] in/out; ctrl [n,nu]; friction [n] / mass_scale
 * [n,nbody] may be NULL; status [n] in/out (bit 0 = non-finite, world frozen; bit 1 =
 * some substep's Newton loop stopped at the iteration cap, cleared at the start of each step);
 * contacts may be NULL and receive the last substep's contacts. */
int rbo_step(const void* m, int32_t n, const double* ctrl, double* qpos, double* qvel,
             double* qacc_ws, const double* friction, const double* mass_scale, uint32_t* status,
             rbo_contacts* contacts, int32_t nthreads);

/* rbo_step plus the work outputs above: sub [n, K, RBO_SUBCOLS] and ops [n, 2, RBO_NSTAGE]
 * (either may be NULL). */
int rbo_step_work(const void* m, int32_t n, const double* ctrl, double* qpos, double* qvel,
                  double* qacc_ws, const double* friction, const double* mass_scale, uint32_t* status,
                  rbo_contacts* contacts, int32_t* sub, double* ops, int32_t nthreads);

/* Per-world values of model fields (any pointer may be NULL: every world uses the model's own
 * values): geom_size [n, ngeom, 3], body_pos [n, nbody, 3] (position in the parent's frame),
 * act_kp [n, nu] and act_kd [n, nu] (position-actuator gains).  World w steps exactly as a
 * model whose description carries world w's values would. */
typedef struct rbo_fields {
    const double *geom_size, *body_pos, *act_kp, *act_kd;
} rbo_fields;

/* rbo_step_work with per-world model fields (fields may be NULL). */
int rbo_step_fields(const void* m, int32_t n, const double* ctrl, double* qpos, double* qvel, double* qacc_ws,
                    const double* friction, const double* mass_scale, const rbo_fields* fields, uint32_t* status,
                    rbo_contacts* contacts, int32_t* sub, double* ops, int32_t nthreads);

/* The constraint cost f(a) of one substep's state (rows built as in rbo_forward) and the exact
 * line search of the Newton method from acceleration a along direction p:
 * alpha = argmin over alpha >= 0 of f(a + alpha p) (cost_out, alpha_out nullable). */
int rbo_line_search(const void* m, const double* qpos, const double* qvel, const double* ctrl,
                    const double* qacc_ws, const double* friction, const double* mass_scale,
                    const double* a, const double* p, double* cost_out, double* alpha_out);

/* Energies of one world: kinetic 0.5 v'Mv and gravitational potential -sum m g.com. */
int rbo_energy(const void* m, const double* qpos, const double* qvel, const double* mass_scale,
               double* kinetic, double* potential);

/* Point Jacobians of a body point p (world): jacp [3,nv], jacr [3,nv]. */
int rbo_jacobian(const void* m, const double* qpos, int32_t body, const double* p, double* jacp,
                 double* jacr);

/* Integrate one semi-implicit Euler substep from a given acceleration (no dynamics). */
int rbo_integrate(const void* m, const double* qpos, const double* qvel, const double* qacc,
                  double* qpos_out, double* qvel_out);

#ifdef __cplusplus
}
#endif
#endif
