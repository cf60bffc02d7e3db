/*
 * rbstep -- batched rigid-body physics step for MI355X (gfx950).
 *
 * The operation: advance N independent worlds of one robot model by one environment step,
 * i.e. K physics substeps with the controls held (paper, section "Manager-Based API",
 * pipeline step "Simulate": d decimation substeps per env step).  The model is static and
 * shared by all worlds; the state has a leading world dimension; selected model fields
 * (friction, body mass scale) can be expanded to one value per world (paper, section
 * "Architecture", paragraph on the GPU physics backend).  A substep performs forward
 * kinematics, the joint-space inertia and its factorisation, bias forces, plane collision,
 * the soft-contact Newton solve and semi-implicit Euler integration.
 *
 * Conventions
 *   - Units SI; quaternions (w, x, y, z); body 0 is the world; parent[b] < b.
 *   - Free joint qpos = [pos(3, world), quat(4)], qvel = [linear velocity of the body
 *     origin (world, 3), angular velocity (body frame, 3)].  Hinge qpos is the angle.
 *   - Every device array is row-major with the world index leading, float32 unless noted,
 *     and belongs to the caller (e.g. a torch tensor); the library never frees it.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the default stream).  Every
 *     function that takes a stream only enqueues work on it and returns; the caller
 *     synchronises (e.g. through torch).  Buffers must stay valid until that work ends.
 *
 * Errors
 *   Functions return RB_OK (0) or a negative code; rb_last_error() then returns a message
 *   (thread-local).  Argument and model validation errors are reported synchronously;
 *   an asynchronous device fault surfaces as RB_EHIP on a later call.  Numerical trouble is
 *   data, not an error: it is reported per world in the status word (RB_STATUS_*).
 */
#ifndef RBSTEP_H
#define RBSTEP_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define RB_OK 0
#define RB_EINVAL (-1)   /* invalid argument or model */
#define RB_ENOMEM (-2)   /* device allocation failed */
#define RB_EHIP (-3)     /* HIP runtime error (including earlier asynchronous faults) */
#define RB_EBUDGET (-4)  /* request exceeds the configured device-memory budget */
#define RB_ESTATE (-5)   /* object used in a state that does not allow the call */

/* per-world status bits */
#define RB_STATUS_NONFINITE 1u   /* non-finite qpos/qvel/qacc: the world is frozen until reset */
#define RB_STATUS_ITERCAP 2u     /* the Newton solve ran its full iteration budget (informational) */
#define RB_STATUS_CONOVERFLOW 4u /* more contacts than the per-world capacity; the extra ones
                                    (last in pair order) were dropped for this substep */

enum { RB_GEOM_PLANE = 0, RB_GEOM_SPHERE = 1, RB_GEOM_CAPSULE = 2, RB_GEOM_BOX = 3, RB_GEOM_HFIELD = 4 };
enum { RB_JNT_FREE = 0, RB_JNT_HINGE = 1 };
enum { RB_ACT_POSITION = 0, RB_ACT_MOTOR = 1 };
enum { RB_EQ_CONNECT = 0, RB_EQ_WELD = 1 };
enum { RB_CONE_PYRAMIDAL = 0, RB_CONE_ELLIPTIC = 1 };
enum {
    RB_PARAM_FRICTION = 0,   /* [n]: friction of every contact of the world (model flag) */
    RB_PARAM_MASS_SCALE = 1, /* [n, nbody]: body mass and rotational inertia scale (model flag) */
    RB_PARAM_GEOM_SIZE = 2,  /* [n, ngeom, 3]: geom sizes (any model; expanded on first use) */
    RB_PARAM_BODY_POS = 3,   /* [n, nbody, 3]: body position in its parent's frame (ditto) */
    RB_PARAM_ACT_KP = 4,     /* [n, nu]: position-actuator stiffness kp (ditto) */
    RB_PARAM_ACT_KD = 5      /* [n, nu]: position-actuator damping kd (ditto) */
};

/* Host-side model description, float64, owned by the caller (copied by rb_model_create).
 * Bodies [nbody] (body 0 = world), joints [njnt] (listed in body order, at most one per
 * body, free joints only on children of the world), geoms [ngeom], actuators [nu]
 * (hinge joints only).  Sizes: sphere (r), capsule (r, half-length along local z), box
 * (half-sizes); a plane's normal is its local +z and it must sit on a static body. */
typedef struct rb_model_desc {
    int32_t nbody, njnt, ngeom, nu;
    const int32_t* body_parent;
    const double *body_pos, *body_quat, *body_ipos, *body_iquat, *body_mass, *body_inertia;
    const int32_t *jnt_type, *jnt_body;
    const double *jnt_pos, *jnt_axis, *jnt_armature;
    const int32_t *geom_type, *geom_body, *geom_contype, *geom_conaffinity;
    const double *geom_pos, *geom_quat, *geom_size, *geom_friction, *geom_margin;
    const int32_t *act_type, *act_joint;
    const double *act_kp, *act_kd, *act_gear;
    double timestep;        /* physics substep, s */
    int32_t nsubsteps;      /* K substeps per env step, controls held */
    double gravity[3];
    int32_t iterations;     /* Newton iteration budget */
    double tolerance;       /* Newton tolerance on the scaled gradient and improvement */
    double solref[2];       /* (time constant, damping ratio) */
    double solimp[5];       /* (dmin, dmax, width, midpoint, power) */
    int32_t friction_per_world, mass_scale_per_world;
    /* joint ranges [njnt, 2] (lower, upper), or NULL for none: a hinge is limited when
     * lower < upper (finite, lower <= upper required); free joints take no range (equal
     * entries).  A limited hinge outside its range gets one soft unilateral constraint row
     * pushing it back, solved with the contacts. */
    const double* jnt_range;
    /* joint damping [njnt] (>= 0; hinges only), or NULL for none: a passive torque
     * -damping * qvel, integrated implicitly -- the step applies (M + dt B)^-1 M qacc, B the
     * diagonal of dampings, instead of the solved qacc (which stays the warm start). */
    const double* jnt_damping;
    /* geom contact dimensionality [ngeom] (1 frictionless, 3 pyramidal sliding friction, 4 with
     * torsional friction, 6 with torsional and rolling friction), or NULL for 3 everywhere; a
     * pair takes the larger of its two geoms' (a condim-1 pair keeps the normal row only and
     * reports zero tangential force).  Condim 4 and 6 add the row pairs J_n +- mu_spin J_spin
     * and J_n +- mu_roll J_roll (J_spin, J_roll the contact frame's n and t1, t2 components of
     * the body's angular velocity); their forces add to the reported normal force, and the
     * torsional and rolling torques are not reported.  A model's equality rows and the rows
     * its condim-4/6 pairs can produce (2 or 6 per contact) number at most 64. */
    const int32_t* geom_condim;
    /* height grid of the model's height-field geoms (type RB_GEOM_HFIELD, static; a geom's
     * size[0], size[1] are the grid's half extents along its local x and y): hfield_nrow rows
     * along y by hfield_ncol columns along x (both >= 2), heights [nrow, ncol] along local z,
     * sample (i, j) at x = -sx + 2 sx j / (ncol - 1), y = -sy + 2 sy i / (nrow - 1).  A cell is
     * split along its diagonal from sample (i, j) to (i + 1, j + 1); a sphere's centre, a
     * capsule's segment ends and a box's vertices are each tested, as against a plane, against
     * the plane of the triangle under them (none off the grid), the height field taking the
     * place of g1.  0 rows and NULL when the model has none.  Cites: paper, section
     * "Components", paragraph "Terrain" (height-field terrains). */
    int32_t hfield_nrow, hfield_ncol;
    const double* hfield_data;
    /* equality constraints [neq] between a moving body and the world (0 and NULLs for none; the
     * rows of all of them together at most 64): eq_type RB_EQ_CONNECT holds the body point
     * eq_anchor [neq, 3] (body frame) at the world point eq_target[0..2] ([neq, 7]); RB_EQ_WELD
     * also holds the body's orientation at the unit quaternion eq_target[3..6].  Each gives soft
     * bilateral rows (connect 3: the anchor's world offset from its target along x, y, z; weld 3
     * more: the rotation vector of R_body R_target') solved with the contacts, always active,
     * with the contacts' solref/solimp.  Cites: paper, section "Architecture", paragraph on the
     * GPU physics backend (the constraint model of the simulator it builds on). */
    int32_t neq;
    const int32_t *eq_type, *eq_body;
    const double *eq_anchor, *eq_target;
    /* torsional and rolling friction coefficients [ngeom] (>= 0), or NULL for 0.005 and 0.0001;
     * a pair takes the larger of its two geoms' and uses them when its condim is 4 or 6.  Cites:
     * paper, section "Architecture", paragraph on the GPU physics backend (the contact model of
     * the simulator it builds on). */
    const double *geom_friction_spin, *geom_friction_roll;
    /* friction cones: RB_CONE_PYRAMIDAL (2 (condim - 1) pyramid rows per contact) or
     * RB_CONE_ELLIPTIC: a contact's condim frame rows (normal, t1, t2, then the spin about the
     * normal with condim 4 and 6, and the rolling about t1, t2 with condim 6) costed together by
     * the soft elliptic cone, its force the projection of -D jar onto the friction cone
     * {sum_i (f_i / mu_i)^2 <= f_n^2} (mu_i: mu, mu_spin or mu_roll) in the metric of D^-1; the
     * friction rows have no distance reference, the tangential rows take the normal row's D
     * times impratio (> 0; 1 when 0 is given), the spin and rolling rows that times
     * (mu_i / mu)^2.  Cites: paper, section "Architecture", paragraph on the GPU physics
     * backend (the constraint model of the simulator it builds on). */
    int32_t cone;
    double impratio;
} rb_model_desc;

typedef struct rb_model rb_model;
typedef struct rb_batch rb_batch;

typedef struct rb_model_info {
    int32_t nq, nv, nu, nbody, ngeom, npair;
    int32_t maxcon;          /* static per-world contact bound of the model */
    int32_t max_depth;       /* longest chain of dofs from the root */
    int32_t lds_bytes;       /* on-chip memory one world uses during a step */
    int32_t bytes_per_world; /* device memory a batch holds per world slot (warm start,
                                status, per-world parameters); the caller's state,
                                control and contact buffers come on top */
    double meaninertia;
} rb_model_info;

/* Contact output of the last substep, struct of device arrays with `cap` slots per world
 * (cap = the batch's contact capacity, rb_batch_contact_capacity()).  Any pointer may be
 * NULL to skip that field.  Contacts appear in collision-pair order; slots >= ncon are
 * left untouched. */
typedef struct rb_contacts {
    int32_t* ncon;     /* [n] */
    int32_t* geom;     /* [n, cap, 2]  (g1, g2), normal points from g1 to g2 */
    int32_t* feature;  /* [n, cap]     0 sphere (on a plane or a box); 0/1 capsule -z/+z end;
                                      0..7 box vertex on a plane; box-box: clipped-point index */
    float* dist;       /* [n, cap]     signed distance, < 0 when penetrating */
    float* pos;        /* [n, cap, 3]  contact point (midway between the surfaces) */
    float* frame;      /* [n, cap, 9]  rows: normal, tangent 1, tangent 2 */
    float* force;      /* [n, cap, 3]  (normal, tangent 1, tangent 2) contact force */
} rb_contacts;

/* The message of this thread's last nonzero return.  Cites: no passage (error reporting of this
 * library). */
const char* rb_last_error(void);

/* Validate and compile a model; uploads its constants to the current HIP device.
 * Cites: paper, section "Architecture", paragraph "Scene pipeline" (a compiled model is
 * transferred to the GPU, put_model), and its paragraph on the GPU physics backend (the static
 * model shared by all worlds).
 * Rejects (RB_EINVAL): parent >= child, non-positive mass or inertia violating the
 * triangle inequality, non-unit quaternions, misplaced joints, unknown types,
 * collision pairs other than plane-{sphere, capsule, box}, box-box and sphere-box, pairs whose bodies can both
 * move, more than 64 dofs, 64 collision pairs, 256 geoms or a dof chain deeper than 32. */
int rb_model_create(const rb_model_desc* desc, rb_model** out);

/* The same model as JSON text (NUL-terminated, owned by the caller).  Cites: paper, section
 * "Architecture", paragraph "Scene pipeline" (a scene description compiled into a model).
 * The text is an object with
 *   "opt": {"timestep", "nsubsteps", "gravity": [3], "iterations", "tolerance",
 *           "solref": [2], "solimp": [5], "cone": "pyramidal" | "elliptic", "impratio"
 *           (the last two optional)},
 *   "bodies": [{"parent", "pos": [3], "quat": [4], "ipos": [3], "iquat": [4], "mass",
 *               "inertia": [3]}, ...]   (body 0 = world),
 *   "joints": [{"type": "free" | "hinge", "body", "pos": [3], "axis": [3], "armature",
 *               "range": [2], "damping" (both optional, hinges only)}, ...],
 *   "geoms": [{"type": "plane" | "sphere" | "capsule" | "box" | "hfield", "body", "pos": [3],
 *              "quat": [4], "size": [3], "friction", "contype", "conaffinity", "margin",
 *              "condim" (optional, 1, 3, 4 or 6), "friction_spin", "friction_roll" (optional)}, ...],
 *   "actuators": [{"type": "position" | "motor", "joint", "kp", "kd", "gear"}, ...],
 *   "per_world": {"friction": bool, "mass_scale": bool}   (optional, default false),
 *   "hfield": {"nrow", "ncol", "data": [nrow * ncol]}    (required with hfield geoms),
 *   "equality": [{"type": "connect" | "weld", "body", "anchor": [3], "target": [3],
 *                 "quat": [4] (welds only)}, ...]   (optional);
 * other keys are ignored.  Each entry maps to the rb_model_desc field of the same name, in
 * list order.  Malformed JSON or a missing or mistyped field is RB_EINVAL (with the field
 * named in rb_last_error) before any device call; the parsed description then goes through
 * rb_model_create and its validation. */
int rb_model_create_json(const char* json, rb_model** out);

/* Release a model and its device constants (after every batch made from it).  Cites: paper,
 * section "Architecture", paragraph "Scene pipeline". */
void rb_model_destroy(rb_model* model);

/* Sizes of a compiled model (rb_model_info), host memory owned by the caller.  RB_EINVAL on
 * NULL.  Cites: paper, section "Architecture", paragraph on the GPU physics backend (the
 * static model description). */
int rb_model_info_get(const rb_model* model, rb_model_info* out);

/* A batch of `capacity` world slots of one model: owns each world's warm start (qacc of
 * the previous substep), status word, per-world parameters and contact capacity.
 * contact_capacity <= 0 selects min(model maxcon, 64); at most 64.  Worlds start with a
 * zero warm start, status 0, per-world friction 1.0 and mass scale 1 (the per-world values
 * are read only by models that declare them per world).  RB_ENOMEM when the device memory
 * cannot be allocated.  Cites: paper, section "Architecture", paragraph on the GPU physics
 * backend (the time-varying state with a leading world dimension) and paragraph "Scene
 * pipeline" (put_data). */
int rb_batch_create(const rb_model* model, int32_t capacity, int32_t contact_capacity, rb_batch** out);

/* Release a batch's device memory (after the work using it has completed).  Cites: as
 * rb_batch_create. */
void rb_batch_destroy(rb_batch* batch);

/* Contact slots per world of the batch's contact output (0 for NULL).  Cites: as rb_step. */
int32_t rb_batch_contact_capacity(const rb_batch* batch);

/* Per-world parameters for slots [0, n): RB_PARAM_FRICTION takes [n] floats (friction of
 * every contact in the world; the model must have friction_per_world), RB_PARAM_MASS_SCALE
 * [n, nbody] floats (scales each body's mass and rotational inertia; the model must have
 * mass_scale_per_world).  RB_PARAM_GEOM_SIZE [n, ngeom, 3], RB_PARAM_BODY_POS [n, nbody, 3],
 * RB_PARAM_ACT_KP and RB_PARAM_ACT_KD [n, nu] expand that model field to one value per world
 * slot on first use: the batch allocates a [capacity, ...] array (synchronously) holding the
 * model's values in every slot, then takes the given slots' values; every world then runs with
 * its own values (a world steps as a model whose description carried them; inertias, static
 * contact bounds and the tolerance scale stay the model's).  Fused plans that bound the batch
 * pick the new arrays up at their next step or graph replay (their argument blocks are
 * rewritten; a captured graph needs no new capture).  Values are not validated.  Device
 * pointer; copied on the stream.  RB_EINVAL for another field, a model without that per-world
 * field (friction, mass scale) or without actuators (gains), or n outside [0, capacity];
 * RB_ENOMEM when the expansion cannot allocate.  Cites: paper, section
 * "Architecture", paragraph on the GPU physics backend (model fields expanded to vary per
 * world), and section "Manager-Based API", paragraph "Event manager" (domain randomisation
 * writing per-world values). */
int rb_batch_set_params(rb_batch* batch, int32_t field, int32_t n, const float* dev_vals, void* hip_stream);

/* As rb_batch_set_params for slots [first, first + n): dev_vals holds those n worlds' values.
 * RB_EINVAL when the range leaves the batch.  Cites: as rb_batch_set_params. */
int rb_batch_set_params_at(rb_batch* batch, int32_t field, int32_t first, int32_t n, const float* dev_vals,
                           void* hip_stream);

/* Resident waves per SIMD of this batch's plain launches: 3, 4, or 0 for the automatic choice
 * (4 when the model's LDS lets 16 worlds share a compute unit, its chain bound is at most 16
 * and the launch has more worlds than one round of 3 waves per SIMD holds; 3 otherwise).  4 is
 * ignored where the chain bound exceeds 16.  Results do not depend on it.  Cites: no passage (a
 * launch knob of this implementation). */
int rb_batch_set_waves(rb_batch* batch, int32_t waves);

/* Reset n worlds named by dev_ids [n] (int32, device, each in [0, capacity)): clear their
 * status and set their warm start from dev_qacc_ws [n, nv] (device; NULL = zero); the caller
 * writes their qpos/qvel.  Cites: paper, section "Manager-Based API", pipeline step "Reset"
 * (entity states reinitialised) and section "Architecture", paragraph "Scene pipeline"
 * (put_data). */
int rb_world_reset(rb_batch* batch, const int32_t* dev_ids, int32_t n, const float* dev_qacc_ws, void* hip_stream);

/* Copy the warm start [n, nv] and status [n] of slots [0, n) out (either may be NULL; device
 * pointers), for checkpoints: rb_world_reset with the saved warm start resumes bit for bit.
 * Cites: paper, section "Architecture", paragraph on the GPU physics backend (the per-world
 * time-varying state). */
int rb_get_state(const rb_batch* batch, int32_t n, float* dev_qacc_ws, uint32_t* dev_status, void* hip_stream);

/* One env step (K substeps) of slots [0, n).  Cites: paper, section "Manager-Based API",
 * pipeline step "Simulate" (d decimation substeps with the controls held), and section
 * "Manager-Based API", paragraph "Termination manager" (non-finite states caught per world).
 * dev_qpos [n, nq] and dev_qvel [n, nv] are
 * read and overwritten in place; dev_ctrl [n, nu] is held for the K substeps (NULL when
 * nu = 0).  contacts (nullable) receives the last substep's contacts; dev_status [n]
 * (nullable) receives each world's status word.  A world with RB_STATUS_NONFINITE set is
 * not advanced. */
int rb_step(rb_batch* batch, int32_t n, const float* dev_ctrl, float* dev_qpos, float* dev_qvel,
            const rb_contacts* contacts, uint32_t* dev_status, void* hip_stream);

/* Diagnostic taps of the first substep of one step of slots [0, n), for parity checks and
 * work accounting: the same computation as rb_step (and it advances the state the same
 * way), plus per world dev_M [n, nv, nv] joint-space inertia, dev_bias [n, nv] bias forces
 * c(q, v), dev_a0 [n, nv] smooth acceleration, dev_qacc [n, nv] constrained acceleration of
 * the first substep, dev_efc [n, cap, 4, 3] per pyramid row (aref, D, A-hat), and
 * dev_stats [n, 50] int32: totals over the K substeps of contacts, rows active at the
 * solution, Newton updates and line-search segments; shader-clock cycles / 16 spent in ten
 * stages (kinematics; inertia, bias forces and M; factorisation of M and a0; collision;
 * constraint rows; Newton start; gradient and Hessian; Hessian factorisation and solve; line
 * search and update; integration); then for each of the first 4 substeps 9 columns: contacts,
 * constraint rows, Newton updates, rows active at the solution, line-search segments, and the
 * fingerprint of the active set each of the first 4 updates was built from (sum over its rows
 * of (id + 1) * 2654435761 mod 2^32, id = 4 c + e for pyramid row e of contact c, a
 * frictionless contact's one row e = 0, 256 + dof for a joint-limit row; 0 past the last
 * update).  Any output may be NULL.  Cites: as rb_step. */
int rb_step_taps(rb_batch* batch, int32_t n, const float* dev_ctrl, float* dev_qpos, float* dev_qvel,
                 const rb_contacts* contacts, uint32_t* dev_status, float* dev_M, float* dev_bias,
                 float* dev_a0, float* dev_qacc, float* dev_efc, int32_t* dev_stats, void* hip_stream);

/* Floats of the library's fixed per-device array that rb_step_noalloc works in (16 MiB). */
#define RB_NOALLOC_MAX_FLOATS (4 << 20)

/* One env step of n worlds, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It computes what rb_step
 * computes on a batch of n slots that was just created or reset (zero warm start, status 0)
 * with the given per-world parameters, and allocates nothing: the per-world working state the
 * kernel keeps (warm start, status word, default parameters) lives in a fixed array of
 * RB_NOALLOC_MAX_FLOATS floats that the library holds on each device it runs on until the
 * process ends, cleared by a fill kernel at the start of every call (no memset, so the call can
 * be captured in a graph).  Consequently the warm start does not carry from one call to the
 * next.  Arguments as rb_step, with the model in place of a batch: dev_ctrl [n, nu] (NULL when
 * nu = 0), dev_qpos [n, nq] and dev_qvel [n, nv] read and overwritten; dev_friction [n] and
 * dev_mass_scale [n, nbody] (nullable, read only) for models with those per-world fields (NULL
 * means 1.0); contacts (nullable) with capacity min(maxcon, 64) per world, as a batch created
 * with contact_capacity 0; dev_status [n] (nullable).  Returns RB_EINVAL, before any launch,
 * when n * (nv + 2 + nbody) exceeds RB_NOALLOC_MAX_FLOATS.  Every call on a GPU uses that GPU's
 * one array: calls that overlap on one GPU (concurrent streams or host threads) race and must
 * be serialised by the caller. */
int rb_step_noalloc(const rb_model* model, int32_t n, const float* dev_ctrl, float* dev_qpos, float* dev_qvel,
                    const float* dev_friction, const float* dev_mass_scale, const rb_contacts* contacts,
                    uint32_t* dev_status, void* hip_stream);

/* ---------------------------------------------------------------------------------------
 * Mixed-model batching: one fused launch steps several batches (of the same or different
 * models) together.  Every world runs the same per-world code as rb_step, so its results do
 * not depend on the schedule or on the other batches; the schedule only decides the order in
 * which worlds are dispatched and the grid.  A fixed sequence of fused steps can be captured
 * once in a hipGraph and replayed (the paper's graph capture of the simulation step, section
 * "Architecture").
 * --------------------------------------------------------------------------------------- */
typedef struct rb_multi rb_multi;

enum { RB_ORDER_BATCH = 0,        /* batch after batch, worlds in index order */
       RB_ORDER_HEAVY_FIRST = 1,  /* most expensive batches first (by cost per world) */
       RB_ORDER_INTERLEAVE = 2 }; /* worlds of all batches interleaved in proportion */

/* A plan over nbatch existing batches (not owned; they must outlive the plan).  Cites: paper,
 * section "Architecture", paragraph on the GPU physics backend (many worlds stepped at once). */
int rb_multi_create(rb_batch* const* batches, int32_t nbatch, rb_multi** out);

/* Release a plan and its captured graph.  Cites: as rb_multi_create. */
void rb_multi_destroy(rb_multi* plan);

/* Step inputs of batch i for the following fused steps (device pointers as in rb_step,
 * slots [0, n)).  Copies a small argument block to the device; synchronous.  Cites: as
 * rb_step. */
int rb_multi_bind(rb_multi* plan, int32_t i, int32_t n, const float* dev_ctrl, float* dev_qpos, float* dev_qvel,
                  const rb_contacts* contacts, uint32_t* dev_status);

/* Dispatch order and grid of the fused launch.  cost [nbatch] (host, nullable) is the
 * relative cost of one world of each batch, used by RB_ORDER_HEAVY_FIRST (default: a
 * per-model estimate).  grid <= 0 launches one workgroup per world; grid > 0 launches that
 * many persistent workgroups walking the list.  Call after every batch is bound.  Cites: no
 * passage (a schedule of this implementation). */
int rb_multi_set_schedule(rb_multi* plan, int32_t order, int32_t grid, const float* cost);

/* An explicit work list instead of a schedule: host_items [n] (host memory, read before the
 * call returns) of batch << 24 | world, each world below the n bound for its batch, in
 * dispatch order; grid as in rb_multi_set_schedule.  The list is uploaded asynchronously on
 * the stream (through pinned staging owned by the plan), so later rb_multi_step calls on the
 * same stream use it and earlier ones keep the previous list; steps must therefore be issued
 * on that stream.  This is how a serving loop steps exactly the worlds of its live requests
 * without stopping the device.  RB_EINVAL on an item outside the bound batches.  Cites: no
 * passage (the serving form's work list). */
int rb_multi_set_items(rb_multi* plan, const int32_t* host_items, int32_t n, int32_t grid, void* hip_stream);

/* Resident waves per SIMD of the fused launch: 4 selects the instantiation compiled for 4
 * (RB_EINVAL unless every model has a chain bound <= 16 and LDS small enough for 16 worlds per
 * compute unit); 3 the default one; 1 or 2 that one capped by giving each workgroup enough LDS
 * that no more fit; 0 the automatic choice (4 when the models fit and the work list is more
 * than one round of 3 waves per SIMD, else 3).  A schedule knob for the autotuner; results do
 * not depend on it.  Cites: no passage. */
int rb_multi_set_occupancy(rb_multi* plan, int32_t waves_per_simd);

/* Worlds per workgroup of the fused launch: 1 (the default), 2 or 4 worlds, one 64-lane wave
 * each, share a workgroup and its LDS allocation (each world keeps its own LDS section; the
 * waves never wait for each other).  The schedule's grid still counts worlds in flight.
 * RB_EINVAL for another count or when the worlds of one workgroup would need more LDS than a
 * workgroup may use.  Composes with rb_multi_set_occupancy (a cap of w waves per SIMD then
 * allows 4 w / count workgroups per compute unit).  A schedule knob for the autotuner; results
 * do not depend on it.  Cites: no passage (the batching form's launch shape). */
int rb_multi_set_group(rb_multi* plan, int32_t worlds_per_workgroup);

/* One env step of every scheduled world in one launch on the stream.  RB_ESTATE until a work
 * list has been set (rb_multi_set_schedule or rb_multi_set_items); an empty one is a no-op.
 * Cites: paper, section "Manager-Based API", pipeline step "Simulate". */
int rb_multi_step(rb_multi* plan, void* hip_stream);

/* Capture nsteps fused steps into a graph on the (non-default) stream, replacing any earlier
 * capture.  RB_ESTATE without a work list.  Cites: paper, section "Architecture", paragraph
 * on the GPU physics backend (the simulation step recorded once as a graph and replayed). */
int rb_multi_graph_capture(rb_multi* plan, int32_t nsteps, void* hip_stream);

/* Replay the captured graph (all nsteps env steps) on a stream; RB_ESTATE when nothing has
 * been captured.  Cites: as rb_multi_graph_capture. */
int rb_multi_graph_launch(rb_multi* plan, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
