// Internal layout shared by the host runtime and the gfx950 step kernel.
//
// A compiled model is one device blob of 4-byte words holding the tables below; the kernel
// receives a DevModel by value with pointers into that blob.  Per-world working state lives
// in LDS (one wavefront per world); its layout (offsets in floats) is part of DevModel.
#pragma once
#include <stdint.h>

#define RB_WAVE 64
#define RB_MAX_WPG 4   // worlds (waves) per workgroup of the fused launch, at most
#define RB_MAX_DOF 64
#define RB_MAX_PAIR 128          // pairs are lanes, in two rounds past 64 (extended code only)
#define RB_MAX_CON 64
#define RB_MAX_GEOM 256           // contact ids pack geom indices into 8-bit fields
#define RB_NSTAGE 10              // timed kernel stages in the stats tap
#define RB_STATS_SUB 4            // substeps with a per-substep record in the stats tap
#define RB_STATS_FP 4             // Newton updates with an active-set fingerprint per substep
#define RB_SUBSTAT (5 + RB_STATS_FP)   // per-substep record columns
#define RB_NSTATS (4 + RB_NSTAGE + RB_STATS_SUB * RB_SUBSTAT)   // stats tap columns per world
#define RB_PAIR_BOXBOX 16         // pair_type of a box-box pair (plane pairs hold g2's geom type)
#define RB_PAIR_SPHEREBOX 17      // pair_type of a sphere (g1) - box (g2) pair
#define RB_PAIR_CAPSULEBOX 18     // pair_type of a capsule (g1) - box (g2) pair: its two end spheres
#define RB_PAIR_ROUND 19          // pair_type of a sphere or capsule (g1) - sphere or capsule (g2) pair
#define RB_PAIR_HFIELD 32         // pair_type of a height field (g1) - geom (g2) pair: this + g2's geom type
#define RB_BB_FLOATS 96           // LDS floats per box-box pair: clip buffers, contacts, normal
#define RB_MAX_GROW 64            // generic rows: equality rows and contacts' torsional / rolling rows
                                  // (one lane each; extended code only)
#define RB_GRF 12                 // LDS floats per generic row: psi[6], D, residual, J p, body, id, pad

struct DevModel {
    // sizes
    int nbody, nv, nq, nu, njnt, npair, ncap, maxd;
    int ngeom;
    int nbb;       // box-box pairs (each has an LDS block)
    int nblevel;   // body levels 1..nblevel (level 0 = world)
    int ndlevel;   // dof depth levels 1..ndlevel
    int K, maxiter;
    int fr_pw, ms_pw;
    int nM;        // packed tree-sparse matrix entries
    // options (float32)
    float dt, grav[3];
    float tol_scale;          // tolerance * meaninertia * nv
    float kref, bref;         // reference-acceleration stiffness and damping
    float dmin, dmax, width, mid, power;
    // bodies [nbody]
    const int* body_parent;
    const int* body_jtype;     // -1 none, RB_JNT_FREE, RB_JNT_HINGE
    const int* body_qadr;
    const int* body_dadr;
    const int* body_lastdof;   // deepest dof of the body's chain, -1 if the body cannot move
    const int* body_depth;     // number of dofs on the chain (0 if static)
    const int* body_level;
    const float* body_pos;     // [3]
    const float* body_quat;    // [4]
    const float* body_ipos;    // [3]
    const float* body_iquat;   // [4]
    const float* body_mass;
    const float* body_inertia; // [3]
    const float* body_jpos;    // [3] joint anchor in the body frame
    const float* body_jaxis;   // [3] unit hinge axis in the body frame
    const uint64_t* body_chainmask;  // bit i set iff dof i lies on the body's chain
    const int* level_start;    // [nblevel + 2] CSR into level_body, levels 0..nblevel
    const int* level_body;
    const int* child_start;    // [nbody + 1] CSR into child_list
    const int* child_list;
    // dofs [nv]
    const int* dof_body;
    const int* dof_depth;      // chain length including the dof itself
    const int* dof_rowadr;     // start of the dof's row in the packed matrices
    const int* dof_anc;        // [nv * maxd] dof at chain position t (root first), -1 padded
    const uint64_t* dof_descmask;  // bit k set iff dof k is a strict descendant of the dof
    const int* desc_start;     // [nv + 1] CSR of strict descendants
    const int* desc_list;
    const int* dof_height;     // steps from the dof to its deepest descendant leaf
    const int* hlevel_start;   // [nhlevel + 1] CSR of dofs by height above their deepest leaf
    const int* hlevel_dof;
    int nhlevel, maxpiv;       // height levels, most dofs in one height level
    const int* body_size;      // bodies in the subtree (bodies are in depth-first order)
    const int* body_children;  // up to 4 children, one byte each (0xff = none)
    const int* dlevel_start;   // [ndlevel + 2] CSR of dofs by depth, depths 1..ndlevel
    const int* dlevel_dof;
    const float* dof_armature;
    const int* dof_limq;       // qpos index of a limited hinge's angle, -1 if the dof is unlimited
    const float* dof_limlo;    // its lower and upper bounds
    const float* dof_limhi;
    int nlim;                  // limited hinges
    const float* dof_damping;  // hinge damping (0 when undamped)
    int ndamp;                 // damped hinges
    int ext;                   // level of extended code: 1 box-box and primitive-box pairs, height fields,
                               // joint limits, damping, condim 1; 2 also equality constraints, condim 4/6,
                               // elliptic cones; 3 also contacts between two moving bodies
    const int* act_start;      // [nv + 1] CSR of actuators driving each dof
    const int* act_list;
    const int* act_type;
    const int* act_qadr;
    const float* act_kp;
    const float* act_kd;
    const float* act_gear;
    // joints [njnt]
    const int* jnt_type;
    const int* jnt_qadr;
    const int* jnt_dadr;
    // collision pairs [npair], in (g1, g2) order; g1 is the plane, the sphere of a sphere-box
    // pair, the capsule of a capsule-box pair, or the lower-numbered box
    const int* pair_g1;
    const int* pair_g2;
    const int* pair_type;      // geom type of g2 (plane pairs), RB_PAIR_BOXBOX, RB_PAIR_SPHEREBOX, RB_PAIR_CAPSULEBOX,
                               // RB_PAIR_ROUND, or RB_PAIR_HFIELD + g2's type
    const int* pair_slot;      // box-box pairs: index of the pair's LDS block; -1 otherwise
    const int* pair_body;      // the body that can move
    const int* pair_cap;       // contacts the pair can produce
    const float* pair_sigma;   // +1 if the moving body carries g2, -1 if it carries g1
    const float* pair_mu;      // friction when it is not per world
    const float* pair_margin;
    const int* pair_frictionless;  // 1 when the pair's larger geom condim is 1 (normal row only)
    const int* geom_body;
    const int* geom_type;      // RB_GEOM_* per geom
    const float* geom_pos;     // [3]
    const float* geom_quat;    // [4]
    const float* geom_size;    // [3]
    const float* hf_data;      // height grid [hf_nrow, hf_ncol] of the height-field geoms (or null)
    int hf_nrow, hf_ncol;
    // equality constraints with the world [neq]; their rows [neqrow] (connect 3, weld 6)
    int neq, neqrow;
    int nxmax;                 // bound on the contacts' torsional / rolling rows (condim 4, 6 pairs)
    int cone;                  // 0 pyramidal, 1 elliptic friction cones (extended code)
    int nmm;                   // pairs of two moving bodies (level-3 code: dense Newton Hessian)
    const int* pair_body1;     // per pair: the second moving body (g1's), 0 when g1's body is static
    float impratio, rsqrt_impratio;
    const int* pair_xrows;     // per pair: 0, 2 (condim 4) or 6 (condim 6) rows per contact
    const int* pair_ellrows;   // per pair, elliptic cones: frame rows beyond three (1 spin: condim 4; 3 spin, rolling: 6)
    const float* pair_mu_spin;
    const float* pair_mu_roll;
    const int* eq_body;
    const float* eq_anchor;    // [3] body frame
    const float* eq_tpos;      // [3] world target point
    const float* eq_tmat;      // [9] world target orientation (welds)
    const int* eqrow_eq;       // the row's constraint
    const int* eqrow_k;        // 0..2 translational axis, 3..5 rotational axis
    // LDS layout (offsets in floats from the world's base)
    int o_q, o_v, o_ctrl, o_aws, o_mscale;
    int o_xpos, o_xmat, o_cinert, o_crb, o_cdof, o_cvel, o_bvec, o_bvec2;
    int o_tau, o_bias, o_a0, o_a, o_Ma, o_g, o_p, o_Mp, o_tmp, o_lD, o_ljar;
    int o_M, o_H, o_piv, o_rowadr, o_bb, o_gr, o_hd;
    int lds_floats;
};

// Per-world resident state owned by a batch.
struct DevWorlds {
    float* qacc_ws;         // [cap, nv]
    uint32_t* status;       // [cap]
    float* friction;        // [cap]
    float* mass_scale;      // [cap, nbody]
    // model fields expanded to one value per world (null: every world uses the model's)
    float* geom_size;       // [cap, ngeom, 3]
    float* body_pos;        // [cap, nbody, 3]
    float* act_kp;          // [cap, nu]
    float* act_kd;          // [cap, nu]
};

struct DevContactsOut {
    int32_t* ncon;
    int32_t* geom;
    int32_t* feature;
    float* dist;
    float* pos;
    float* frame;
    float* force;
};

struct DevTaps {
    float* M;
    float* bias;
    float* a0;
    float* qacc;
    float* efc;
    int32_t* stats;
};
