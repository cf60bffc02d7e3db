// Fused batched physics step for gfx950: one 64-lane wavefront advances one world through
// K substeps (controls held), with the world's working state staged in LDS.
//
// Per substep (paper, section "Manager-Based API", pipeline step "Simulate"; the contents of
// the step follow MuJoCo's published formulation, section "Architecture" cites it):
//   actuation -> forward kinematics -> spatial inertias and motion subspaces -> recursive
//   Newton-Euler bias forces -> composite-rigid-body inertia M -> tree-sparse L'DL of M ->
//   smooth acceleration a0 -> plane collision -> soft pyramidal contact rows -> primal Newton
//   with exact line search -> semi-implicit Euler.
//
// Lane mappings: bodies, dofs, joints, collision pairs and contacts are each spread one per
// lane; tree passes are level-synchronous over precomputed level lists.  Spatial vectors are
// Plucker coordinates in a world-aligned frame whose origin O is body 1's origin at the start
// of the substep (keeps FP32 cross products small).  Contacts live in registers (one per
// lane); the Newton Hessian keeps M's tree sparsity because every contact involves one
// moving body, so H = M + sum J'DJ factors in place without fill-in.
#include <hip/hip_runtime.h>

#include "rb_internal.h"
#include "rbstep.h"

#define DEV __device__ __forceinline__

namespace rbk {

// ------------------------------------------------------------------ wave utilities
DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// x from the lane selected by a DPP control (rows of 16 lanes); lanes without a source keep `old`
template <int CTRL, int ROWMASK>
DEV float dpp(float old, float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROWMASK, 0xf, false));
}
DEV float rl(float x, int c);
// Wave-wide sum: prefix sums within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row
// totals carried across rows (row_bcast 15, 31); lane 63 ends with the total, which is
// broadcast.  The association order is fixed, so the result is deterministic.
DEV float wsum(float x) {
    x += dpp<0x111, 0xf>(0.f, x);
    x += dpp<0x112, 0xf>(0.f, x);
    x += dpp<0x114, 0xf>(0.f, x);
    x += dpp<0x118, 0xf>(0.f, x);
    x += dpp<0x142, 0xa>(0.f, x);
    x += dpp<0x143, 0xc>(0.f, x);
    return rl(x, 63);
}
DEV float wmin(float x) {
    x = fminf(x, dpp<0x111, 0xf>(INFINITY, x));
    x = fminf(x, dpp<0x112, 0xf>(INFINITY, x));
    x = fminf(x, dpp<0x114, 0xf>(INFINITY, x));
    x = fminf(x, dpp<0x118, 0xf>(INFINITY, x));
    x = fminf(x, dpp<0x142, 0xa>(INFINITY, x));
    x = fminf(x, dpp<0x143, 0xc>(INFINITY, x));
    return rl(x, 63);
}
DEV int wscan_incl(int x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}
// wave-wide sum of unsigned 32-bit integers (modulo 2^32)
DEV uint32_t wsum_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o);
    return x;
}
DEV bool finitef(float x) { return __builtin_isfinite(x); }
// x, opaque to the optimiser at this point: values derived from it are computed where they are
// used instead of being hoisted out of loops (and then spilled) as loop invariants
DEV uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
// value of x in lane c (c uniform across the wave)
DEV float rl(float x, int c) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), c)); }

// ------------------------------------------------------------------ small vector math
DEV void cross(const float* a, const float* b, float* o) {
    float t0 = a[1] * b[2] - a[2] * b[1], t1 = a[2] * b[0] - a[0] * b[2], t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
DEV float dot(const float* a, const float* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
DEV void qmul(const float* a, const float* b, float* o) {
    float w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    float x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    float y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    float z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}
DEV void qmat(const float* q, float* R) {
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
DEV void mv(const float* R, const float* v, float* o) {
    float a = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    float b = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    float c = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
DEV void mm(const float* A, const float* B, float* O) {
    float t[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
#pragma unroll
    for (int i = 0; i < 9; i++) O[i] = t[i];
}

// spatial inertia about O stored as (m, h[3] = m c, I[6] = xx yy zz xy xz yz);
// product with a motion vector (w, v): (I w + h x v, m v - h x w)
DEV void inert_mul(const float* I, const float* s, float* f) {
    float m = I[0];
    const float* h = I + 1;
    const float* J = I + 4;
    float hv[3], hw[3];
    cross(h, s + 3, hv);
    cross(h, s, hw);
    f[0] = J[0] * s[0] + J[3] * s[1] + J[4] * s[2] + hv[0];
    f[1] = J[3] * s[0] + J[1] * s[1] + J[5] * s[2] + hv[1];
    f[2] = J[4] * s[0] + J[5] * s[1] + J[2] * s[2] + hv[2];
    f[3] = m * s[3] - hw[0];
    f[4] = m * s[4] - hw[1];
    f[5] = m * s[5] - hw[2];
}
// motion cross motion: (w, v) x (w', v') = (w x w', w x v' + v x w')
DEV void crm(const float* a, const float* b, float* o) {
    float t0[3], t1[3], t2[3];
    cross(a, b, t0);
    cross(a, b + 3, t1);
    cross(a + 3, b, t2);
    o[0] = t0[0]; o[1] = t0[1]; o[2] = t0[2];
    o[3] = t1[0] + t2[0]; o[4] = t1[1] + t2[1]; o[5] = t1[2] + t2[2];
}
// motion cross force: (w, v) x* (n, f) = (w x n + v x f, w x f)
DEV void crf(const float* a, const float* b, float* o) {
    float t0[3], t1[3], t2[3];
    cross(a, b, t0);
    cross(a + 3, b + 3, t1);
    cross(a, b + 3, t2);
    o[0] = t0[0] + t1[0]; o[1] = t0[1] + t1[1]; o[2] = t0[2] + t1[2];
    o[3] = t2[0]; o[4] = t2[1]; o[5] = t2[2];
}
DEV float sdot(const float* a, const float* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

// triangular pair index p -> (a, b) with b <= a
DEV void tri_decode(int p, int& a, int& b) {
    int t = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while (t * (t + 1) / 2 > p) t--;
    while ((t + 1) * (t + 2) / 2 <= p) t++;
    a = t;
    b = p - t * (t + 1) / 2;
}

// ------------------------------------------------------------------ tree-sparse L'DL
// In-place factorisation of a packed tree-sparse symmetric matrix (row i holds the entries
// of the dofs on i's chain, root first).  Leaves first: for each dof k, the outer product
// of its row updates the ancestor block, then the row is divided by its diagonal.  On exit
// row k holds L (unit lower triangle, ancestors of k) and D_k on the diagonal: M = L' D L.
template <int MAXD>
DEV void ldl_factor(const DevModel& m, float* buf, int lane) {
    for (int k = m.nv - 1; k >= 0; k--) {
        int dk = m.dof_depth[k] - 1;
        int rk = m.dof_rowadr[k];
        float invd = 1.0f / buf[rk + dk];
        int np = dk * (dk + 1) / 2;
        for (int p = lane; p < np; p += RB_WAVE) {
            int a, b;
            tri_decode(p, a, b);
            int i = m.dof_anc[k * m.maxd + a];
            float lka = buf[rk + a] * invd;
            buf[m.dof_rowadr[i] + b] -= lka * buf[rk + b];
        }
        wave_sync();
        if (lane < dk) buf[rk + lane] *= invd;
        wave_sync();
    }
}

// x <- M^-1 x with M = L'DL held in buf; level-parallel over dof depths.
DEV void ldl_solve(const DevModel& m, const float* buf, float* x, int lane) {
    // L' y = x: deepest dofs first, each dof pulls from its descendants
    for (int lev = m.ndlevel; lev >= 1; lev--) {
        for (int idx = m.dlevel_start[lev] + lane; idx < m.dlevel_start[lev + 1]; idx += RB_WAVE) {
            int i = m.dlevel_dof[idx];
            int col = m.dof_depth[i] - 1;
            float s = x[i];
            for (int c = m.desc_start[i]; c < m.desc_start[i + 1]; c++) {
                int k = m.desc_list[c];
                s -= buf[m.dof_rowadr[k] + col] * x[k];
            }
            x[i] = s;
        }
        wave_sync();
    }
    for (int i = lane; i < m.nv; i += RB_WAVE) x[i] /= buf[m.dof_rowadr[i] + m.dof_depth[i] - 1];
    wave_sync();
    // L x = z: root first, each dof pulls from its ancestors
    for (int lev = 1; lev <= m.ndlevel; lev++) {
        for (int idx = m.dlevel_start[lev] + lane; idx < m.dlevel_start[lev + 1]; idx += RB_WAVE) {
            int i = m.dlevel_dof[idx];
            int d = m.dof_depth[i] - 1;
            int r = m.dof_rowadr[i];
            float s = x[i];
            for (int t = 0; t < d; t++) s -= buf[r + t] * x[m.dof_anc[i * m.maxd + t]];
            x[i] = s;
        }
        wave_sync();
    }
}

// y = M x with M packed (lower rows) -- each dof pulls its chain and its descendants.
DEV void sym_mul(const DevModel& m, const float* M, const float* x, float* y, int lane) {
    for (int i = lane; i < m.nv; i += RB_WAVE) {
        int d = m.dof_depth[i];
        int r = m.dof_rowadr[i];
        float s = 0.f;
        for (int t = 0; t < d; t++) s += M[r + t] * x[m.dof_anc[i * m.maxd + t]];
        for (int c = m.desc_start[i]; c < m.desc_start[i + 1]; c++) {
            int k = m.desc_list[c];
            s += M[m.dof_rowadr[k] + d - 1] * x[k];
        }
        y[i] = s;
    }
    wave_sync();
}

// spatial motion of every body produced by dof vector x: out[b] = sum over the body's chain S_i x_i
// (the chain comes from the body's deepest dof lane).
template <typename BL_t, typename DL_t>
DEV void body_motion(const DevModel& m, const BL_t& BL, const DL_t& DL, const float* cdof, const float* x, float* out,
                     int lane) {
    constexpr int NW = sizeof(DL.anc) / sizeof(DL.anc[0]);
    uint32_t ba[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) ba[w] = (uint32_t)__shfl((int)DL.anc[w], BL.src);
    if (lane < m.nbody) {
        float acc[6] = {0, 0, 0, 0, 0, 0};
        for (int t = 0; t < BL.depth; t++) {
            const int i = (int)((ba[t >> 2] >> (8 * (t & 3))) & 0xffu);
            const float xi = x[i];
#pragma unroll
            for (int c = 0; c < 6; c++) acc[c] += cdof[6 * i + c] * xi;
        }
#pragma unroll
        for (int c = 0; c < 6; c++) out[6 * lane + c] = acc[c];
    }
    wave_sync();
}

// y = M x through the bodies: y_i = S_i . sum over the subtree of body(i) of I_b (J_b x),
// plus armature; `bm` receives the body motions J_b x and `bf` the body momenta I_b J_b x.
template <typename BL_t, typename DL_t>
DEV void spatial_mul(const DevModel& m, const BL_t& BL, const DL_t& DL, const float* cdof, const float* cinert,
                     const float* x, float* bm, float* bf, float* y, int lane) {
    body_motion(m, BL, DL, cdof, x, bm, lane);
    if (lane < m.nbody) {
        float f[6];
        inert_mul(cinert + 10 * lane, bm + 6 * lane, f);
#pragma unroll
        for (int c = 0; c < 6; c++) bf[6 * lane + c] = f[c];
    }
    wave_sync();
    if (lane < m.nv) {
        const int b0 = m.dof_body[lane], bs = m.body_size[b0];
        float F[6] = {0, 0, 0, 0, 0, 0};
        for (int b = b0; b < b0 + bs; b++)
#pragma unroll
            for (int c = 0; c < 6; c++) F[c] += bf[6 * b + c];
        y[lane] = sdot(cdof + 6 * lane, F) + m.dof_armature[lane] * x[lane];
    }
    wave_sync();
}

// ------------------------------------------------------------------ register-resident L'DL
// Per-lane constants of the dof held by the lane (lanes >= nv: depth 0).
template <int MAXD>
struct DofLane {
    int depth;             // chain length including the dof
    int rowadr;            // start of its row in the packed matrices
    int height;            // elimination level: steps to its deepest descendant leaf (-1 off lanes)
    uint64_t descmask;     // strict descendants
    uint32_t anc[MAXD / 4];   // chain dofs, root first, one byte each
    DEV int ancestor(int t) const { return (int)((anc[t >> 2] >> (8 * (t & 3))) & 0xffu); }
};

// Per-lane constants of the body held by the lane (lane b holds body b).
template <int MAXD>
struct BodyLane {
    int depth;             // dofs on the chain (0 for static bodies)
    uint64_t chainmask;    // dofs on the chain
    int src;               // the chain's deepest dof, whose lane holds the chain (0 if none)
};

// Constants used once per substep (tree passes, inertias) are read from the model tables in
// the stage that needs them rather than held in registers through the Newton loop: per body
// parent, joint type, qpos and dof address, level, packed children.
struct BodyTab { int parent, jtype, qadr, dadr, level; uint32_t children; };
DEV BodyTab body_tab(const DevModel& m, int lane) {
    if (lane >= m.nbody) return BodyTab{0, -1, 0, 0, -1, 0xffffffffu};
    return BodyTab{m.body_parent[lane], m.body_jtype[lane], m.body_qadr[lane], m.body_dadr[lane],
                   m.body_level[lane], (uint32_t)m.body_children[lane]};
}

template <int MAXD>
DEV DofLane<MAXD> load_dof_lane(const DevModel& m, int lane) {
    DofLane<MAXD> D;
    bool on = lane < m.nv;
    D.depth = on ? m.dof_depth[lane] : 0;
    D.rowadr = on ? m.dof_rowadr[lane] : 0;
    D.height = on ? m.dof_height[lane] : -1;
    D.descmask = on ? m.dof_descmask[lane] : 0ull;
#pragma unroll
    for (int w = 0; w < MAXD / 4; w++) D.anc[w] = 0u;
#pragma unroll
    for (int t = 0; t < MAXD; t++) {
        int a = (on && t < D.depth) ? m.dof_anc[lane * m.maxd + t] : 0;
        D.anc[t >> 2] |= (uint32_t)a << (8 * (t & 3));
    }
    return D;
}

template <int MAXD>
DEV BodyLane<MAXD> load_body_lane(const DevModel& m, const DofLane<MAXD>& DL, int lane) {
    BodyLane<MAXD> B;
    bool on = lane < m.nbody;
    B.chainmask = on ? m.body_chainmask[lane] : 0ull;
    int ld = on ? m.body_lastdof[lane] : -1;
    // the body's chain is the chain of its deepest dof: that dof lane holds it
    int src = ld < 0 ? 0 : ld;
    int dsrc = __shfl(DL.depth, src);
    B.depth = ld < 0 ? 0 : dsrc;
    B.src = src;
    return B;
}

// Factor the tree-sparse matrix whose row i (chain positions, root first) sits in lane i's
// registers Hr, as L'DL, and solve (L'DL) x = b for the lane's right-hand side bi.
// Leaves first: the pivot lane k publishes its row, its right-hand side y_k and 1/D_k in the
// LDS buffer piv; every lane reads the row back with broadcast loads and its own multiplier
// l_i = H_ki / D_k with one addressed load (0 for lanes that are not ancestors of k), then
// applies H_i. -= l_i H_k. and b_i -= l_i y_k (the L' solve rides along).  Updates land only
// in positions a lane never reads as data, so no lane masking is needed: an ancestor i of k
// (depth d_i < d_k) takes k's entries t < d_i, and everything from d_i on is its own padding;
// any other lane has l_i = 0 exactly.  Padding starts at zero and only ever receives
// multiples of other rows' entries, so it stays finite and rows are published whole.  Rows stay unscaled:
// L_ij = H_ij / D_i is applied in the L solve, which runs by depth level with one cross-lane
// shuffle per level.  On return Hr holds the unscaled factor rows, *inv_out = 1/D_i; returns x_i.
template <int MAXD>
DEV float factor_solve(const DevModel& m, const DofLane<MAXD>& D, float (&Hr)[MAXD], float bi, int lane,
                       float* piv, float* inv_out) {
    float inv_self = 0.f;
    const int di = D.depth;
    const int a = di - 1 < 0 ? 0 : di - 1;
    constexpr int STRIDE = MAXD + 4;
    // dofs of equal height never lie on each other's chain, so a whole height level is
    // eliminated in one step; an ancestor applies the level's pivots one after another
    for (int h = 0; h < m.nhlevel; h++) {
        // the level's pivots: a wave ballot over the lanes' heights, no table reads
        const bool mine = D.height == h;
        const uint64_t pmask = __ballot(mine);
        if (mine) {
            const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(pmask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)pmask, 0u));
            float* P = piv + slot * STRIDE;
            float4* P4 = reinterpret_cast<float4*>(P);
#pragma unroll
            for (int j = 0; j < MAXD / 4; j++) P4[j] = make_float4(Hr[4 * j], Hr[4 * j + 1], Hr[4 * j + 2], Hr[4 * j + 3]);
            P[MAXD] = bi;
        }
        wave_sync();
        uint64_t left = pmask;
        for (int pp = 0; left != 0ull; pp++) {
            const int k = __builtin_ctzll(left);
            left &= left - 1ull;
            const int dk = __builtin_amdgcn_readlane(di, k);
            const float* P = piv + pp * STRIDE;
            // pivot rows start on 16-byte boundaries (section offsets and the row stride are
            // multiples of four floats): read them four at a time
            float hk[MAXD];
            const float4* P4 = reinterpret_cast<const float4*>(P);
#pragma unroll
            for (int j = 0; j < MAXD / 4; j++) {
                const float4 x4 = P4[j];
                hk[4 * j] = x4.x; hk[4 * j + 1] = x4.y; hk[4 * j + 2] = x4.z; hk[4 * j + 3] = x4.w;
            }
            const float yk = P[MAXD];
            const float d = P[dk - 1];
            const bool anc = (D.descmask >> k) & 1ull;
            const float pa = P[a];               // a < MAXD: inside the published row
            const float hka = anc ? pa : 0.f;
            const float inv = __builtin_amdgcn_rcpf(d);
            if (lane == k) inv_self = inv;
            const float l = hka * inv;
            // l = 0 off the pivot's chain; positions past an ancestor's own depth are padding
            // (bounding the update by the pivot's depth with uniform branches measured slower)
#pragma unroll
            for (int b = 0; b < MAXD; b++) Hr[b] -= l * hk[b];
            bi -= l * yk;
        }
        wave_sync();
    }
    const float z = bi * inv_self;
    float acc = 0.f, x = 0.f;
#pragma unroll
    for (int t = 0; t < MAXD; t++) {
        if (t >= m.ndlevel) break;
        if (di == t + 1) x = z - acc * inv_self;
        const float xa = __shfl(x, D.ancestor(t));
        if (di > t + 1) acc += Hr[t] * xa;
    }
    *inv_out = inv_self;
    return x;
}

// ------------------------------------------------------------------ contacts (one per lane)
struct Con {
    float r[3];            // contact point relative to O
    float n[3], t1[3];     // normal and first tangent (t2 = n x t1)
    float mu, sigma, dist;
    int body;
    int body1;             // g1's body when both bodies move (rows of g2's minus g1's motion), else 0
    int ids;               // g1 | g2 << 8 | feature << 16
    // rows: the pyramid's four, or an elliptic contact's frame rows (normal, t1, t2, spin, and
    // the two rolling rows, used only by the extended instantiations)
    float D[6], aref[6], jar[6];
};

// velocity of the contact's pyramid rows for body spatial motions `bm` (already includes sign);
// of its frame rows for an elliptic-cone contact: normal, t1, t2, then the spin about n (ell 2
// or 3, else 0) and the rolling about t1 and t2 (ell 3; out [6]); b1 > 0: the contact's second
// moving body, whose motion is subtracted
DEV void rows_of(const Con& c, const float* bm, float* out, int ell = 0, int b1 = 0) {
    const float* sv = bm + 6 * c.body;
    float wr[3], t2[3];
    cross(sv, c.r, wr);
    cross(c.n, c.t1, t2);
    float vp[3] = {sv[3] + wr[0], sv[4] + wr[1], sv[5] + wr[2]};
    if (b1 > 0) {
        const float* s1 = bm + 6 * b1;
        float w1[3];
        cross(s1, c.r, w1);
        vp[0] -= s1[3] + w1[0]; vp[1] -= s1[4] + w1[1]; vp[2] -= s1[5] + w1[2];
    }
    float vn = c.sigma * dot(c.n, vp), v1 = c.sigma * dot(c.t1, vp), v2 = c.sigma * dot(t2, vp);
    if (ell) {
        float wa[3] = {sv[0], sv[1], sv[2]};   // angular motion, relative to b1's
        if (b1 > 0) {
            wa[0] -= bm[6 * b1]; wa[1] -= bm[6 * b1 + 1]; wa[2] -= bm[6 * b1 + 2];
        }
        out[0] = vn; out[1] = v1; out[2] = v2;
        out[3] = ell >= 2 ? c.sigma * dot(c.n, wa) : 0.f;
        if (ell == 3) {
            out[4] = c.sigma * dot(c.t1, wa);
            out[5] = c.sigma * dot(t2, wa);
        }
        return;
    }
    out[0] = vn + c.mu * v1;
    out[1] = vn - c.mu * v1;
    out[2] = vn + c.mu * v2;
    out[3] = vn - c.mu * v2;
}

// Soft elliptic cone of one contact at its frame-row residuals jar [6] (normal, t1, t2, spin about
// n, rolling about t1 and t2), with regulariser inverses D0 (normal), Dt (tangents), Ds (spin)
// and Dr (rolling; 0 for the rows a contact does not have, which leaves the smaller cone) and
// cone slope mu: with x = sqrt(D) jar, cost 0 when mu |x_t| <= x_n (separating), |x|^2 / 2 when
// |x_t| <= -mu x_n (inside the cone), else (mu |x_t| - x_n)^2 / (2 (1 + mu^2)) (the force on the
// cone's surface).  ell_eval returns the zone (0, 1 surface, 2 inside), the cost and
// g = d cost / d jar [6], and keeps what the Hessian's products need: on the surface the Hessian
// is diag(sqrt D) c (w w' + k (I - u u') on the friction block) diag(sqrt D), w the gradient of
// mu |x_t| - x_n in x, u = x_t / |x_t|, c = 1 / (1 + mu^2), k = (mu |x_t| - x_n) mu / |x_t|;
// inside the cone it is diag(D).  The products are formed from these in O(rows), never the
// 6 x 6 matrix.
struct EllCone {
    int zone;
    float c, k, mu;
    float sq[6];   // sqrt(D) per row
    float u[6];    // u[0] unused
};

// NE: the rows the instantiation carries (4: normal, tangents, spin; 6: also rolling); jar, g and
// the products' vectors have NE entries.
template <int NE>
DEV int ell_eval(const float* jar, float D0, float Dt, float Ds, float Dr, float mu, float* cost, float* g,
                 EllCone* E) {
    const float st = sqrtf(Dt);
    E->sq[0] = sqrtf(D0); E->sq[1] = st; E->sq[2] = st; E->sq[3] = sqrtf(Ds);
    if (NE > 4) E->sq[4] = E->sq[5] = sqrtf(Dr);
    E->mu = mu;
    float x[NE], T2 = 0.f;
#pragma unroll
    for (int a = 0; a < NE; a++) x[a] = E->sq[a] * jar[a];
#pragma unroll
    for (int a = 1; a < NE; a++) T2 += x[a] * x[a];
    const float N = x[0], T = sqrtf(T2);
#pragma unroll
    for (int k = 0; k < NE; k++) g[k] = 0.f;
    *cost = 0.f;
    E->c = E->k = 0.f;
#pragma unroll
    for (int a = 0; a < NE; a++) E->u[a] = 0.f;
    if (mu * T <= N) return E->zone = 0;
    if (T <= -mu * N) {
        const float Dd[6] = {D0, Dt, Dt, Ds, Dr, Dr};
        float cs = N * N;
#pragma unroll
        for (int a = 1; a < NE; a++) cs += x[a] * x[a];
        *cost = 0.5f * cs;
#pragma unroll
        for (int a = 0; a < NE; a++) g[a] = Dd[a] * jar[a];
        return E->zone = 2;
    }
    const float c = 1.f / (1.f + mu * mu), hh = mu * T - N, iT = 1.f / T;
    E->c = c;
    E->k = hh * mu * iT;
#pragma unroll
    for (int a = 1; a < NE; a++) E->u[a] = x[a] * iT;
    *cost = 0.5f * c * hh * hh;
    g[0] = E->sq[0] * c * hh * -1.f;
#pragma unroll
    for (int a = 1; a < NE; a++) {
        const float wa = mu * E->u[a];   // the gradient of mu |x_t| - x_n in x
        g[a] = E->sq[a] * c * hh * wa;
    }
    return E->zone = 1;
}

// out = H v for the cone's Hessian H (zone 0: 0)
template <int NE>
DEV void ell_hv(const EllCone& E, const float* v, float* out) {
    float y[NE];
#pragma unroll
    for (int a = 0; a < NE; a++) y[a] = E.sq[a] * v[a];
    if (E.zone == 2) {
#pragma unroll
        for (int a = 0; a < NE; a++) out[a] = E.sq[a] * y[a];
        return;
    }
    float uy = 0.f;
#pragma unroll
    for (int a = 1; a < NE; a++) uy += E.u[a] * y[a];
    const float wy = E.mu * uy - y[0];
    out[0] = -E.sq[0] * E.c * wy;
#pragma unroll
    for (int a = 1; a < NE; a++) out[a] = E.sq[a] * E.c * (E.mu * E.u[a] * wy + E.k * (y[a] - E.u[a] * uy));
}

// v' H v
template <int NE>
DEV float ell_vhv(const EllCone& E, const float* v) {
    float y[NE];
#pragma unroll
    for (int a = 0; a < NE; a++) y[a] = E.sq[a] * v[a];
    float yy = 0.f, uy = 0.f;
#pragma unroll
    for (int a = 1; a < NE; a++) {
        yy += y[a] * y[a];
        uy += E.u[a] * y[a];
    }
    if (E.zone == 2) return y[0] * y[0] + yy;
    const float wy = E.mu * uy - y[0];
    return E.c * (wy * wy + E.k * (yy - uy * uy));
}

DEV void contact_frame(const float* n, float* t1) {
    int k = 0;
    if (fabsf(n[1]) < fabsf(n[k])) k = 1;
    if (fabsf(n[2]) < fabsf(n[k])) k = 2;
    float e[3] = {0.f, 0.f, 0.f};
    e[k] = 1.f;
    float dn = n[k];
    float t[3] = {e[0] - dn * n[0], e[1] - dn * n[1], e[2] - dn * n[2]};
    float inv = 1.0f / sqrtf(dot(t, t));
    t1[0] = t[0] * inv; t1[1] = t[1] * inv; t1[2] = t[2] * inv;
}

// world pose of geom g from its body's pose in LDS
DEV void geom_pose(const DevModel& m, const float* L, int g, float* x, float* R) {
    int b = m.geom_body[g];
    const float* Rb = L + m.o_xmat + 9 * b;
    float off[3];
    mv(Rb, m.geom_pos + 3 * g, off);
    x[0] = L[m.o_xpos + 3 * b] + off[0];
    x[1] = L[m.o_xpos + 3 * b + 1] + off[1];
    x[2] = L[m.o_xpos + 3 * b + 2] + off[2];
    float Rg[9];
    qmat(m.geom_quat + 4 * g, Rg);
    mm(Rb, Rg, R);
}

DEV float pick3(const float* a, int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }

// Candidate contacts of a plane pair, in feature order: sphere 0; capsule ends 0 (-z), 1 (+z);
// box vertices k = 4x + 2y + z by sign bits.  A sphere-box pair has the one candidate 0.
DEV int pair_ncand(int type) {
    if (type >= RB_PAIR_HFIELD) type -= RB_PAIR_HFIELD;   // a height field: as the plane
    return (type == RB_GEOM_SPHERE || type == RB_PAIR_SPHEREBOX || type == RB_PAIR_ROUND) ? 1
           : (type == RB_GEOM_CAPSULE || type == RB_PAIR_CAPSULEBOX) ? 2
                                                                     : 8;
}

// The plane of the height-field triangle under world point e (by its local x and y): outward
// (local +z side) unit normal n and vertex p0; false when e lies outside the grid.  Rows run
// along local y, columns along x; a cell is split along its diagonal from sample (i, j) to
// (i + 1, j + 1).
DEV bool hfield_plane(const DevModel& m, const float* gsize, int g, const float* xg, const float* Rg, const float* e,
                      float* n, float* p0) {
    const float sx = gsize[3 * g], sy = gsize[3 * g + 1];
    const float rel[3] = {e[0] - xg[0], e[1] - xg[1], e[2] - xg[2]};
    const float lx = Rg[0] * rel[0] + Rg[3] * rel[1] + Rg[6] * rel[2];
    const float ly = Rg[1] * rel[0] + Rg[4] * rel[1] + Rg[7] * rel[2];
    const int nr = m.hf_nrow, nc = m.hf_ncol;
    const float u = (lx + sx) / (2.f * sx) * (float)(nc - 1), v = (ly + sy) / (2.f * sy) * (float)(nr - 1);
    if (!(u >= 0.f && u <= (float)(nc - 1) && v >= 0.f && v <= (float)(nr - 1))) return false;
    const int j = min((int)floorf(u), nc - 2), i = min((int)floorf(v), nr - 2);
    auto vert = [&](int a, int b, float* P) {
        P[0] = -sx + 2.f * sx * (float)b / (float)(nc - 1);
        P[1] = -sy + 2.f * sy * (float)a / (float)(nr - 1);
        P[2] = m.hf_data[a * nc + b];
    };
    float P0[3], P1[3], P2[3];
    vert(i, j, P0);
    if (u - (float)j >= v - (float)i) {
        vert(i, j + 1, P1);
        vert(i + 1, j + 1, P2);
    } else {
        vert(i + 1, j + 1, P1);
        vert(i + 1, j, P2);
    }
    const float a[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    const float b[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    float nl[3];
    cross(a, b, nl);
    const float il = 1.0f / sqrtf(dot(nl, nl));
    nl[0] *= il; nl[1] *= il; nl[2] *= il;
    mv(Rg, nl, n);
    float pw[3];
    mv(Rg, P0, pw);
    p0[0] = xg[0] + pw[0]; p0[1] = xg[1] + pw[1]; p0[2] = xg[2] + pw[2];
    return true;
}

// Candidate k of plane pair p: distance to the plane, contact point (halfway between the
// surfaces) and the plane normal.  Sphere-box pair: the box's point closest to the sphere's
// centre c (c clamped to the box in its frame), or the nearest face when c is inside (least
// depth, lowest axis on ties, + side at 0); distance |c - closest| - r outside, -(depth + r)
// inside; normal from the sphere towards the box.  Capsule-box pair: candidate k is the sphere
// at the capsule's segment end k (0 at -z, 1 at +z) against the box by the same rule.
template <int EXT>
DEV void pair_candidate(const DevModel& m, const float* L, const float* gsize, int p, int k, float* dist, float* pos,
                        float* nrm) {
    float xp[3], Rp[9], x[3], R[9];
    geom_pose(m, L, m.pair_g1[p], xp, Rp);
    geom_pose(m, L, m.pair_g2[p], x, R);
    const float* sz = gsize + 3 * m.pair_g2[p];
    const int type = m.pair_type[p];
    if (EXT && type == RB_PAIR_ROUND) {
        // spheres and capsules: segments (a sphere's of length 0) swept by their radii; the
        // closest points of the two segments (Ericson, Real-Time Collision Detection, section
        // 5.1.9; nearly parallel segments, a e - b^2 <= 1e-6 a e, take s = 0), the contact
        // joining them from g1 to g2 (+z when they coincide), halfway between the surfaces
        const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
        const float h1 = m.geom_type[g1] == RB_GEOM_CAPSULE ? gsize[3 * g1 + 1] : 0.f;
        const float h2 = m.geom_type[g2] == RB_GEOM_CAPSULE ? gsize[3 * g2 + 1] : 0.f;
        const float d1[3] = {2.f * h1 * Rp[2], 2.f * h1 * Rp[5], 2.f * h1 * Rp[8]};
        const float d2[3] = {2.f * h2 * R[2], 2.f * h2 * R[5], 2.f * h2 * R[8]};
        const float p1[3] = {xp[0] - h1 * Rp[2], xp[1] - h1 * Rp[5], xp[2] - h1 * Rp[8]};
        const float p2[3] = {x[0] - h2 * R[2], x[1] - h2 * R[5], x[2] - h2 * R[8]};
        const float rr[3] = {p1[0] - p2[0], p1[1] - p2[1], p1[2] - p2[2]};
        const float a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, rr);
        auto clamp01 = [](float v) { return fminf(fmaxf(v, 0.f), 1.f); };
        float s = 0.f, t = 0.f;
        if (a <= 1e-12f && e <= 1e-12f) {
        } else if (a <= 1e-12f) {
            t = clamp01(f / e);
        } else {
            const float c = dot(d1, rr);
            if (e <= 1e-12f) {
                s = clamp01(-c / a);
            } else {
                const float b = dot(d1, d2), den = a * e - b * b;
                s = den > 1e-6f * a * e ? clamp01((b * f - c * e) / den) : 0.f;
                t = (b * s + f) / e;
                if (t < 0.f) {
                    t = 0.f;
                    s = clamp01(-c / a);
                } else if (t > 1.f) {
                    t = 1.f;
                    s = clamp01((b - c) / a);
                }
            }
        }
        const float c1[3] = {p1[0] + d1[0] * s, p1[1] + d1[1] * s, p1[2] + d1[2] * s};
        const float c2[3] = {p2[0] + d2[0] * t, p2[1] + d2[1] * t, p2[2] + d2[2] * t};
        float n[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
        const float len = sqrtf(dot(n, n));
        if (len > 0.f) {
            const float il = 1.0f / len;
            n[0] *= il; n[1] *= il; n[2] *= il;
        } else {
            n[0] = 0.f; n[1] = 0.f; n[2] = 1.f;
        }
        const float r1 = gsize[3 * g1], r2 = gsize[3 * g2];
        const float dd = len - r1 - r2;
        *dist = dd;
        nrm[0] = n[0]; nrm[1] = n[1]; nrm[2] = n[2];
        const float hh = r1 + 0.5f * dd;
        pos[0] = c1[0] + n[0] * hh; pos[1] = c1[1] + n[1] * hh; pos[2] = c1[2] + n[2] * hh;
        return;
    }
    if (EXT && (type == RB_PAIR_SPHEREBOX || type == RB_PAIR_CAPSULEBOX)) {
        const float rad = gsize[3 * m.pair_g1[p]];
        if (type == RB_PAIR_CAPSULEBOX) {
            // the segment end: the sphere's centre
            const float hl = k == 0 ? -gsize[3 * m.pair_g1[p] + 1] : gsize[3 * m.pair_g1[p] + 1];
            xp[0] += hl * Rp[2]; xp[1] += hl * Rp[5]; xp[2] += hl * Rp[8];
        }
        const float rel[3] = {xp[0] - x[0], xp[1] - x[1], xp[2] - x[2]};
        float pl[3], ql[3];
        bool inside = true;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            pl[i] = R[i] * rel[0] + R[3 + i] * rel[1] + R[6 + i] * rel[2];
            ql[i] = fminf(fmaxf(pl[i], -sz[i]), sz[i]);
            inside = inside && ql[i] == pl[i];
        }
        float nl[3] = {0.f, 0.f, 0.f}, d;
        if (!inside) {
            const float df[3] = {pl[0] - ql[0], pl[1] - ql[1], pl[2] - ql[2]};
            const float len = sqrtf(dot(df, df));
            const float il = 1.0f / len;
            nl[0] = df[0] * il; nl[1] = df[1] * il; nl[2] = df[2] * il;
            d = len - rad;
        } else {
            int a = 0;
            if (sz[1] - fabsf(pl[1]) < sz[a] - fabsf(pl[a])) a = 1;
            if (sz[2] - fabsf(pl[2]) < sz[a] - fabsf(pl[a])) a = 2;
            const float pa = pick3(pl, a), ha = pick3(sz, a);
            const float sg = pa < 0.f ? -1.f : 1.f;
            nl[0] = a == 0 ? sg : 0.f; nl[1] = a == 1 ? sg : 0.f; nl[2] = a == 2 ? sg : 0.f;
            d = -(ha - fabsf(pa) + rad);
        }
        float nw[3];
        mv(R, nl, nw);
        nrm[0] = -nw[0]; nrm[1] = -nw[1]; nrm[2] = -nw[2];
        *dist = d;
        const float h = rad + 0.5f * d;
        pos[0] = xp[0] - nw[0] * h; pos[1] = xp[1] - nw[1] * h; pos[2] = xp[2] - nw[2] * h;
        return;
    }
    // a plane, or a height field: the plane of the triangle under the candidate point
    const bool hf = EXT && type >= RB_PAIR_HFIELD;
    const int shape = hf ? type - RB_PAIR_HFIELD : type;
    float n[3] = {Rp[2], Rp[5], Rp[8]};
    float e[3], rad = 0.f;
    if (shape == RB_GEOM_SPHERE) {
        e[0] = x[0]; e[1] = x[1]; e[2] = x[2];
        rad = sz[0];
    } else if (shape == RB_GEOM_CAPSULE) {
        const float sgn = k == 0 ? -sz[1] : sz[1];
        e[0] = x[0] + sgn * R[2]; e[1] = x[1] + sgn * R[5]; e[2] = x[2] + sgn * R[8];
        rad = sz[0];
    } else {
        const float loc[3] = {(k & 4) ? sz[0] : -sz[0], (k & 2) ? sz[1] : -sz[1], (k & 1) ? sz[2] : -sz[2]};
        mv(R, loc, e);
        e[0] += x[0]; e[1] += x[1]; e[2] += x[2];
    }
    float p0[3] = {xp[0], xp[1], xp[2]};
    if (hf && !hfield_plane(m, gsize, m.pair_g1[p], xp, Rp, e, n, p0)) {
        *dist = INFINITY;   // off the grid: no contact
        nrm[0] = n[0]; nrm[1] = n[1]; nrm[2] = n[2];
        pos[0] = e[0]; pos[1] = e[1]; pos[2] = e[2];
        return;
    }
    nrm[0] = n[0]; nrm[1] = n[1]; nrm[2] = n[2];
    const float r[3] = {e[0] - p0[0], e[1] - p0[1], e[2] - p0[2]};
    const float d = dot(n, r) - rad;
    *dist = d;
    const float h = rad + 0.5f * d;
    pos[0] = e[0] - n[0] * h; pos[1] = e[1] - n[1] * h; pos[2] = e[2] - n[2] * h;
}

// Bit k set iff candidate k of plane pair p is below the margin.  Computed once per pair; the
// contact lanes then pick their candidate from these bits, so membership never depends on
// re-evaluating a distance that sits on the margin.
template <int EXT>
DEV uint32_t pair_mask(const DevModel& m, const float* L, const float* gsize, int p) {
    const int nc = pair_ncand(m.pair_type[p]);
    const float margin = m.pair_margin[p];
    uint32_t mask = 0;
    for (int k = 0; k < nc; k++) {
        float d, pos[3], nrm[3];
        pair_candidate<EXT>(m, L, gsize, p, k, &d, pos, nrm);
        if (d < margin) mask |= 1u << k;
    }
    return mask;
}

DEV void pick_axis(const float (&a)[3][3], int i, float* o) {
#pragma unroll
    for (int k = 0; k < 3; k++) o[k] = i == 0 ? a[0][k] : (i == 1 ? a[1][k] : a[2][k]);
}

// Box-box contacts of pair p by the separating-axis test (Ericson, Real-Time Collision
// Detection, 2004, sections 4.4 and 5.2), written into the pair's LDS block S:
//   S[0, 24), S[24, 48)   clip buffers (8 points each)
//   S[48 + 5 j ...]       contact j: dist, pos[3], feature
//   S[88, 91)             normal, from g1 towards g2
// The 15 candidate axes are the 6 face normals and the 9 normalised edge cross products
// (skipped when nearly parallel).  The axis of least overlap wins; a later axis displaces an
// earlier one only when smaller by more than 1e-5 (1 + overlap).  A face axis clips the
// incident face (the other box's face most anti-parallel to the reference face) against the
// reference face's four side planes; every clipped point below the reference face is a
// contact, placed halfway between the point and the face, numbered by its position in the
// clipped polygon.  An edge axis gives one contact halfway between the closest points of
// the two supporting edges, at depth minus the overlap.  Returns the number of contacts.
DEV int box_box(const DevModel& m, const float* L, const float* gsize, int p, float* S) {
    float cA[3], RA[9], cB[3], RB[9];
    const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
    geom_pose(m, L, g1, cA, RA);
    geom_pose(m, L, g2, cB, RB);
    const float hA[3] = {gsize[3 * g1], gsize[3 * g1 + 1], gsize[3 * g1 + 2]};
    const float hB[3] = {gsize[3 * g2], gsize[3 * g2 + 1], gsize[3 * g2 + 2]};
    const float margin = m.pair_margin[p];
    float aA[3][3], aB[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            aA[i][k] = RA[3 * k + i];
            aB[i][k] = RB[3 * k + i];
        }
    const float dc[3] = {cB[0] - cA[0], cB[1] - cA[1], cB[2] - cA[2]};
    int best = -1;
    float best_ov = 0.f, bx[3] = {0.f, 0.f, 0.f};
    bool separated = false;
#pragma unroll
    for (int ax = 0; ax < 15; ax++) {
        float Lx[3];
        bool skip = false;
        if (ax < 3) {
            Lx[0] = aA[ax][0]; Lx[1] = aA[ax][1]; Lx[2] = aA[ax][2];
        } else if (ax < 6) {
            Lx[0] = aB[ax - 3][0]; Lx[1] = aB[ax - 3][1]; Lx[2] = aB[ax - 3][2];
        } else {
            cross(aA[(ax - 6) / 3], aB[(ax - 6) % 3], Lx);
            float nl = sqrtf(dot(Lx, Lx));
            skip = nl < 1e-6f;
            float inv = skip ? 0.f : 1.0f / nl;
            Lx[0] *= inv; Lx[1] *= inv; Lx[2] *= inv;
        }
        float rA = hA[0] * fabsf(dot(Lx, aA[0])) + hA[1] * fabsf(dot(Lx, aA[1])) + hA[2] * fabsf(dot(Lx, aA[2]));
        float rB = hB[0] * fabsf(dot(Lx, aB[0])) + hB[1] * fabsf(dot(Lx, aB[1])) + hB[2] * fabsf(dot(Lx, aB[2]));
        float ov = rA + rB - fabsf(dot(Lx, dc));
        if (!skip) {
            separated = separated || (-ov >= margin);
            if (best < 0 || ov < best_ov - 1e-5f * (1.f + fabsf(best_ov))) {
                best = ax;
                best_ov = ov;
                bx[0] = Lx[0]; bx[1] = Lx[1]; bx[2] = Lx[2];
            }
        }
    }
    if (separated || best < 0) return 0;
    const float sgn = dot(bx, dc) < 0.f ? -1.f : 1.f;
    const float n[3] = {sgn * bx[0], sgn * bx[1], sgn * bx[2]};
    S[88] = n[0]; S[89] = n[1]; S[90] = n[2];
    if (best >= 6) {
        const int i = (best - 6) / 3, j = (best - 6) % 3;
        float PA[3] = {cA[0], cA[1], cA[2]}, PB[3] = {cB[0], cB[1], cB[2]};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            float sa = a == i ? 0.f : (dot(n, aA[a]) >= 0.f ? hA[a] : -hA[a]);
            float sb = a == j ? 0.f : (dot(n, aB[a]) >= 0.f ? -hB[a] : hB[a]);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                PA[k] += sa * aA[a][k];
                PB[k] += sb * aB[a][k];
            }
        }
        float ei[3], ej[3];
        pick_axis(aA, i, ei);
        pick_axis(aB, j, ej);
        const float hi = pick3(hA, i), hj = pick3(hB, j);
        const float r[3] = {PA[0] - PB[0], PA[1] - PB[1], PA[2] - PB[2]};
        const float b = dot(ei, ej), c = dot(ei, r), f = dot(ej, r);
        const float den = 1.f - b * b;
        float t = den > 1e-12f ? (b * f - c) / den : 0.f;
        t = fminf(fmaxf(t, -hi), hi);
        float w = b * t + f;
        if (w < -hj || w > hj) {
            w = fminf(fmaxf(w, -hj), hj);
            t = fminf(fmaxf(b * w - c, -hi), hi);
        }
        S[48] = -best_ov;
#pragma unroll
        for (int k = 0; k < 3; k++) S[49 + k] = 0.5f * (PA[k] + t * ei[k] + PB[k] + w * ej[k]);
        S[52] = 0.f;
        return 1;
    }
    // face axis: reference box R, incident box I
    const bool refA = best < 3;
    const int rax = refA ? best : best - 3;
    float aR[3][3], aI[3][3], hR[3], hI[3], cR[3], cI[3], nr[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        hR[a] = refA ? hA[a] : hB[a];
        hI[a] = refA ? hB[a] : hA[a];
        cR[a] = refA ? cA[a] : cB[a];
        cI[a] = refA ? cB[a] : cA[a];
        nr[a] = refA ? n[a] : -n[a];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            aR[a][k] = refA ? aA[a][k] : aB[a][k];
            aI[a][k] = refA ? aB[a][k] : aA[a][k];
        }
    }
    const float hr = pick3(hR, rax);
    const float pR[3] = {cR[0] + hr * nr[0], cR[1] + hr * nr[1], cR[2] + hr * nr[2]};
    // side axes of the reference face, in increasing axis order
    const int u = rax == 0 ? 1 : 0, v = rax == 2 ? 1 : 2;
    float du[3], dv[3];
    pick_axis(aR, u, du);
    pick_axis(aR, v, dv);
    const float hu = pick3(hR, u), hv = pick3(hR, v);
    int ia = 0;
    float bestdot = -1.f;
#pragma unroll
    for (int jj = 0; jj < 3; jj++) {
        float a = fabsf(dot(aI[jj], nr));
        if (a > bestdot + 1e-12f) { bestdot = a; ia = jj; }
    }
    float ea[3];
    pick_axis(aI, ia, ea);
    const float s = dot(ea, nr) > 0.f ? -1.f : 1.f;
    const int pa = ia == 0 ? 1 : 0, qa = ia == 2 ? 1 : 2;
    float ep[3], eq[3];
    pick_axis(aI, pa, ep);
    pick_axis(aI, qa, eq);
    const float hia = pick3(hI, ia), hp = pick3(hI, pa), hq = pick3(hI, qa);
    float* buf = S;
    float* out = S + 24;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const float sp = (c == 0 || c == 3) ? 1.f : -1.f, sq = c < 2 ? 1.f : -1.f;
#pragma unroll
        for (int k = 0; k < 3; k++) buf[3 * c + k] = cI[k] + s * hia * ea[k] + sp * hp * ep[k] + sq * hq * eq[k];
    }
    int np = 4;
    // Sutherland-Hodgman against x.u <= hu, -x.u <= hu, x.v <= hv, -x.v <= hv (x = point - pR)
#pragma unroll
    for (int plane = 0; plane < 4; plane++) {
        const float* dir = plane < 2 ? du : dv;
        const float ext = plane < 2 ? hu : hv;
        const float sg = (plane & 1) ? -1.f : 1.f;
        int no = 0;
        for (int a = 0; a < np; a++) {
            const int b2 = a + 1 == np ? 0 : a + 1;
            const float P[3] = {buf[3 * a], buf[3 * a + 1], buf[3 * a + 2]};
            const float Q[3] = {buf[3 * b2], buf[3 * b2 + 1], buf[3 * b2 + 2]};
            const float x[3] = {P[0] - pR[0], P[1] - pR[1], P[2] - pR[2]};
            const float y[3] = {Q[0] - pR[0], Q[1] - pR[1], Q[2] - pR[2]};
            const float fp = sg * dot(x, dir) - ext, fq = sg * dot(y, dir) - ext;
            // a convex quad clipped by four half-planes keeps at most 8 points; the bound
            // also holds the buffers when rounding bends the polygon
            if (fp <= 0.f && no < 8) {
                out[3 * no] = P[0]; out[3 * no + 1] = P[1]; out[3 * no + 2] = P[2];
                no++;
            }
            if (((fp < 0.f && fq > 0.f) || (fp > 0.f && fq < 0.f)) && no < 8) {
                const float t = fp / (fp - fq);
                out[3 * no] = P[0] + t * (Q[0] - P[0]);
                out[3 * no + 1] = P[1] + t * (Q[1] - P[1]);
                out[3 * no + 2] = P[2] + t * (Q[2] - P[2]);
                no++;
            }
        }
        float* tmpb = buf; buf = out; out = tmpb;
        np = no;
        if (np == 0) return 0;
    }
    int cnt = 0;
    for (int a = 0; a < np; a++) {
        const float x[3] = {buf[3 * a] - pR[0], buf[3 * a + 1] - pR[1], buf[3 * a + 2] - pR[2]};
        const float dd = dot(x, nr);
        if (dd < margin) {
            float* o = S + 48 + 5 * cnt;
            o[0] = dd;
            o[1] = buf[3 * a] - 0.5f * dd * nr[0];
            o[2] = buf[3 * a + 1] - 0.5f * dd * nr[1];
            o[3] = buf[3 * a + 2] - 0.5f * dd * nr[2];
            o[4] = (float)a;
            cnt++;
        }
    }
    return cnt;
}

DEV float impedance(const DevModel& m, float r) {
    float x = fminf(fabsf(r) / m.width, 1.0f);
    float y;
    if (x <= m.mid)
        y = powf(x, m.power) / powf(m.mid, m.power - 1.0f);
    else
        y = 1.0f - powf(1.0f - x, m.power) / powf(1.0f - m.mid, m.power - 1.0f);
    float imp = m.dmin + y * (m.dmax - m.dmin);
    return fminf(fmaxf(imp, 1e-4f), 0.9999f);
}

// ------------------------------------------------------------------ the kernel
struct StepArgs {
    int n;
    const float* ctrl;
    float* qpos;
    float* qvel;
    DevWorlds W;
    DevContactsOut co;
    uint32_t* status_out;
    DevTaps taps;
    int want_contacts, want_taps;
};

// MAXD: longest dof chain the instantiation supports; TIMED: the diagnostic instantiation that
// serves rb_step_taps (stage taps, work totals and per-stage shader-clock cycles); the plain
// instantiation carries none of that code.  EXT: the level of extended code -- 1: box-box,
// sphere-box and capsule-box pairs, more than 64 pairs, frictionless pairs, joint limits and
// joint damping; 2: also generic rows (equality constraints, pyramidal torsional / rolling rows)
// and elliptic cones up to condim 4; 3: level 2 and contacts between two moving bodies; 4: level
// 2 with elliptic cones up to condim 6 (two more rows per contact lane).  Each model runs the
// lowest level that has its features.
#ifndef RB_WAVES_PER_EU
#define RB_WAVES_PER_EU 3
#endif
template <int MAXD, bool TIMED, int EXT>
DEV void world_step(const DevModel& m, const StepArgs& A, const int w, float* lds) {
    // an elliptic contact's frame rows: normal, tangents and spin; with the rolling rows too in the
    // level-4 instantiation (elliptic cones with condim 6)
    constexpr int NE = EXT == 4 ? 6 : 4;
    const int lane = threadIdx.x & (RB_WAVE - 1);   // a fused workgroup may hold several worlds
    float* L = lds;
    float* q = L + m.o_q;
    float* v = L + m.o_v;
    float* ctrl = L + m.o_ctrl;
    float* aws = L + m.o_aws;
    float* msc = L + m.o_mscale;
    float* xpos = L + m.o_xpos;
    float* xmat = L + m.o_xmat;
    float* cinert = L + m.o_cinert;
    float* crb = L + m.o_crb;
    float* cdof = L + m.o_cdof;
    float* cvel = L + m.o_cvel;
    float* bvec = L + m.o_bvec;
    float* bvec2 = L + m.o_bvec2;
    float* tau = L + m.o_tau;
    float* bias = L + m.o_bias;
    float* a0 = L + m.o_a0;
    float* acc = L + m.o_a;
    float* Ma = L + m.o_Ma;
    float* g = L + m.o_g;
    float* p = L + m.o_p;
    float* Mp = L + m.o_Mp;
    float* tmp = L + m.o_tmp;
    float* Mm = L + m.o_M;
    float* H = L + m.o_H;
    float* piv = L + m.o_piv;

    const int nq = m.nq, nv = m.nv, nu = m.nu, nb = m.nbody;
    const DofLane<MAXD> DL = load_dof_lane<MAXD>(m, lane);
    const BodyLane<MAXD> BL = load_body_lane<MAXD>(m, DL, lane);
    int* rowadr_l = (int*)(L + m.o_rowadr);
    if (lane < m.nv) rowadr_l[lane] = DL.rowadr;
    // ---- ingress
    for (int i = lane; i < nq; i += RB_WAVE) q[i] = A.qpos[(size_t)w * nq + i];
    for (int i = lane; i < nv; i += RB_WAVE) {
        v[i] = A.qvel[(size_t)w * nv + i];
        aws[i] = A.W.qacc_ws[(size_t)w * nv + i];
    }
    for (int i = lane; i < nu; i += RB_WAVE) ctrl[i] = A.ctrl[(size_t)w * nu + i];
    for (int b = lane; b < nb; b += RB_WAVE) msc[b] = m.ms_pw ? A.W.mass_scale[(size_t)w * nb + b] : 1.0f;
    const float mu_world = m.fr_pw ? A.W.friction[w] : 0.0f;
    if (lane == 0) {
        xpos[0] = xpos[1] = xpos[2] = 0.f;
        for (int c = 0; c < 10; c++) cinert[c] = 0.f;
        for (int c = 0; c < 6; c++) cvel[c] = 0.f;
    }
    uint32_t status = A.W.status[w];
    // per-substep record of the stats tap: substeps and updates never reached stay 0
    int32_t* SUBREC = (TIMED && A.want_taps && A.taps.stats) ? A.taps.stats + (size_t)w * RB_NSTATS + 4 + RB_NSTAGE
                                                               : nullptr;
    if (TIMED && SUBREC && lane < RB_STATS_SUB * RB_SUBSTAT) SUBREC[lane] = 0;
    wave_sync();

    Con C;
    int ncon = 0;
    // torsional / rolling pyramid rows of the lane's contact (condim 4: 2, condim 6: 6), kept in
    // LDS as generic rows after the equality rows at slot xbase; nx of them in the world
    int xr = 0, xbase = 0, nx = 0;
    int st_con = 0, st_rows = 0, st_iter = 0, st_seg = 0;   // work totals for the stats tap
    uint64_t stage_cyc[RB_NSTAGE] = {};                          // cycles per stage (stats tap)
    uint64_t t_mark = TIMED ? clock64() : 0;
#define RB_STAGE(id)                                    \
    do {                                                \
        if (TIMED) {                                    \
            uint64_t t_now = clock64();                 \
            stage_cyc[id] += t_now - t_mark;            \
            t_mark = t_now;                             \
        }                                               \
    } while (0)
    bool frozen = (status & RB_STATUS_NONFINITE) != 0;
    status &= ~(uint32_t)(RB_STATUS_ITERCAP | RB_STATUS_CONOVERFLOW);

    for (int sub = 0; sub < m.K && !frozen; sub++) {
        // the lane index, opaque at the top of each substep: per-lane addresses are recomputed
        // in the substep rather than hoisted out of the loop and spilled
        const int lane = (int)opaque((uint32_t)threadIdx.x & (RB_WAVE - 1));
        // ---- actuation: tau = kp (ctrl - q) - kd v  (position) or gear * ctrl (motor)
        for (int i = lane; i < nv; i += RB_WAVE) {
            float t = 0.f;
            for (int c = m.act_start[i]; c < m.act_start[i + 1]; c++) {
                int u = m.act_list[c];
                if (m.act_type[u] == RB_ACT_POSITION) {
                    // gains: the world's own where the fields are expanded per world
                    const float kp = A.W.act_kp ? A.W.act_kp[(size_t)w * nu + u] : m.act_kp[u];
                    const float kd = A.W.act_kd ? A.W.act_kd[(size_t)w * nu + u] : m.act_kd[u];
                    t += kp * (ctrl[u] - q[m.act_qadr[u]]) - kd * v[i];
                } else {
                    t += m.act_gear[u] * ctrl[u];
                }
            }
            // passive joint damping (its implicit integration follows the solve)
            if (EXT && m.ndamp > 0) t -= m.dof_damping[i] * v[i];
            tau[i] = t;
        }
        // ---- forward kinematics.  Each body's pose relative to its parent is computed for all
        // bodies at once: R_loc = R(quat_b * rot(axis, theta)) and t_loc = pos_b + R(quat_b) p -
        // R_loc p for a hinge anchored at p (the anchor stays put while the child turns about it);
        // free bodies take their pose from qpos.  Then levels compose x_b = x_p + R_p t_loc,
        // R_b = R_p R_loc from the root.
        float tl[3] = {0.f, 0.f, 0.f};
        float Rl[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        const BodyTab BK = body_tab(m, lane);
        // the world's rotation: its space held the Newton vectors of the previous substep
        if (lane == 0)
            for (int c = 0; c < 9; c++) xmat[c] = (c % 4 == 0) ? 1.f : 0.f;
        if (lane >= 1 && lane < nb) {
            const int b = lane;
            float ql[4], d0[3] = {0.f, 0.f, 0.f};
            if (BK.jtype == RB_JNT_FREE) {
                const int a = BK.qadr;
                tl[0] = q[a]; tl[1] = q[a + 1]; tl[2] = q[a + 2];
                float nrm = sqrtf(q[a + 3] * q[a + 3] + q[a + 4] * q[a + 4] + q[a + 5] * q[a + 5] + q[a + 6] * q[a + 6]);
                float inv = 1.0f / nrm;
                ql[0] = q[a + 3] * inv; ql[1] = q[a + 4] * inv; ql[2] = q[a + 5] * inv; ql[3] = q[a + 6] * inv;
            } else {
                const float* qb = m.body_quat + 4 * b;
                // position in the parent: the world's own where the field is expanded per world
                const float* pb = A.W.body_pos ? A.W.body_pos + ((size_t)w * nb + b) * 3 : m.body_pos + 3 * b;
                ql[0] = qb[0]; ql[1] = qb[1]; ql[2] = qb[2]; ql[3] = qb[3];
                tl[0] = pb[0]; tl[1] = pb[1]; tl[2] = pb[2];
                if (BK.jtype == RB_JNT_HINGE) {
                    const float* ax = m.body_jaxis + 3 * b;
                    const float* jp = m.body_jpos + 3 * b;
                    float th = 0.5f * q[BK.qadr];
                    float sh = sinf(th), ch = cosf(th);
                    float qh[4] = {ch, sh * ax[0], sh * ax[1], sh * ax[2]};
                    float R0[9], q1[4];
                    qmat(ql, R0);
                    mv(R0, jp, d0);
                    qmul(ql, qh, q1);
                    ql[0] = q1[0]; ql[1] = q1[1]; ql[2] = q1[2]; ql[3] = q1[3];
                }
            }
            qmat(ql, Rl);
            if (BK.jtype == RB_JNT_HINGE) {
                const float* jp = m.body_jpos + 3 * b;
                float d1[3];
                mv(Rl, jp, d1);
                tl[0] += d0[0] - d1[0]; tl[1] += d0[1] - d1[1]; tl[2] += d0[2] - d1[2];
            }
        }
        wave_sync();
        for (int lev = 1; lev <= m.nblevel; lev++) {
            if (BK.level == lev) {
                const int b = lane;
                const int par = BK.parent;
                if (BK.jtype == RB_JNT_FREE) {
                    xpos[3 * b] = tl[0]; xpos[3 * b + 1] = tl[1]; xpos[3 * b + 2] = tl[2];
#pragma unroll
                    for (int c = 0; c < 9; c++) xmat[9 * b + c] = Rl[c];
                } else {
                    float off[3];
                    mv(xmat + 9 * par, tl, off);
                    xpos[3 * b] = xpos[3 * par] + off[0];
                    xpos[3 * b + 1] = xpos[3 * par + 1] + off[1];
                    xpos[3 * b + 2] = xpos[3 * par + 2] + off[2];
                    mm(xmat + 9 * par, Rl, xmat + 9 * b);
                }
            }
            wave_sync();
        }
        RB_STAGE(0);
        const float O[3] = {xpos[3], xpos[4], xpos[5]};
        // ---- spatial inertias about O, motion subspaces of the dofs
        if (lane >= 1 && lane < nb) {
            const int b = lane;
            const float* R = xmat + 9 * b;
            float Ri[9], RR[9];
            qmat(m.body_iquat + 4 * b, Ri);
            mm(R, Ri, RR);
            float s = msc[b];
            float mass = s * m.body_mass[b];
            float d0 = s * m.body_inertia[3 * b], d1 = s * m.body_inertia[3 * b + 1], d2 = s * m.body_inertia[3 * b + 2];
            float off[3];
            mv(R, m.body_ipos + 3 * b, off);
            float c[3] = {xpos[3 * b] + off[0] - O[0], xpos[3 * b + 1] + off[1] - O[1], xpos[3 * b + 2] + off[2] - O[2]};
            // rotational inertia about the COM: RR diag(d) RR'
            float Ixx = RR[0] * RR[0] * d0 + RR[1] * RR[1] * d1 + RR[2] * RR[2] * d2;
            float Iyy = RR[3] * RR[3] * d0 + RR[4] * RR[4] * d1 + RR[5] * RR[5] * d2;
            float Izz = RR[6] * RR[6] * d0 + RR[7] * RR[7] * d1 + RR[8] * RR[8] * d2;
            float Ixy = RR[0] * RR[3] * d0 + RR[1] * RR[4] * d1 + RR[2] * RR[5] * d2;
            float Ixz = RR[0] * RR[6] * d0 + RR[1] * RR[7] * d1 + RR[2] * RR[8] * d2;
            float Iyz = RR[3] * RR[6] * d0 + RR[4] * RR[7] * d1 + RR[5] * RR[8] * d2;
            float cc = dot(c, c);
            float* I = cinert + 10 * b;
            I[0] = mass;
            I[1] = mass * c[0]; I[2] = mass * c[1]; I[3] = mass * c[2];
            I[4] = Ixx + mass * (cc - c[0] * c[0]);
            I[5] = Iyy + mass * (cc - c[1] * c[1]);
            I[6] = Izz + mass * (cc - c[2] * c[2]);
            I[7] = Ixy - mass * c[0] * c[1];
            I[8] = Ixz - mass * c[0] * c[2];
            I[9] = Iyz - mass * c[1] * c[2];
            for (int k = 0; k < 10; k++) crb[10 * b + k] = I[k];
            const BodyTab BI = body_tab(m, lane);
            const int jt = BI.jtype;
            const int da = BI.dadr;
            float xo[3] = {xpos[3 * b] - O[0], xpos[3 * b + 1] - O[1], xpos[3 * b + 2] - O[2]};
            if (jt == RB_JNT_HINGE) {
                float u[3], o[3];
                mv(R, m.body_jaxis + 3 * b, u);
                mv(R, m.body_jpos + 3 * b, o);
                o[0] += xo[0]; o[1] += xo[1]; o[2] += xo[2];
                float* S = cdof + 6 * da;
                S[0] = u[0]; S[1] = u[1]; S[2] = u[2];
                cross(o, u, S + 3);
            } else if (jt == RB_JNT_FREE) {
                for (int k = 0; k < 3; k++) {
                    float* S = cdof + 6 * (da + k);
                    S[0] = S[1] = S[2] = 0.f;
                    S[3] = k == 0; S[4] = k == 1; S[5] = k == 2;
                    float* Sr = cdof + 6 * (da + 3 + k);
                    float r[3] = {R[k], R[3 + k], R[6 + k]};
                    Sr[0] = r[0]; Sr[1] = r[1]; Sr[2] = r[2];
                    cross(xo, r, Sr + 3);
                }
            }
        }
        wave_sync();
        // ---- recursive Newton-Euler bias forces (qacc = 0, world accelerating at -gravity)
        if (lane == 0) {
            bvec[0] = bvec[1] = bvec[2] = 0.f;
            bvec[3] = -m.grav[0]; bvec[4] = -m.grav[1]; bvec[5] = -m.grav[2];
        }
        wave_sync();
        const BodyTab BR = body_tab(m, lane);
        for (int lev = 1; lev <= m.nblevel; lev++) {
            if (BR.level == lev) {
                const int b = lane;
                const int par = BR.parent;
                float vb[6], ab[6];
                for (int c = 0; c < 6; c++) { vb[c] = cvel[6 * par + c]; ab[c] = bvec[6 * par + c]; }
                const int jt = BR.jtype, da = BR.dadr;
                int nd = jt == RB_JNT_FREE ? 6 : (jt == RB_JNT_HINGE ? 1 : 0);
                for (int k = 0; k < nd; k++) {
                    const float* S = cdof + 6 * (da + k);
                    float qd = v[da + k];
                    for (int c = 0; c < 6; c++) vb[c] += S[c] * qd;
                }
                int k0 = jt == RB_JNT_FREE ? 3 : 0;   // free-joint translation axes are fixed in the world
                for (int k = k0; k < nd; k++) {
                    float t[6];
                    crm(vb, cdof + 6 * (da + k), t);
                    float qd = v[da + k];
                    for (int c = 0; c < 6; c++) ab[c] += t[c] * qd;
                }
                for (int c = 0; c < 6; c++) { cvel[6 * b + c] = vb[c]; bvec[6 * b + c] = ab[c]; }
            }
            wave_sync();
        }
        if (lane >= 1 && lane < nb) {
            const int b = lane;
            float f[6], Iv[6], t[6];
            inert_mul(cinert + 10 * b, bvec + 6 * b, f);
            inert_mul(cinert + 10 * b, cvel + 6 * b, Iv);
            crf(cvel + 6 * b, Iv, t);
            for (int c = 0; c < 6; c++) bvec2[6 * b + c] = f[c] + t[c];
        }
        wave_sync();
        // ---- backward passes: bias wrenches and composite inertias accumulate to the root
        const BodyTab BB2 = body_tab(m, lane);
        for (int lev = m.nblevel - 1; lev >= 1; lev--) {
            if (BB2.level == lev) {
                const int b = lane;
                // accumulate in registers: one read and one write of the body's own entries
                float fw[6], ci[10];
#pragma unroll
                for (int k = 0; k < 6; k++) fw[k] = bvec2[6 * b + k];
#pragma unroll
                for (int k = 0; k < 10; k++) ci[k] = crb[10 * b + k];
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    int ch = (BB2.children >> (8 * c)) & 0xff;
                    if (ch == 0xff) break;
#pragma unroll
                    for (int k = 0; k < 6; k++) fw[k] += bvec2[6 * ch + k];
#pragma unroll
                    for (int k = 0; k < 10; k++) ci[k] += crb[10 * ch + k];
                }
#pragma unroll
                for (int k = 0; k < 6; k++) bvec2[6 * b + k] = fw[k];
#pragma unroll
                for (int k = 0; k < 10; k++) crb[10 * b + k] = ci[k];
            }
            wave_sync();
        }
        if (lane < nv) bias[lane] = sdot(cdof + 6 * lane, bvec2 + 6 * m.dof_body[lane]);
        wave_sync();   // the body forces share space with M, whose rows are written next
        if (lane < nv) {
            const int i = lane;
            const float* S = cdof + 6 * i;
            const int b = m.dof_body[i];
            // joint-space inertia row i: M_ij = S_j . (Ic_b S_i) over the chain of i
            float F[6];
            inert_mul(crb + 10 * b, S, F);
            const int d = DL.depth, r = DL.rowadr;
#pragma unroll
            for (int t = 0; t < MAXD; t++)
                if (t < d) Mm[r + t] = sdot(cdof + 6 * DL.ancestor(t), F);
            Mm[r + d - 1] += m.dof_armature[i];
            a0[i] = tau[i] - bias[i];
        }
        wave_sync();
        RB_STAGE(1);
        {
            // factor M with a0 = M^-1 (tau - c) solved in the same sweep; keep the factor in H
            float Hr[MAXD];
#pragma unroll
            for (int t = 0; t < MAXD; t++) Hr[t] = t < DL.depth ? Mm[DL.rowadr + t] : 0.f;
            float invd;
            float x = factor_solve<MAXD>(m, DL, Hr, lane < nv ? a0[lane] : 0.f, lane, piv, &invd);
            if (lane < nv) {
                // packed factor for the contact rows: L (scaled) off the diagonal, D on it
                a0[lane] = x;
#pragma unroll
                for (int t = 0; t < MAXD; t++)
                    if (t < DL.depth - 1) H[DL.rowadr + t] = Hr[t] * invd;
                H[DL.rowadr + DL.depth - 1] = 1.0f / invd;
            }
            wave_sync();
        }
        RB_STAGE(2);

        // ---- collision: count per pair, scan, then each contact lane rebuilds its contact
        int cnt = 0, cnt2 = 0;
        uint32_t cmask = 0, cmask2 = 0;    // plane-like pairs: candidates below the margin
        float pos_[3];
        // geom sizes: the world's own where the field is expanded per world
        const float* gsize = A.W.geom_size ? A.W.geom_size + (size_t)w * 3 * m.ngeom : m.geom_size;
        auto pair_count = [&](int p, int& c, uint32_t& mk) {
            if (EXT && m.pair_type[p] == RB_PAIR_BOXBOX) {
                c = box_box(m, L, gsize, p, L + m.o_bb + RB_BB_FLOATS * m.pair_slot[p]);
            } else {
                mk = pair_mask<EXT>(m, L, gsize, p);
                c = __builtin_popcount(mk);
            }
        };
        if (lane < m.npair) pair_count(lane, cnt, cmask);
        // more pairs than lanes (extended code): a second round, pair lane + 64
        const bool two = EXT && m.npair > RB_WAVE;
        if (two && lane + RB_WAVE < m.npair) pair_count(lane + RB_WAVE, cnt2, cmask2);
        if (EXT) wave_sync();   // box-box blocks written by their pair lanes are read by contact lanes
        int incl = wscan_incl(cnt, lane);
        const int total1 = __shfl(incl, RB_WAVE - 1);
        int incl2 = 0, total = total1;
        if (two) {
            incl2 = wscan_incl(cnt2, lane);
            total += __shfl(incl2, RB_WAVE - 1);
        }
        ncon = total < m.ncap ? total : m.ncap;
        if (total > m.ncap) status |= RB_STATUS_CONOVERFLOW;
        ncon = __builtin_amdgcn_readfirstlane(ncon);
        bool has = lane < ncon;
        // this lane's contact comes from the first round's pairs, or the second's past total1
        const bool second = two && lane >= total1;
        const int key = second ? lane - total1 : lane;
        int src = 0;
        {
            // smallest pair whose inclusive count exceeds this lane's contact index
            int lo = 0, hi = RB_WAVE - 1;
#pragma unroll
            for (int it = 0; it < 6; it++) {
                int mid = (lo + hi) >> 1;
                int vmid = __shfl(incl, mid);
                if (two) {
                    const int v2 = __shfl(incl2, mid);
                    if (second) vmid = v2;
                }
                if (vmid > key) hi = mid; else lo = mid + 1;
            }
            src = lo;
        }
        int before = __shfl(incl - cnt, src);
        uint32_t smask = (uint32_t)__shfl((int)cmask, src);
        if (two) {
            const int before2 = __shfl(incl2 - cnt2, src) + total1;
            const uint32_t smask2 = (uint32_t)__shfl((int)cmask2, src);
            if (second) {
                before = before2;
                smask = smask2;
                src += RB_WAVE;
            }
        }
        float margin_c = 0.f;
        xr = 0;
        float mu_spin = 0.f, mu_roll = 0.f;
        int ellx = 0;   // an elliptic contact's rows beyond the three: 1 spin (condim 4), 3 spin and rolling (6)
        if (has) {
            int j = lane - before, feat;
            if (EXT && m.pair_type[src] == RB_PAIR_BOXBOX) {
                const float* S = L + m.o_bb + RB_BB_FLOATS * m.pair_slot[src];
                C.dist = S[48 + 5 * j];
                pos_[0] = S[49 + 5 * j]; pos_[1] = S[50 + 5 * j]; pos_[2] = S[51 + 5 * j];
                feat = (int)S[52 + 5 * j];
                C.n[0] = S[88]; C.n[1] = S[89]; C.n[2] = S[90];
            } else {
                // the j-th set bit of the pair's candidate mask
                for (int t = 0; t < j; t++) smask &= smask - 1u;
                feat = __builtin_ctz(smask);
                pair_candidate<EXT>(m, L, gsize, src, feat, &C.dist, pos_, C.n);
            }
            C.r[0] = pos_[0] - O[0]; C.r[1] = pos_[1] - O[1]; C.r[2] = pos_[2] - O[2];
            contact_frame(C.n, C.t1);
            C.ids = m.pair_g1[src] | (m.pair_g2[src] << 8) | (feat << 16);
            C.body = m.pair_body[src];
            C.body1 = (EXT == 3 && m.nmm > 0) ? m.pair_body1[src] : 0;
            C.sigma = m.pair_sigma[src];
            C.mu = m.fr_pw ? mu_world : m.pair_mu[src];
            if (EXT && m.pair_frictionless[src]) {
                // frictionless pair: mu = 0 makes the four rows the normal row; only the first
                // is kept (the others get D = 0 below)
                C.mu = 0.f;
                C.ids |= 1 << 24;
            }
            margin_c = m.pair_margin[src];
            if (EXT >= 2 && (m.nxmax > 0 || m.cone)) {
                xr = m.pair_xrows[src];
                mu_spin = m.pair_mu_spin[src];
                mu_roll = m.pair_mu_roll[src];
                ellx = m.pair_ellrows[src];
            }
        } else {
            C.body = 0;
            C.body1 = 0;
        }
        // an elliptic-cone contact (extended code): frame rows costed by the soft elliptic cone;
        // frictionless contacts keep their one normal row
        const bool cell = EXT >= 2 && m.cone && has && !(C.ids >> 24);
        const bool cspin = cell && ellx >= 1, croll = EXT == 4 && cell && ellx == 3;
        const int cellm = cell ? (croll ? 3 : (cspin ? 2 : 1)) : 0;   // rows_of's elliptic frame rows
        const int celld = croll ? 6 : (cspin ? 4 : 3);                 // and their number
        RB_STAGE(3);
        // generic-row slots of the contacts' extra rows: after the equality rows, in contact order
        float* GR = L + m.o_gr;
        xbase = 0;
        nx = 0;
        if (EXT >= 2 && m.nxmax > 0) {
            const int xi = wscan_incl(xr, lane);
            xbase = m.neqrow + xi - xr;
            nx = __builtin_amdgcn_readfirstlane(__shfl(xi, RB_WAVE - 1));
        }
        // ---- constraint rows: exact A-hat from the chain half-solve with M's factor
        {
            // the contact body's chain, from the body lane
            const int d = __shfl(BL.depth, C.body);
            const int csrc = __shfl(BL.src, C.body);
            uint32_t cw[MAXD / 4];
#pragma unroll
            for (int w2 = 0; w2 < MAXD / 4; w2++) cw[w2] = (uint32_t)__shfl((int)DL.anc[w2], csrc);
#define CROW(t) rowadr_l[(int)((cw[(t) >> 2] >> (8 * ((t) & 3))) & 0xffu)]
            // the second moving body's chain (contacts between two moving bodies)
            int d1 = 0;
            uint32_t cw1[MAXD / 4];
#pragma unroll
            for (int w2 = 0; w2 < MAXD / 4; w2++) cw1[w2] = 0u;
            if (EXT == 3 && m.nmm > 0) {
                d1 = __shfl(BL.depth, C.body1);
                const int csrc1 = __shfl(BL.src, C.body1);
#pragma unroll
                for (int w2 = 0; w2 < MAXD / 4; w2++) cw1[w2] = (uint32_t)__shfl((int)DL.anc[w2], csrc1);
            }
        if (has) {
            // A_c = J_c M^-1 J_c' from Y = L'^-1 J_c' on the body's chain (positions t < d): one
            // column (normal, t1, t2) at a time, keeping only the normal column (fewer values live
            // than solving the three together)
            float t2c[3];
            cross(C.n, C.t1, t2c);
            auto half_solve = [&](const float* dir, float (&Y)[MAXD]) {
#pragma unroll
                for (int t = 0; t < MAXD; t++) {
                    // past the chain the byte is 0, a valid dof: computed and discarded
                    const float* S = cdof + 6 * (int)((cw[t >> 2] >> (8 * (t & 3))) & 0xffu);
                    float wr[3];
                    cross(S, C.r, wr);
                    const float vp[3] = {S[3] + wr[0], S[4] + wr[1], S[5] + wr[2]};
                    Y[t] = t < d ? C.sigma * dot(dir, vp) : 0.f;
                }
#pragma unroll
                for (int tp = MAXD - 1; tp >= 1; tp--) {
                    if (tp < d) {
                        const int row = CROW(tp);
#pragma unroll
                        for (int t = 0; t < tp; t++) Y[t] -= H[row + t] * Y[tp];
                    }
                }
            };
            float Z0[MAXD];
            float A00 = 0, A11 = 0, A22 = 0, A01 = 0, A02 = 0;
            {
                float Y[MAXD];
                half_solve(C.n, Y);
#pragma unroll
                for (int t = 0; t < MAXD; t++) {
                    Z0[t] = 0.f;
                    if (t < d) {
                        Z0[t] = Y[t] * __builtin_amdgcn_rcpf(H[CROW(t) + t]);
                        A00 += Y[t] * Z0[t];
                    }
                }
            }
            {
                float Y[MAXD];
                half_solve(C.t1, Y);
#pragma unroll
                for (int t = 0; t < MAXD; t++)
                    if (t < d) {
                        A11 += Y[t] * Y[t] * __builtin_amdgcn_rcpf(H[CROW(t) + t]);
                        A01 += Z0[t] * Y[t];
                    }
            }
            {
                float Y[MAXD];
                half_solve(t2c, Y);
#pragma unroll
                for (int t = 0; t < MAXD; t++)
                    if (t < d) {
                        A22 += Y[t] * Y[t] * __builtin_amdgcn_rcpf(H[CROW(t) + t]);
                        A02 += Z0[t] * Y[t];
                    }
            }
            if (EXT == 3 && C.body1 > 0) {
                // both bodies move: J = J(b2) - J(b1), and Y = L'^-1 J' is the sum of the half-solves
                // along each chain (+dir on b2's, -dir on b1's), the two adding on their common
                // prefix; A-hat sums Y^2 / D over the union of the two chains
                auto byte_of = [](const uint32_t* cwx, int t) { return (int)((cwx[t >> 2] >> (8 * (t & 3))) & 0xffu); };
                int cpl = 0;
#pragma unroll
                for (int t = 0; t < MAXD; t++)
                    if (t == cpl && t < d && t < d1 && byte_of(cw, t) == byte_of(cw1, t)) cpl = t + 1;
                auto solve_on = [&](const uint32_t* cwx, int dx, const float* dir, float sg, float (&Y)[MAXD]) {
#pragma unroll
                    for (int t = 0; t < MAXD; t++) {
                        const float* S = cdof + 6 * byte_of(cwx, t);
                        float wr[3];
                        cross(S, C.r, wr);
                        const float vp[3] = {S[3] + wr[0], S[4] + wr[1], S[5] + wr[2]};
                        Y[t] = t < dx ? sg * dot(dir, vp) : 0.f;
                    }
#pragma unroll
                    for (int tp = MAXD - 1; tp >= 1; tp--) {
                        if (tp < dx) {
                            const int row = rowadr_l[byte_of(cwx, tp)];
#pragma unroll
                            for (int t = 0; t < tp; t++) Y[t] -= H[row + t] * Y[tp];
                        }
                    }
                };
                // a direction's column on the union: U2 over b2's chain (the common prefix
                // summed), U1 over b1's positions past the prefix
                auto column = [&](const float* dir, float (&U2)[MAXD], float (&U1)[MAXD]) {
                    float Y1[MAXD];
                    solve_on(cw, d, dir, 1.f, U2);
                    solve_on(cw1, d1, dir, -1.f, Y1);
#pragma unroll
                    for (int t = 0; t < MAXD; t++) {
                        if (t < cpl) U2[t] += Y1[t];
                        U1[t] = (t >= cpl && t < d1) ? Y1[t] : 0.f;
                    }
                };
                auto dinv2 = [&](int t) { return __builtin_amdgcn_rcpf(H[rowadr_l[byte_of(cw, t)] + t]); };
                auto dinv1 = [&](int t) { return __builtin_amdgcn_rcpf(H[rowadr_l[byte_of(cw1, t)] + t]); };
                float Zn2[MAXD], Zn1[MAXD];
                A00 = A11 = A22 = A01 = A02 = 0.f;
                {
                    float U2[MAXD], U1[MAXD];
                    column(C.n, U2, U1);
#pragma unroll
                    for (int t = 0; t < MAXD; t++) {
                        Zn2[t] = t < d ? U2[t] * dinv2(t) : 0.f;
                        Zn1[t] = (t >= cpl && t < d1) ? U1[t] * dinv1(t) : 0.f;
                        A00 += U2[t] * Zn2[t] + U1[t] * Zn1[t];
                    }
                }
                for (int k = 0; k < 2; k++) {
                    float U2[MAXD], U1[MAXD];
                    column(k == 0 ? C.t1 : t2c, U2, U1);
                    float Akk = 0.f, A0k = 0.f;
#pragma unroll
                    for (int t = 0; t < MAXD; t++) {
                        const float z2 = t < d ? U2[t] * dinv2(t) : 0.f;
                        const float z1 = (t >= cpl && t < d1) ? U1[t] * dinv1(t) : 0.f;
                        Akk += U2[t] * z2 + U1[t] * z1;
                        A0k += Zn2[t] * U2[t] + Zn1[t] * U1[t];
                    }
                    if (k == 0) { A11 = Akk; A01 = A0k; } else { A22 = Akk; A02 = A0k; }
                }
            }
            float vrow[6] = {0, 0, 0, 0, 0, 0};
            rows_of(C, cvel, vrow, cellm, EXT == 3 ? C.body1 : 0);
            float rd = C.dist - margin_c;
            float imp = impedance(m, rd);
            float mu = C.mu, mu2 = mu * mu;
            float ah[4] = {A00 + mu2 * A11 + 2.f * mu * A01, A00 + mu2 * A11 - 2.f * mu * A01,
                           A00 + mu2 * A22 + 2.f * mu * A02, A00 + mu2 * A22 - 2.f * mu * A02};
#pragma unroll
            for (int e = 0; e < 4; e++) {
                C.aref[e] = -m.bref * vrow[e] - m.kref * imp * rd;
                float R = fmaxf(1e-15f, (1.0f - imp) / imp * ah[e]);
                C.D[e] = 1.0f / R;
            }
            if (EXT && (C.ids >> 24)) C.D[1] = C.D[2] = C.D[3] = 0.f;
            if (cell) {
                // elliptic cone: the frame rows, the distance reference on the normal only, the
                // tangential regulariser the normal's divided by impratio
                const float D0 = 1.0f / fmaxf(1e-15f, (1.0f - imp) / imp * A00);
                C.aref[0] = -m.bref * vrow[0] - m.kref * imp * rd;
                C.aref[1] = -m.bref * vrow[1];
                C.aref[2] = -m.bref * vrow[2];
                C.aref[3] = -m.bref * vrow[3];
                if (EXT == 4) {
                    C.aref[4] = -m.bref * vrow[4];
                    C.aref[5] = -m.bref * vrow[5];
                }
                C.D[0] = D0;
                C.D[1] = C.D[2] = m.impratio * D0;
                // the spin row (condim 4, 6) and the rolling rows (6): regulariser the normal's
                // times mu^2 / (mu_d^2 impratio), which keeps the cone circular in the D-scaled rows
                const float rs = (cspin && C.mu > 0.f) ? mu_spin / C.mu : 0.f;
                const float rr = (croll && C.mu > 0.f) ? mu_roll / C.mu : 0.f;
                C.D[3] = m.impratio * D0 * rs * rs;
                if (EXT == 4) C.D[4] = C.D[5] = m.impratio * D0 * rr * rr;
                ah[0] = A00; ah[1] = A11; ah[2] = A22; ah[3] = 0.f;
            } else if (EXT == 4) {
                C.aref[4] = C.aref[5] = 0.f;
                C.D[4] = C.D[5] = 0.f;
            }
            if (TIMED && A.want_taps && sub == 0 && A.taps.efc) {
                float* E = A.taps.efc + ((size_t)w * m.ncap + lane) * 12;
                for (int e = 0; e < 4; e++) {
                    E[3 * e] = C.aref[e];
                    E[3 * e + 1] = C.D[e];
                    E[3 * e + 2] = ah[e];
                }
            }
            if (EXT >= 2 && xr > 0) {
                // torsional (about n) and rolling (about t1, t2) pyramid rows J_n +- mu_d J_d,
                // J_d the frame component of the body's angular velocity: as spatial forces at O,
                // psi = sigma (r x n +- mu_d k_d, n); A-hat from one more half-solve per axis
                // (Y = L'^-1 J_d' for the pure torque k_d) and the normal column's Z0
                float rxn[3];
                cross(C.r, C.n, rxn);
                const float vn = 0.5f * (vrow[0] + vrow[1]);
                const float* wb = cvel + 6 * C.body;
                for (int dir = 0; 2 * dir < xr; dir++) {
                    const float* k = dir == 0 ? C.n : (dir == 1 ? C.t1 : t2c);
                    float Y[MAXD];
#pragma unroll
                    for (int t = 0; t < MAXD; t++) {
                        const float* S = cdof + 6 * (int)((cw[t >> 2] >> (8 * (t & 3))) & 0xffu);
                        Y[t] = t < d ? C.sigma * dot(k, S) : 0.f;
                    }
#pragma unroll
                    for (int tp = MAXD - 1; tp >= 1; tp--) {
                        if (tp < d) {
                            const int row = CROW(tp);
#pragma unroll
                            for (int t = 0; t < tp; t++) Y[t] -= H[row + t] * Y[tp];
                        }
                    }
                    float Akk = 0.f, Ank = 0.f;
#pragma unroll
                    for (int t = 0; t < MAXD; t++)
                        if (t < d) {
                            Akk += Y[t] * Y[t] * __builtin_amdgcn_rcpf(H[CROW(t) + t]);
                            Ank += Z0[t] * Y[t];
                        }
                    const float mud = dir == 0 ? mu_spin : mu_roll;
                    const float wk = C.sigma * dot(k, wb);
                    for (int sg = 0; sg < 2; sg++) {
                        const float sm = sg ? -mud : mud;
                        const float ahx = A00 + mud * mud * Akk + 2.f * sm * Ank;
                        float* G = GR + RB_GRF * (xbase + 2 * dir + sg);
                        G[0] = C.sigma * (rxn[0] + sm * k[0]);
                        G[1] = C.sigma * (rxn[1] + sm * k[1]);
                        G[2] = C.sigma * (rxn[2] + sm * k[2]);
                        G[3] = C.sigma * C.n[0];
                        G[4] = C.sigma * C.n[1];
                        G[5] = C.sigma * C.n[2];
                        G[6] = 1.0f / fmaxf(1e-15f, (1.0f - imp) / imp * ahx);
                        G[7] = -m.bref * (vn + sm * wk) - m.kref * imp * rd;
                        G[8] = 0.f;
                        G[9] = __int_as_float(C.body);
                        G[10] = __int_as_float(1024 + 6 * lane + 2 * dir + sg);
                    }
                }
            }
        }
        }

        // ---- equality constraints with the world (extended code): lane r < neqrow builds row r.
        // A row is a spatial force direction psi at O on its body's chain: translational row k of
        // a connect or weld is the unit axis e_k applied at the anchor's world point c,
        // psi = (r x e_k, e_k) with r = c - O, against the offset c_k - target_k; rotational row
        // k is e_k as a pure torque, psi = (e_k, 0), against component k of the rotation vector of
        // E = R_body R_target'.  LDS keeps psi, D, the residual J a - aref (aref until the Newton
        // start), the line-search direction J p and the body.  Bilateral: always active.
        const int ngr = m.neqrow + nx;            // generic rows: equality, then contact extras
        const bool gract = EXT >= 2 && ngr > 0;
        if (EXT >= 2 && m.neqrow > 0) {
            const bool own = lane < m.neqrow;
            const int qe = own ? m.eqrow_eq[lane] : 0;
            const int k = own ? m.eqrow_k[lane] : 0;
            const int body = own ? m.eq_body[qe] : 0;
            float psi[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float rdist = 0.f;
            if (own) {
                const float* Rb = xmat + 9 * body;
                float c[3];
                mv(Rb, m.eq_anchor + 3 * qe, c);
                for (int i = 0; i < 3; i++) c[i] += xpos[3 * body + i];
                if (k < 3) {
                    const float r[3] = {c[0] - O[0], c[1] - O[1], c[2] - O[2]};
                    const float e[3] = {k == 0 ? 1.f : 0.f, k == 1 ? 1.f : 0.f, k == 2 ? 1.f : 0.f};
                    cross(r, e, psi);
                    psi[3 + k] = 1.f;
                    rdist = c[k] - m.eq_tpos[3 * qe + k];
                } else {
                    // E = R_b R_t'; rotation vector = angle * axis from the skew part
                    // E - E' = 2 sin(angle) [axis]x and the trace, the angle by atan2 (well
                    // conditioned at small angles, where acos of the trace is not in FP32)
                    const float* Rt = m.eq_tmat + 9 * qe;
                    float E[9];
                    for (int i = 0; i < 3; i++)
                        for (int j = 0; j < 3; j++)
                            E[3 * i + j] = Rb[3 * i] * Rt[3 * j] + Rb[3 * i + 1] * Rt[3 * j + 1] + Rb[3 * i + 2] * Rt[3 * j + 2];
                    const float wv[3] = {E[7] - E[5], E[2] - E[6], E[3] - E[1]};
                    const float s2 = sqrtf(dot(wv, wv));          // 2 sin(angle)
                    const float ang = atan2f(0.5f * s2, 0.5f * (E[0] + E[4] + E[8] - 1.f));
                    const float f = s2 > 1e-4f ? ang / s2 : 0.5f + ang * ang * (1.f / 12.f);
                    psi[k - 3] = 1.f;
                    rdist = f * pick3(wv, k - 3);
                }
            }
            // A-hat = J M^-1 J' from Y = L'^-1 J' on the body's chain, as for a contact row
            const int d = __shfl(BL.depth, body);
            const int csrc = __shfl(BL.src, body);
            uint32_t cw[MAXD / 4];
#pragma unroll
            for (int w2 = 0; w2 < MAXD / 4; w2++) cw[w2] = (uint32_t)__shfl((int)DL.anc[w2], csrc);
            auto eq_anc = [&](int t) { return (int)((cw[t >> 2] >> (8 * (t & 3))) & 0xffu); };
            if (own) {
                float Y[MAXD];
#pragma unroll
                for (int t = 0; t < MAXD; t++) Y[t] = t < d ? sdot(cdof + 6 * eq_anc(t), psi) : 0.f;
#pragma unroll
                for (int tp = MAXD - 1; tp >= 1; tp--) {
                    if (tp < d) {
                        const int row = rowadr_l[eq_anc(tp)];
#pragma unroll
                        for (int t = 0; t < tp; t++) Y[t] -= H[row + t] * Y[tp];
                    }
                }
                float Ah = 0.f;
#pragma unroll
                for (int t = 0; t < MAXD; t++)
                    if (t < d) Ah += Y[t] * Y[t] * __builtin_amdgcn_rcpf(H[rowadr_l[eq_anc(t)] + t]);
                const float jvel = sdot(cvel + 6 * body, psi);
                const float imp = impedance(m, rdist);
                float* Er = GR + RB_GRF * lane;
                for (int c6 = 0; c6 < 6; c6++) Er[c6] = psi[c6];
                Er[6] = 1.0f / fmaxf(1e-15f, (1.0f - imp) / imp * Ah);
                Er[7] = -m.bref * jvel - m.kref * imp * rdist;
                Er[8] = 0.f;
                Er[9] = __int_as_float(body);
                Er[10] = __int_as_float(512 + 6 * qe + k);
            }
        }
        if (gract) wave_sync();   // rows read by every lane; xmat's space is reused next

        // ---- joint limits: a hinge outside its range gets one row J = s e_i (s = +1 below the
        // lower bound, -1 above the upper one), held in LDS by the dof's lane: lD = s D (0 when
        // the hinge is inside its range) and ljar, the residual J a - aref (-aref until the
        // Newton start).  Only the owning lane ever reads them.
        float* lD = L + m.o_lD;
        float* ljar = L + m.o_ljar;
        bool limact = false;
        if (EXT && m.nlim > 0) {
            const int lq = lane < nv ? m.dof_limq[lane] : -1;
            float dist = 0.f, sgn = 0.f;
            if (lq >= 0) {
                const float qa = q[lq];
                const float dlo = qa - m.dof_limlo[lane], dhi = m.dof_limhi[lane] - qa;
                if (dlo < 0.f) { dist = dlo; sgn = 1.f; }
                else if (dhi < 0.f) { dist = dhi; sgn = -1.f; }
            }
            limact = __ballot(sgn != 0.f) != 0ull;
            if (limact && lane < nv) {
                float Ds = 0.f, nar = 0.f;
                if (sgn != 0.f) {
                    // A-hat = (M^-1)_ii = sum_t y_t^2 / D_t with y = L'^-1 e_i on the lane's chain
                    const int d = DL.depth;
                    float Y[MAXD];
#pragma unroll
                    for (int t = 0; t < MAXD; t++) Y[t] = t == d - 1 ? 1.f : 0.f;
#pragma unroll
                    for (int tp = MAXD - 1; tp >= 1; tp--) {
                        if (tp < d) {
                            const int row = rowadr_l[DL.ancestor(tp)];
#pragma unroll
                            for (int t = 0; t < tp; t++) Y[t] -= H[row + t] * Y[tp];
                        }
                    }
                    float Ah = 0.f;
#pragma unroll
                    for (int t = 0; t < MAXD; t++)
                        if (t < d) Ah += Y[t] * Y[t] * __builtin_amdgcn_rcpf(H[rowadr_l[DL.ancestor(t)] + t]);
                    const float imp = impedance(m, dist);
                    nar = m.bref * sgn * v[lane] + m.kref * imp * dist;
                    Ds = sgn / fmaxf(1e-15f, (1.0f - imp) / imp * Ah);
                }
                lD[lane] = Ds;
                ljar[lane] = nar;
            }
        }

        RB_STAGE(4);
        // ---- primal Newton solve
        bool itercap = false;
        if (ncon == 0 && !limact && !gract) {
            for (int i = lane; i < nv; i += RB_WAVE) acc[i] = a0[i];
            wave_sync();
        } else {
            // cost at a0 and at the warm start; keep the better (ties go to a0)
            body_motion(m, BL, DL, cdof, a0, bvec, lane);
            constexpr int NR = EXT == 4 ? 6 : 4;   // rows per contact lane in this instantiation
            float j0[6] = {0, 0, 0, 0, 0, 0};
            float f0 = 0.f;
            // the lane's contact cost at residuals j: pyramid rows, or the elliptic cone
            auto con_cost = [&](const float* j) {
                if (cell) {
                    float cst, ge[6];
                    EllCone E;
                    ell_eval<NE>(j, C.D[0], C.D[1], C.D[3], NE > 4 ? C.D[4] : 0.f, C.mu * m.rsqrt_impratio, &cst, ge, &E);
                    return cst;
                }
                float cst = 0.f;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float mn = fminf(j[e], 0.f);
                    cst += 0.5f * C.D[e] * mn * mn;
                }
                return cst;
            };
            if (has) {
                rows_of(C, bvec, j0, cellm, EXT == 3 ? C.body1 : 0);
#pragma unroll
                for (int e = 0; e < NR; e++) j0[e] -= C.aref[e];
                f0 += con_cost(j0);
            }
            // limit rows at a0 and at the warm start (their residuals are linear in a too);
            // recomputed from LDS where needed rather than held across the tree passes
            auto lim_res = [&](bool at_ws) {
                const float Ds = lD[lane], sl = Ds > 0.f ? 1.f : (Ds < 0.f ? -1.f : 0.f);
                const float j0l = sl * a0[lane] + ljar[lane];
                return at_ws ? j0l + sl * (aws[lane] - a0[lane]) : j0l;
            };
            if (limact && lane < nv) {
                const float mn = fminf(lim_res(false), 0.f);
                f0 += 0.5f * fabsf(lD[lane]) * mn * mn;
            }
            // generic rows at a0: lane r holds row r; equality rows are bilateral (the whole
            // residual counts), the contacts' extra rows unilateral
            const bool grown = gract && lane < ngr;
            const bool grbil = lane < m.neqrow;
            float* Er = GR + RB_GRF * (grown ? lane : 0);
            auto gr_cost = [&](float j) { const float mn = grbil ? j : fminf(j, 0.f); return 0.5f * Er[6] * mn * mn; };
            float ej0 = 0.f;
            if (grown) {
                ej0 = sdot(bvec + 6 * __float_as_int(Er[9]), Er) - Er[7];
                f0 += gr_cost(ej0);
            }
            f0 = wsum(f0);
            for (int i = lane; i < nv; i += RB_WAVE) tmp[i] = aws[i] - a0[i];
            wave_sync();
            // g <- M (aws - a0); bvec keeps the body motions of (aws - a0), and the rows are
            // linear in the motion, so the residuals at aws are those at a0 plus these
            spatial_mul(m, BL, DL, cdof, cinert, tmp, bvec, cvel, g, lane);
            float jw[6] = {0, 0, 0, 0, 0, 0};
            float fw = 0.f;
            if (has) {
                rows_of(C, bvec, jw, cellm, EXT == 3 ? C.body1 : 0);
#pragma unroll
                for (int e = 0; e < NR; e++) jw[e] += j0[e];
                fw += con_cost(jw);
            }
            float qf = 0.f;
            for (int i = lane; i < nv; i += RB_WAVE) qf += tmp[i] * g[i];
            if (limact && lane < nv) {
                const float mn = fminf(lim_res(true), 0.f);
                fw += 0.5f * fabsf(lD[lane]) * mn * mn;
            }
            float ejw = 0.f;
            if (grown) {
                ejw = ej0 + sdot(bvec + 6 * __float_as_int(Er[9]), Er);
                fw += gr_cost(ejw);
            }
            fw = wsum(fw) + 0.5f * wsum(qf);
            bool use_ws = fw < f0;
            if (limact && lane < nv) ljar[lane] = lim_res(use_ws);
            if (grown) Er[7] = use_ws ? ejw : ej0;
            float fcur = use_ws ? fw : f0;
            for (int i = lane; i < nv; i += RB_WAVE) {
                acc[i] = use_ws ? aws[i] : a0[i];
                Ma[i] = use_ws ? (tau[i] - bias[i]) + g[i] : (tau[i] - bias[i]);
            }
#pragma unroll
            for (int e = 0; e < NR; e++) C.jar[e] = use_ws ? jw[e] : j0[e];
            wave_sync();
            RB_STAGE(5);

            int it = 0;
            int seg_sub = 0;   // line-search segments of this substep (stats tap)
            uint32_t prev_bits = 0;
            for (; it < m.maxiter; it++) {
                // Converged when no row changed sides since the Hessian was last built: the
                // step then stayed inside one quadratic piece of the cost, and the exact line
                // search along the Newton direction of that piece lands on its minimiser, where
                // the gradient vanishes (in exact arithmetic; the FP32 gradient does not reach
                // the tolerance, so this is the test that ends the iteration).
                uint32_t bits = 0;
                bool mid = false;   // an elliptic contact on its cone's surface: cost not quadratic
                if (cell) {
                    float cst, ge[6];
                    EllCone E;
                    const int zone = ell_eval<NE>(C.jar, C.D[0], C.D[1], C.D[3], NE > 4 ? C.D[4] : 0.f, C.mu * m.rsqrt_impratio, &cst, ge, &E);
                    bits = (uint32_t)zone;
                    mid = zone == 1;
                } else if (has) {
#pragma unroll
                    for (int e = 0; e < 4; e++) bits |= (C.jar[e] < 0.f ? 1u : 0u) << e;
                }
                if (limact && lane < nv) bits |= (ljar[lane] < 0.f ? 1u : 0u) << 4;
                if (grown && !grbil) bits |= (Er[7] < 0.f ? 1u : 0u) << 5;
                // (with a contact on its cone's surface the cost is not piecewise quadratic, and
                // an unchanged active set does not mean the minimum was reached)
                if (it > 0 && __ballot(bits != prev_bits) == 0 && __ballot(mid) == 0) break;
                prev_bits = bits;
                // gradient and the contact part of the Hessian, one contact at a time
                float gc = 0.f;
                float F[6] = {0, 0, 0, 0, 0, 0};
                float S[6] = {0, 0, 0, 0, 0, 0};
                bool dof_lane = lane < nv;
                if (dof_lane)
                    for (int c = 0; c < 6; c++) S[c] = cdof[6 * lane + c];
                for (int c = 0; c < ncon; c++) {
                    const int body = __builtin_amdgcn_readlane(C.body, c);
                    const uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)BL.chainmask, body);
                    const uint32_t mhi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(BL.chainmask >> 32), body);
                    const uint64_t mask = ((uint64_t)mhi << 32) | mlo;
                    float r[3], n[3], t1[3], t2[3], D[6], jar[6];
                    for (int k = 0; k < 3; k++) {
                        r[k] = rl(C.r[k], c); n[k] = rl(C.n[k], c);
                        t1[k] = rl(C.t1[k], c);
                    }
                    cross(n, t1, t2);
                    for (int e = 0; e < 4; e++) { D[e] = rl(C.D[e], c); jar[e] = rl(C.jar[e], c); }
                    D[4] = D[5] = jar[4] = jar[5] = 0.f;
                    if (EXT == 4) {
                        // an elliptic contact's rolling rows
                        D[4] = D[5] = rl(C.D[4], c);
                        jar[4] = rl(C.jar[4], c); jar[5] = rl(C.jar[5], c);
                    }
                    float mu = rl(C.mu, c), sg = rl(C.sigma, c);
                    // an elliptic contact: its cost's gradient and Hessian in its frame rows
                    const bool ellc = EXT >= 2 && m.cone && !(__builtin_amdgcn_readlane(C.ids, c) >> 24);
                    float ge[6];
                    EllCone E;
                    if (ellc) {
                        float cst;
                        ell_eval<NE>(jar, D[0], D[1], D[3], NE > 4 ? D[4] : 0.f, mu * m.rsqrt_impratio, &cst, ge, &E);
                    }
                    if (ellc && dof_lane && ((mask >> lane) & 1ull)) {
                        float wr[3];
                        cross(S, r, wr);
                        const float vp[3] = {S[3] + wr[0], S[4] + wr[1], S[5] + wr[2]};
                        // the rows' Jacobian entries: sliding from the point's velocity, spin and
                        // rolling from the angular one (rows a contact lacks have D = 0)
                        const float je[6] = {sg * dot(n, vp), sg * dot(t1, vp), sg * dot(t2, vp),
                                             sg * dot(n, S), sg * dot(t1, S), sg * dot(t2, S)};
                        float u[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
                        for (int a = 0; a < NE; a++) gc += ge[a] * je[a];
                        ell_hv<NE>(E, je, u);
                        // Hessian term: the rows' directions weighted by h je, as a spatial force
                        // (the spin and rolling rows' directions are the pure torques n, t1, t2)
                        float a[3], ra[3], tq[3];
                        for (int k = 0; k < 3; k++) {
                            a[k] = sg * (u[0] * n[k] + u[1] * t1[k] + u[2] * t2[k]);
                            tq[k] = sg * (u[3] * n[k] + u[4] * t1[k] + u[5] * t2[k]);
                        }
                        cross(r, a, ra);
                        F[0] += ra[0] + tq[0]; F[1] += ra[1] + tq[1]; F[2] += ra[2] + tq[2];
                        F[3] += a[0]; F[4] += a[1]; F[5] += a[2];
                    }
                    // a contact between two moving bodies (level-3 code): a dof on b2's chain
                    // only takes the rows with +, on b1's only with -, on both (the common
                    // ancestors) not at all; its Hessian terms go to the dense Hessian instead
                    int b1c = 0;
                    uint64_t mask1 = 0ull;
                    if (EXT == 3 && m.nmm > 0) {
                        b1c = __builtin_amdgcn_readlane(C.body1, c);
                        if (b1c > 0) {
                            const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)BL.chainmask, b1c);
                            const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(BL.chainmask >> 32), b1c);
                            mask1 = ((uint64_t)khi << 32) | klo;
                        }
                    }
                    const float cf = EXT == 3 ? (float)((mask >> lane) & 1ull) - (float)((mask1 >> lane) & 1ull) : 1.f;
                    const bool onrow = EXT == 3 ? cf != 0.f : (bool)((mask >> lane) & 1ull);
                    if (!ellc && dof_lane && onrow) {
                        float wr[3];
                        cross(S, r, wr);
                        float vp[3] = {S[3] + wr[0], S[4] + wr[1], S[5] + wr[2]};
                        if (EXT == 3) sg *= cf;
                        float jn = sg * dot(n, vp), j1 = sg * dot(t1, vp), j2 = sg * dot(t2, vp);
                        float je[4] = {jn + mu * j1, jn - mu * j1, jn + mu * j2, jn - mu * j2};
                        // active row e's direction is n +- mu t_k; their weighted sum is kept as
                        // the coefficients of n, t1 and t2 and turned into one spatial force at O,
                        // sg (r x a, a), after the rows
                        float wn = 0.f, w1 = 0.f, w2 = 0.f;
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            if (EXT == 3 && b1c > 0) {
                                if (jar[e] < 0.f) gc += D[e] * jar[e] * je[e];
                                continue;
                            }
                            if (jar[e] < 0.f) {
                                gc += D[e] * jar[e] * je[e];
                                const float wgt = D[e] * je[e] * sg;
                                const float mw = (e & 1) ? -mu * wgt : mu * wgt;
                                wn += wgt;
                                if (e < 2) w1 += mw; else w2 += mw;
                            }
                        }
                        if (!(EXT == 3 && b1c > 0)) {
                            float a[3], ra[3];
                            for (int k = 0; k < 3; k++) a[k] = wn * n[k] + w1 * t1[k] + w2 * t2[k];
                            cross(r, a, ra);
                            F[0] += ra[0]; F[1] += ra[1]; F[2] += ra[2];
                            F[3] += a[0]; F[4] += a[1]; F[5] += a[2];
                        }
                    }
                }
                // generic rows: psi, D and the residual from LDS; equality rows always active
                if (gract) {
                    for (int rr = 0; rr < ngr; rr++) {
                        const float* Eo = GR + RB_GRF * rr;
                        if (rr >= m.neqrow && !(Eo[7] < 0.f)) continue;
                        const int body = __builtin_amdgcn_readfirstlane(__float_as_int(Eo[9]));
                        const uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)BL.chainmask, body);
                        const uint32_t mhi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(BL.chainmask >> 32), body);
                        const uint64_t mask = ((uint64_t)mhi << 32) | mlo;
                        if (dof_lane && ((mask >> lane) & 1ull)) {
                            const float Dj = Eo[6] * sdot(S, Eo);
                            gc += Dj * Eo[7];
#pragma unroll
                            for (int c6 = 0; c6 < 6; c6++) F[c6] += Dj * Eo[c6];
                        }
                    }
                }
                float gi = 0.f;
                if (dof_lane) {
                    gi = Ma[lane] - (tau[lane] - bias[lane]) + gc;
                    if (limact) {
                        const float lj = ljar[lane];
                        if (lj < 0.f) gi += lD[lane] * lj;
                    }
                    g[lane] = gi;
                }
                float gn = sqrtf(wsum(gi * gi));
                if (gn < m.tol_scale) break;
                if (TIMED && SUBREC && sub < RB_STATS_SUB && it < RB_STATS_FP) {
                    // fingerprint of the active set this update is built from: sum over active rows
                    // of (id + 1) * 2654435761 mod 2^32, id = 4 c + e for pyramid row e of contact c
                    // (a frictionless contact's one row is e = 0), 256 + dof for a limit row
                    uint32_t fpl = 0;
                    if (cell) {
                        // an elliptic contact's three rows count unless it separates (zone 0),
                        // as 2048 + id inside the cone (zone 2)
                        if (bits != 0)
                            for (int e = 0; e < celld; e++)
                                fpl += (uint32_t)((e < 4 ? 4 * lane + e : 1024 + 6 * lane + e - 4) + (bits == 2 ? 2048 : 0) + 1) *
                                       2654435761u;
                    } else if (has) {
#pragma unroll
                        for (int e = 0; e < 4; e++)
                            if (C.jar[e] < 0.f && (e == 0 || !(EXT && (C.ids >> 24))))
                                fpl += (uint32_t)(4 * lane + e + 1) * 2654435761u;
                    }
                    if (limact && dof_lane && lD[lane] != 0.f && ljar[lane] < 0.f)
                        fpl += (uint32_t)(256 + lane + 1) * 2654435761u;
                    // generic rows: equality row k of constraint q 512 + 6 q + k (always active),
                    // extra row e of contact c 1024 + 6 c + e
                    if (grown && (grbil || Er[7] < 0.f))
                        fpl += (uint32_t)(__float_as_int(Er[10]) + 1) * 2654435761u;
                    fpl = wsum_u32(fpl);
                    if (lane == 0) SUBREC[RB_SUBSTAT * sub + 5 + it] = (int32_t)fpl;
                }
                // Hessian row in registers: H_ij = M_ij + S_j . F_i over the chain of i
                // (computed for every position and selected: past the chain the index stays in
                // LDS -- the next rows of M, or H after it -- and the value is discarded)
                float Hr[MAXD];
#pragma unroll
                for (int t = 0; t < MAXD; t++) {
                    const int anc_t = (int)((opaque(DL.anc[t >> 2]) >> (8 * (t & 3))) & 0xffu);
                    const float h = Mm[DL.rowadr + t] + sdot(cdof + 6 * anc_t, F);
                    Hr[t] = t < DL.depth ? h : 0.f;
                }
                if (limact) {
                    // the active limit row's term D on the dof's diagonal
                    const float hl = (dof_lane && ljar[lane] < 0.f) ? fabsf(lD[lane]) : 0.f;
#pragma unroll
                    for (int t = 0; t < MAXD; t++)
                        if (t == DL.depth - 1) Hr[t] += hl;
                }
                RB_STAGE(6);
                if (EXT == 3 && m.nmm > 0) {
                    // Dense Newton Hessian: a contact between two moving bodies couples the two
                    // branches below their common ancestor, beyond M's tree sparsity.  The tree
                    // part is the row above; each such contact adds U' W U (U: its frame rows'
                    // Jacobian, W: the sum over its active pyramid rows of D a a', a = (1, +-mu, 0)
                    // or (1, 0, +-mu)); then a right-looking L D L' of the lower triangle in LDS,
                    // row i on lane i, and the two triangular solves by lane broadcasts.
                    float* HD = L + m.o_hd;
                    float* UD = HD + ((nv * nv + 3) & ~3);
                    if (dof_lane) {
                        for (int j = 0; j <= lane; j++) HD[lane * nv + j] = 0.f;
#pragma unroll
                        for (int t = 0; t < MAXD; t++)
                            if (t < DL.depth) HD[lane * nv + DL.ancestor(t)] = Hr[t];
                    }
                    for (int c = 0; c < ncon; c++) {
                        const int b1c = __builtin_amdgcn_readlane(C.body1, c);
                        if (b1c == 0) continue;
                        const int b2c = __builtin_amdgcn_readlane(C.body, c);
                        const uint64_t m2 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(BL.chainmask >> 32), b2c) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)BL.chainmask, b2c);
                        const uint64_t m1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(BL.chainmask >> 32), b1c) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)BL.chainmask, b1c);
                        float r[3], n[3], t1[3], t2[3];
                        for (int k = 0; k < 3; k++) {
                            r[k] = rl(C.r[k], c); n[k] = rl(C.n[k], c); t1[k] = rl(C.t1[k], c);
                        }
                        cross(n, t1, t2);
                        const float mu = rl(C.mu, c);
                        float W00 = 0.f, W01 = 0.f, W02 = 0.f, W11 = 0.f, W22 = 0.f;
                        for (int e = 0; e < 4; e++) {
                            const float De = rl(C.D[e], c), je = rl(C.jar[e], c);
                            if (je < 0.f) {
                                const float sm = (e & 1) ? -mu : mu;
                                W00 += De;
                                if (e < 2) { W01 += De * sm; W11 += De * sm * sm; }
                                else { W02 += De * sm; W22 += De * sm * sm; }
                            }
                        }
                        float u0 = 0.f, u1 = 0.f, u2 = 0.f;
                        if (dof_lane) {
                            const float cf = (float)((m2 >> lane) & 1ull) - (float)((m1 >> lane) & 1ull);
                            float wr[3];
                            cross(S, r, wr);
                            const float vp[3] = {S[3] + wr[0], S[4] + wr[1], S[5] + wr[2]};
                            u0 = cf * dot(n, vp); u1 = cf * dot(t1, vp); u2 = cf * dot(t2, vp);
                            UD[lane] = u0; UD[nv + lane] = u1; UD[2 * nv + lane] = u2;
                        }
                        wave_sync();
                        if (dof_lane) {
                            const float v0 = W00 * u0 + W01 * u1 + W02 * u2;
                            const float v1 = W01 * u0 + W11 * u1;
                            const float v2 = W02 * u0 + W22 * u2;
                            for (int j = 0; j <= lane; j++)
                                HD[lane * nv + j] += v0 * UD[j] + v1 * UD[nv + j] + v2 * UD[2 * nv + j];
                        }
                        wave_sync();
                    }
                    for (int k = 0; k < nv; k++) {
                        wave_sync();
                        const float ik = 1.f / HD[k * nv + k];
                        if (lane > k && lane < nv) {
                            const float l = HD[lane * nv + k] * ik;
                            for (int j = k + 1; j <= lane; j++) HD[lane * nv + j] -= l * HD[j * nv + k];
                        }
                    }
                    wave_sync();
                    float y = dof_lane ? -gi : 0.f;
                    for (int k = 0; k < nv; k++) {
                        const float yk = rl(y, k);
                        if (lane > k && lane < nv) y -= HD[lane * nv + k] / HD[k * nv + k] * yk;
                    }
                    if (dof_lane) y /= HD[lane * nv + lane];
                    for (int k = nv - 1; k >= 0; k--) {
                        const float xk = rl(y, k);
                        if (lane < k) y -= HD[k * nv + lane] / HD[lane * nv + lane] * xk;
                    }
                    if (dof_lane) p[lane] = y;
                    wave_sync();
                } else {
                    float invd;
                    float x = factor_solve<MAXD>(m, DL, Hr, -gi, lane, piv, &invd);
                    if (dof_lane) p[lane] = x;
                    wave_sync();
                }
                RB_STAGE(7);
                // directional quantities for the line search
                spatial_mul(m, BL, DL, cdof, cinert, p, bvec, cvel, Mp, lane);
                float sr[6] = {0, 0, 0, 0, 0, 0};
                if (has) rows_of(C, bvec, sr, cellm, EXT == 3 ? C.body1 : 0);
                float pa = 0.f, pb = 0.f;
                if (dof_lane) {
                    pa = p[lane] * Mp[lane];
                    pb = p[lane] * (Ma[lane] - (tau[lane] - bias[lane]));
                }
                float gsr = 0.f;   // J p of the lane's generic row
                if (grown) {
                    gsr = sdot(bvec + 6 * __float_as_int(Er[9]), Er);
                    Er[8] = gsr;
                    if (grbil) {
                        // bilateral rows are quadratic along p: constant terms of every segment
                        pa += Er[6] * gsr * gsr;
                        pb += Er[6] * gsr * Er[7];
                    }
                }
                float A0 = wsum(pa), B0 = wsum(pb);
                float alpha = 0.f;
                // the limit row's direction J p, from LDS wherever it is needed
                auto lim_dir = [&]() {
                    const float Ds = lD[lane];
                    return Ds > 0.f ? p[lane] : (Ds < 0.f ? -p[lane] : 0.f);
                };
                if (A0 > 0.f) {
                    float bp[4];
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        bp[e] = (has && sr[e] != 0.f) ? -C.jar[e] * __builtin_amdgcn_rcpf(sr[e]) : INFINITY;
                    }
                    // the lane's unilateral generic row: residual, D and breakpoint
                    const bool gu = grown && !grbil;
                    const float gj = gu ? Er[7] : 0.f, gD = gu ? Er[6] : 0.f;
                    const float gbp = (gu && gsr != 0.f) ? -gj * __builtin_amdgcn_rcpf(gsr) : INFINITY;
                    if (EXT >= 2 && m.cone && ncon > 0) {
                        // elliptic contacts make phi(alpha) convex and C1 but not piecewise
                        // quadratic: Newton's method on phi'(alpha) = 0 from alpha = 0, kept inside
                        // the bracket of a sign change (bisection when a step leaves it)
                        const float mue = C.mu * m.rsqrt_impratio;
                        auto dphi = [&](float al, float* d2) {
                            float d1l = 0.f, d2l = 0.f;
                            if (cell) {
                                float jj[NE];
#pragma unroll
                                for (int a = 0; a < NE; a++) jj[a] = C.jar[a] + al * sr[a];
                                float cst, ge[6];
                                EllCone E;
                                ell_eval<NE>(jj, C.D[0], C.D[1], C.D[3], NE > 4 ? C.D[4] : 0.f, mue, &cst, ge, &E);
#pragma unroll
                                for (int a = 0; a < NE; a++) d1l += ge[a] * sr[a];
                                d2l += ell_vhv<NE>(E, sr);
                            } else if (has) {
#pragma unroll
                                for (int e = 0; e < 4; e++) {
                                    const float j = C.jar[e] + al * sr[e];
                                    if (j < 0.f || (j == 0.f && sr[e] < 0.f)) {
                                        d1l += C.D[e] * sr[e] * j;
                                        d2l += C.D[e] * sr[e] * sr[e];
                                    }
                                }
                            }
                            if (limact && dof_lane) {
                                const float sl = lim_dir(), lj = ljar[lane] + al * sl, Dl = fabsf(lD[lane]);
                                if (lj < 0.f || (lj == 0.f && sl < 0.f)) {
                                    d1l += Dl * sl * lj;
                                    d2l += Dl * sl * sl;
                                }
                            }
                            if (gu) {
                                const float j = gj + al * gsr;
                                if (j < 0.f || (j == 0.f && gsr < 0.f)) {
                                    d1l += gD * gsr * j;
                                    d2l += gD * gsr * gsr;
                                }
                            }
                            *d2 = A0 + wsum(d2l);
                            return al * A0 + B0 + wsum(d1l);
                        };
                        float d2, d1 = dphi(0.f, &d2);
                        if (d1 < 0.f) {
                            const float tolg = 1e-6f * fabsf(d1);
                            float lo = 0.f, hi = INFINITY, al = 0.f;
                            for (int k = 0; k < 24; k++) {
                                if (TIMED) seg_sub++;
                                if (fabsf(d1) <= tolg) break;
                                if (d1 < 0.f) lo = al; else hi = al;
                                if (hi < INFINITY && hi - lo <= 1e-7f * hi) break;
                                float nxt = al - d1 / d2;
                                if (!(nxt > lo && nxt < hi)) nxt = hi < INFINITY ? 0.5f * (lo + hi) : 2.f * fmaxf(lo, 1.f);
                                al = nxt;
                                d1 = dphi(al, &d2);
                            }
                            alpha = al;
                        }
                    } else {
                    float at = 0.f;
                    int guard = 4 * ncon + 2 + (limact ? nv : 0) + nx;
                    for (int k = 0; k < guard; k++) {
                        if (TIMED) seg_sub++;
                        float sa = 0.f, sb = 0.f, nxt = INFINITY;
                        if (has) {
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                float s = sr[e];
                                bool act = s > 0.f ? (at < bp[e]) : (s < 0.f ? (at >= bp[e]) : (C.jar[e] < 0.f));
                                if (act) {
                                    sa += C.D[e] * s * s;
                                    sb += C.D[e] * s * C.jar[e];
                                }
                                if (bp[e] > at) nxt = fminf(nxt, bp[e]);
                            }
                        }
                        if (limact && dof_lane) {
                            const float lj = ljar[lane], Dl = fabsf(lD[lane]), sl = lim_dir();
                            const float bpl = sl != 0.f ? -lj * __builtin_amdgcn_rcpf(sl) : INFINITY;
                            const bool act = sl > 0.f ? (at < bpl) : (sl < 0.f ? (at >= bpl) : (lj < 0.f));
                            if (act) {
                                sa += Dl * sl * sl;
                                sb += Dl * sl * lj;
                            }
                            if (bpl > at) nxt = fminf(nxt, bpl);
                        }
                        if (gu) {
                            const bool act = gsr > 0.f ? (at < gbp) : (gsr < 0.f ? (at >= gbp) : (gj < 0.f));
                            if (act) {
                                sa += gD * gsr * gsr;
                                sb += gD * gsr * gj;
                            }
                            if (gbp > at) nxt = fminf(nxt, gbp);
                        }
                        float Aseg = A0 + wsum(sa), Bseg = B0 + wsum(sb);
                        nxt = wmin(nxt);
                        float root = -Bseg * __builtin_amdgcn_rcpf(Aseg);
                        if (root <= nxt) {
                            alpha = fmaxf(root, 0.f);
                            break;
                        }
                        at = nxt;
                        alpha = at;
                    }
                    }
                }
                // update a, M a and the row residuals along p
                float qf2 = 0.f;
                for (int i = lane; i < nv; i += RB_WAVE) {
                    acc[i] += alpha * p[i];
                    Ma[i] += alpha * Mp[i];
                    qf2 += (acc[i] - a0[i]) * (Ma[i] - (tau[i] - bias[i]));
                }
                float fc = 0.f;
                if (has) {
#pragma unroll
                    for (int e = 0; e < (EXT == 4 ? 6 : 4); e++) C.jar[e] += alpha * sr[e];
                    fc += con_cost(C.jar);
                }
                if (limact && dof_lane) {
                    const float lj = ljar[lane] + alpha * lim_dir();
                    ljar[lane] = lj;
                    const float mn = fminf(lj, 0.f);
                    fc += 0.5f * fabsf(lD[lane]) * mn * mn;
                }
                if (grown) {
                    const float ej = Er[7] + alpha * Er[8];
                    Er[7] = ej;
                    fc += gr_cost(ej);
                }
                float fnew = 0.5f * wsum(qf2) + wsum(fc);
                wave_sync();
                float improvement = fcur - fnew;
                fcur = fnew;
                RB_STAGE(8);
                if (improvement < m.tol_scale) { it++; break; }
            }
            if (it >= m.maxiter) itercap = true;
            if (TIMED) {
                st_iter += it;
                st_seg += seg_sub;
                // rows, and rows active at the solution (a frictionless contact has one row)
                const bool fl = has && EXT && (C.ids >> 24);
                int act = 0, nrow = has ? (fl ? 1 : (cell ? celld : 4)) : 0;
                if (cell) {
                    float cst, ge[6];
                    EllCone E;
                    act += ell_eval<NE>(C.jar, C.D[0], C.D[1], C.D[3], NE > 4 ? C.D[4] : 0.f, C.mu * m.rsqrt_impratio, &cst, ge, &E) != 0
                               ? celld : 0;
                } else if (has) {
                    for (int e = 0; e < 4; e++) act += C.jar[e] < 0.f && (e == 0 || !fl);
                }
                if (limact && lane < nv && lD[lane] != 0.f) {
                    act += ljar[lane] < 0.f;
                    nrow += 1;
                }
                if (grown) {
                    act += grbil || Er[7] < 0.f;
                    nrow += 1;
                }
                const int actw = (int)wsum_u32((uint32_t)act);
                const int nroww = (int)wsum_u32((uint32_t)nrow);
                st_rows += actw;
                if (SUBREC && sub < RB_STATS_SUB && lane == 0) {
                    SUBREC[RB_SUBSTAT * sub + 1] = nroww;
                    SUBREC[RB_SUBSTAT * sub + 2] = it;
                    SUBREC[RB_SUBSTAT * sub + 3] = actw;
                    SUBREC[RB_SUBSTAT * sub + 4] = seg_sub;
                }
            }
        }
        if (TIMED) st_con += ncon;
        if (TIMED && SUBREC && sub < RB_STATS_SUB && lane == 0) SUBREC[RB_SUBSTAT * sub] = ncon;
        RB_STAGE(6);
        if (itercap) status |= RB_STATUS_ITERCAP;

        // ---- first-substep taps
        if (TIMED && A.want_taps && sub == 0) {
            for (int i = lane; i < nv; i += RB_WAVE) {
                size_t base = (size_t)w * nv;
                if (A.taps.bias) A.taps.bias[base + i] = bias[i];
                if (A.taps.a0) A.taps.a0[base + i] = a0[i];
                if (A.taps.qacc) A.taps.qacc[base + i] = acc[i];
                if (A.taps.M) {
                    // dense row i: M_ij from row i if j is on i's chain, from row j if i is on j's
                    float* Mo = A.taps.M + (size_t)w * nv * nv + (size_t)i * nv;
                    int di = m.dof_depth[i];
                    for (int j = 0; j < nv; j++) {
                        int dj = m.dof_depth[j];
                        float val = 0.f;
                        if (dj <= di && m.dof_anc[i * m.maxd + dj - 1] == j)
                            val = Mm[m.dof_rowadr[i] + dj - 1];
                        else if (di < dj && m.dof_anc[j * m.maxd + di - 1] == i)
                            val = Mm[m.dof_rowadr[j] + di - 1];
                        Mo[j] = val;
                    }
                }
            }

        }

        // ---- joint damping integrated implicitly: the step applies a_int = (M + dt B)^-1 M a,
        // M a being the total force the solution carries (tau - c without a solve, the tracked
        // M a after one).  Factored like M, with dt B on the damped dofs' diagonals; a_int goes
        // to tmp, while the solver's a stays the next warm start.
        const float* aI = acc;
        if (EXT && m.ndamp > 0) {
            float Hr[MAXD];
#pragma unroll
            for (int t = 0; t < MAXD; t++) Hr[t] = t < DL.depth ? Mm[DL.rowadr + t] : 0.f;
            const float bd = lane < nv ? m.dt * m.dof_damping[lane] : 0.f;
#pragma unroll
            for (int t = 0; t < MAXD; t++)
                if (t == DL.depth - 1) Hr[t] += bd;
            const bool solved = ncon > 0 || limact || gract;
            const float rhs = lane < nv ? (solved ? Ma[lane] : tau[lane] - bias[lane]) : 0.f;
            float invd;
            const float x = factor_solve<MAXD>(m, DL, Hr, rhs, lane, piv, &invd);
            if (lane < nv) tmp[lane] = x;
            wave_sync();
            aI = tmp;
        }

        // ---- semi-implicit Euler (one lane per joint), committed only if everything is finite.
        // The joint update is evaluated twice -- once to test, once to write -- rather than
        // holding the new state in registers across the wave-wide test.
        const int jl = lane < m.njnt ? lane : -1;
        auto euler = [&](bool commit) {
            bool bad = false;
            if (jl < 0) return bad;
            const int jt = m.jnt_type[jl], qa = m.jnt_qadr[jl], da = m.jnt_dadr[jl];
            const float dt = m.dt;
            if (jt == RB_JNT_HINGE) {
                const float vn = v[da] + dt * aI[da];
                const float qn = q[qa] + dt * vn;
                bad = !finitef(vn) || !finitef(qn);
                if (commit) { v[da] = vn; q[qa] = qn; }
            } else {
                float vn[6], qn[7];
                for (int k = 0; k < 6; k++) vn[k] = v[da + k] + dt * aI[da + k];
                for (int k = 0; k < 3; k++) qn[k] = q[qa + k] + dt * vn[k];
                float th[3] = {dt * vn[3], dt * vn[4], dt * vn[5]};
                float ang = sqrtf(dot(th, th));
                float dq[4] = {1.f, 0.f, 0.f, 0.f};
                if (ang > 0.f) {
                    float sn = sinf(0.5f * ang) / ang;
                    dq[0] = cosf(0.5f * ang); dq[1] = th[0] * sn; dq[2] = th[1] * sn; dq[3] = th[2] * sn;
                }
                float qq[4];
                qmul(q + qa + 3, dq, qq);
                float inv = 1.0f / sqrtf(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
                for (int k = 0; k < 4; k++) qn[3 + k] = qq[k] * inv;
                for (int k = 0; k < 7; k++) bad |= !finitef(qn[k]);
                for (int k = 0; k < 6; k++) bad |= !finitef(vn[k]);
                if (commit) {
                    for (int k = 0; k < 6; k++) v[da + k] = vn[k];
                    for (int k = 0; k < 7; k++) q[qa + k] = qn[k];
                }
            }
            return bad;
        };
        bool bad = false;
        for (int i = lane; i < nv; i += RB_WAVE) bad |= !finitef(aI[i]);
        bad |= euler(false);
        bool anybad = __any(bad);
        wave_sync();
        if (anybad) {
            status |= RB_STATUS_NONFINITE;
            frozen = true;
            ncon = 0;
            break;
        }
        euler(true);
        for (int i = lane; i < nv; i += RB_WAVE) aws[i] = acc[i];
        wave_sync();
        RB_STAGE(9);
    }

    // ---- egress
    for (int i = lane; i < nq; i += RB_WAVE) A.qpos[(size_t)w * nq + i] = q[i];
    for (int i = lane; i < nv; i += RB_WAVE) {
        A.qvel[(size_t)w * nv + i] = v[i];
        A.W.qacc_ws[(size_t)w * nv + i] = aws[i];
    }
    if (TIMED && A.want_taps && A.taps.stats && lane == 0) {
        int32_t* S = A.taps.stats + (size_t)w * RB_NSTATS;
        S[0] = st_con; S[1] = st_rows; S[2] = st_iter; S[3] = st_seg;
        for (int k = 0; k < RB_NSTAGE; k++) S[4 + k] = (int32_t)(stage_cyc[k] >> 4);
    }
    if (lane == 0) {
        A.W.status[w] = status;
        if (A.status_out) A.status_out[w] = status;
        if (A.want_contacts && A.co.ncon) A.co.ncon[w] = ncon;
    }
    if (A.want_contacts && lane < ncon) {
        size_t slot = (size_t)w * m.ncap + lane;
        if (A.co.geom) { A.co.geom[2 * slot] = C.ids & 0xff; A.co.geom[2 * slot + 1] = (C.ids >> 8) & 0xff; }
        if (A.co.feature) A.co.feature[slot] = (C.ids >> 16) & 0xff;
        if (A.co.dist) A.co.dist[slot] = C.dist;
        if (A.co.pos) {
            A.co.pos[3 * slot] = C.r[0] + xpos[3];
            A.co.pos[3 * slot + 1] = C.r[1] + xpos[4];
            A.co.pos[3 * slot + 2] = C.r[2] + xpos[5];
        }
        if (A.co.frame) {
            float* F = A.co.frame + 9 * slot;
            float t2o[3];
            cross(C.n, C.t1, t2o);
            for (int k = 0; k < 3; k++) { F[k] = C.n[k]; F[3 + k] = C.t1[k]; F[6 + k] = t2o[k]; }
        }
        if (A.co.force && EXT >= 2 && m.cone && !(C.ids >> 24)) {
            // elliptic cone: the frame rows' forces, minus the cost's gradient
            float cst, ge[6];
            EllCone E;
            ell_eval<NE>(C.jar, C.D[0], C.D[1], C.D[3], NE > 4 ? C.D[4] : 0.f, C.mu * m.rsqrt_impratio, &cst, ge, &E);
            A.co.force[3 * slot] = -ge[0];
            A.co.force[3 * slot + 1] = -ge[1];
            A.co.force[3 * slot + 2] = -ge[2];
        } else if (A.co.force) {
            float f[4];
            for (int e = 0; e < 4; e++) f[e] = -C.D[e] * fminf(C.jar[e], 0.f);
            // every pyramid row, the torsional and rolling ones included, carries the normal once
            float fx = 0.f;
            if (EXT >= 2)
                for (int e = 0; e < xr; e++) {
                    const float* G = L + m.o_gr + RB_GRF * (xbase + e);
                    fx += -G[6] * fminf(G[7], 0.f);
                }
            A.co.force[3 * slot] = f[0] + f[1] + f[2] + f[3] + fx;
            A.co.force[3 * slot + 1] = C.mu * (f[0] - f[1]);
            A.co.force[3 * slot + 2] = C.mu * (f[2] - f[3]);
        }
    }
}

// One world per 64-lane workgroup.  EXT: the level of extended code -- 1 for box-box,
// sphere-box, capsule-box and height-field pairs, more than 64 pairs, joint limits, damping and
// frictionless contacts; 2 adds equality constraints, torsional / rolling friction and elliptic
// cones up to condim 4; 3 is level 2 with contacts between two moving bodies, 4 level 2 with
// elliptic cones up to condim 6 (each level kept out of the other instantiations so their
// register allocation is not shaped by it).
template <int MAXD, bool TIMED, int EXT>
__global__ __launch_bounds__(RB_WAVE) __attribute__((amdgpu_waves_per_eu(RB_WAVES_PER_EU, 8))) void step_kernel(
    DevModel m, StepArgs A) {
    extern __shared__ float lds[];
    const int w = blockIdx.x;
    if (w >= A.n) return;
    world_step<MAXD, TIMED, EXT>(m, A, w, lds);
}

// The same step compiled for 4 resident waves per SIMD (at most 128 registers, more spills):
// worth it when the model's LDS lets 16 worlds share a CU and the batch is more than one
// round of the 3-wave kernel -- the last round then has fewer worlds waiting on it.
template <int MAXD, int EXT>
__global__ __launch_bounds__(RB_WAVE) __attribute__((amdgpu_waves_per_eu(4, 8))) void step_kernel_w4(
    DevModel m, StepArgs A) {
    extern __shared__ float lds[];
    const int w = blockIdx.x;
    if (w >= A.n) return;
    world_step<MAXD, false, EXT>(m, A, w, lds);
}

// Mixed-model launch: the grid walks an ordered list of (batch, world) items; each batch has
// its own compiled model and step arguments.  Every world runs exactly the code of the plain
// launch, so its result does not depend on the schedule or on the other batches.
struct MultiArgs {
    const DevModel* models;   // [nbatch]
    const StepArgs* args;     // [nbatch]
    const int* items;         // [nitems] batch << 24 | world
    int nitems;
    int wpg;                  // worlds per workgroup (one wave each, 1 .. RB_MAX_WPG)
    int lds_stride;           // LDS floats of one world's section of the workgroup's LDS
};

// Each item runs the instantiation the plain launch would use for its model (chain bound and
// box-box code), so a world computes exactly as in rb_step and small models keep lean code;
// MAXD and EXT bound what the plan's models need.
template <int MAXD, int EXT>
DEV void world_step_level(const DevModel& m, const StepArgs& A, int w, float* lds) {
    // the model's own level of extended code, at most the plan's
    const int lv = m.ext < EXT ? m.ext : EXT;
    if (EXT >= 4 && lv == 4) world_step<MAXD, false, (EXT >= 4 ? 4 : 0)>(m, A, w, lds);
    else if (EXT >= 3 && lv == 3) world_step<MAXD, false, (EXT >= 3 ? 3 : 0)>(m, A, w, lds);
    else if (EXT >= 2 && lv == 2) world_step<MAXD, false, (EXT >= 2 ? 2 : 0)>(m, A, w, lds);
    else if (EXT >= 1 && lv == 1) world_step<MAXD, false, (EXT >= 1 ? 1 : 0)>(m, A, w, lds);
    else world_step<MAXD, false, 0>(m, A, w, lds);
}

template <int MAXD, int EXT>
DEV void world_step_as_plain(const DevModel& m, const StepArgs& A, int w, float* lds) {
    if (MAXD >= 32 && m.maxd > 16) world_step_level<(MAXD >= 32 ? 32 : MAXD), EXT>(m, A, w, lds);
    else if (MAXD >= 16 && m.maxd > 8) world_step_level<(MAXD >= 16 ? 16 : MAXD), EXT>(m, A, w, lds);
    else world_step_level<8, EXT>(m, A, w, lds);
}

// The waves of a workgroup are independent worlds: wave k of workgroup g takes items g wpg + k,
// then every (grid size x wpg)-th after it, in its own LDS section.  No workgroup barrier is
// ever taken, so a wave that runs out of items simply ends.
template <int MAXD, int EXT>
DEV void multi_items(const MultiArgs& M, float* lds) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RB_WAVE));
    float* L = lds + wave * M.lds_stride;
    for (int it = blockIdx.x * M.wpg + wave; it < M.nitems; it += gridDim.x * M.wpg) {
        const int item = __builtin_amdgcn_readfirstlane(M.items[it]);
        const int b = item >> 24, w = item & 0xffffff;
        const DevModel& m = M.models[b];
        const StepArgs& A = M.args[b];
        if (w < A.n) world_step_as_plain<MAXD, EXT>(m, A, w, L);
    }
}

template <int MAXD, int EXT>
__global__ __launch_bounds__(RB_WAVE * RB_MAX_WPG) __attribute__((amdgpu_waves_per_eu(RB_WAVES_PER_EU, 8))) void multi_kernel(
    MultiArgs M) {
    extern __shared__ float lds[];
    multi_items<MAXD, EXT>(M, lds);
}

// 4 resident waves per SIMD, for plans whose models all fit that (chain bound <= 16 and LDS
// small enough for 16 worlds per CU)
template <int MAXD, int EXT>
__global__ __launch_bounds__(RB_WAVE * RB_MAX_WPG) __attribute__((amdgpu_waves_per_eu(4, 8))) void multi_kernel_w4(
    MultiArgs M) {
    extern __shared__ float lds[];
    multi_items<MAXD, EXT>(M, lds);
}

}  // namespace rbk

// ------------------------------------------------------------------ launch
// The instantiations are many (chain bound x level of extended code x plain, diagnostic, 4-wave
// and fused forms) and each carries a whole inlined step, so the library compiles this file in
// parts, in parallel: with RB_PART = k a translation unit defines only the launchers of part k
// (the explicit instantiations below), and part 0 also holds the dispatchers, which reach every
// launcher through explicit instantiation declarations.  Without RB_PART one unit holds all.
#ifndef RB_PART
#define RB_PART -1
#endif
#define RB_IN_PART(k) (RB_PART < 0 || RB_PART == (k))

template <int MAXD, bool TIMED, int EXT>
void launch_step_t(const DevModel& m, const rbk::StepArgs& A, int n, size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((rbk::step_kernel<MAXD, TIMED, EXT>), dim3(n), dim3(RB_WAVE), shmem, stream, m, A);
}
template <int MAXD, int EXT>
void launch_step_w4_t(const DevModel& m, const rbk::StepArgs& A, int n, size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((rbk::step_kernel_w4<MAXD, EXT>), dim3(n), dim3(RB_WAVE), shmem, stream, m, A);
}
template <int MAXD, int EXT>
void launch_multi_t(const rbk::MultiArgs& M, dim3 g, size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((rbk::multi_kernel<MAXD, EXT>), g, dim3(RB_WAVE * M.wpg), shmem, stream, M);
}
template <int MAXD, int EXT>
void launch_multi_w4_t(const rbk::MultiArgs& M, dim3 g, size_t shmem, hipStream_t stream) {
    hipLaunchKernelGGL((rbk::multi_kernel_w4<MAXD, EXT>), g, dim3(RB_WAVE * M.wpg), shmem, stream, M);
}

// X is empty (an explicit instantiation definition) or `extern` (a declaration)
#define RB_STEP_I(X, D, T, E) \
    X template void launch_step_t<D, T, E>(const DevModel&, const rbk::StepArgs&, int, size_t, hipStream_t);
#define RB_W4_I(X, D, E) \
    X template void launch_step_w4_t<D, E>(const DevModel&, const rbk::StepArgs&, int, size_t, hipStream_t);
#define RB_MULTI_I(X, D, E) X template void launch_multi_t<D, E>(const rbk::MultiArgs&, dim3, size_t, hipStream_t);
#define RB_MULTI_W4_I(X, D, E) \
    X template void launch_multi_w4_t<D, E>(const rbk::MultiArgs&, dim3, size_t, hipStream_t);
#define RB_LEVELS(F, X, ...) \
    F(X, __VA_ARGS__, 0) F(X, __VA_ARGS__, 1) F(X, __VA_ARGS__, 2) F(X, __VA_ARGS__, 3) F(X, __VA_ARGS__, 4)

// every launcher the dispatchers use
RB_LEVELS(RB_STEP_I, extern, 8, false) RB_LEVELS(RB_STEP_I, extern, 16, false) RB_LEVELS(RB_STEP_I, extern, 32, false)
RB_LEVELS(RB_STEP_I, extern, 8, true) RB_LEVELS(RB_STEP_I, extern, 16, true) RB_LEVELS(RB_STEP_I, extern, 32, true)
RB_LEVELS(RB_W4_I, extern, 8) RB_LEVELS(RB_W4_I, extern, 16)
RB_LEVELS(RB_MULTI_I, extern, 8) RB_LEVELS(RB_MULTI_I, extern, 16) RB_LEVELS(RB_MULTI_I, extern, 32)
RB_LEVELS(RB_MULTI_W4_I, extern, 8) RB_LEVELS(RB_MULTI_W4_I, extern, 16)

// The parts, each defining launchers that inline 10 to 19 steps in all (a fused launcher inlines
// one step per chain bound and level at or below its own).  RB_NPARTS must match the list.
#define RB_NPARTS 12
#if RB_IN_PART(0)
RB_LEVELS(RB_STEP_I, , 8, false) RB_LEVELS(RB_STEP_I, , 16, false) RB_LEVELS(RB_STEP_I, , 32, false)
#endif
#if RB_IN_PART(1)
RB_LEVELS(RB_STEP_I, , 8, true) RB_LEVELS(RB_STEP_I, , 16, true) RB_LEVELS(RB_STEP_I, , 32, true)
#endif
#if RB_IN_PART(2)
RB_LEVELS(RB_W4_I, , 8) RB_LEVELS(RB_W4_I, , 16)
RB_MULTI_I(, 8, 0) RB_MULTI_I(, 8, 1) RB_MULTI_I(, 8, 2)
#endif
#if RB_IN_PART(3)
RB_MULTI_I(, 8, 3) RB_LEVELS(RB_MULTI_W4_I, , 8)
#endif
#if RB_IN_PART(4)
RB_MULTI_I(, 16, 0) RB_MULTI_I(, 16, 1) RB_MULTI_I(, 16, 3)
#endif
#if RB_IN_PART(5)
RB_MULTI_I(, 16, 2) RB_MULTI_W4_I(, 16, 3)
#endif
#if RB_IN_PART(6)
RB_MULTI_W4_I(, 16, 0) RB_MULTI_W4_I(, 16, 1) RB_MULTI_W4_I(, 16, 2)
#endif
#if RB_IN_PART(7)
RB_MULTI_I(, 32, 0) RB_MULTI_I(, 32, 3)
#endif
#if RB_IN_PART(8)
RB_MULTI_I(, 32, 1) RB_MULTI_I(, 32, 2)
#endif
#if RB_IN_PART(9)
RB_MULTI_I(, 8, 4) RB_MULTI_I(, 16, 4)
#endif
#if RB_IN_PART(10)
RB_MULTI_I(, 32, 4)
#endif
#if RB_IN_PART(11)
RB_MULTI_W4_I(, 16, 4)
#endif

#if RB_IN_PART(0)
rbk::StepArgs rb_make_args(int n, const float* ctrl, float* qpos, float* qvel, const DevWorlds& W,
                           const DevContactsOut* co, uint32_t* status_out) {
    rbk::StepArgs A;
    A.n = n;
    A.ctrl = ctrl;
    A.qpos = qpos;
    A.qvel = qvel;
    A.W = W;
    A.want_contacts = co != nullptr;
    if (co) A.co = *co; else A.co = DevContactsOut{};
    A.status_out = status_out;
    A.want_taps = 0;
    A.taps = DevTaps{};
    return A;
}

size_t rb_step_args_size() { return sizeof(rbk::StepArgs); }

void rb_fill_step_args(void* dst, int n, const float* ctrl, float* qpos, float* qvel, const DevWorlds& W,
                       const DevContactsOut* co, uint32_t* status_out) {
    rbk::StepArgs A = rb_make_args(n, ctrl, qpos, qvel, W, co, status_out);
    *(rbk::StepArgs*)dst = A;
}

template <int EXT>
static void launch_multi_b(int maxd, const rbk::MultiArgs& M, dim3 g, size_t shmem, bool w4, hipStream_t stream) {
    if (maxd <= 8) {
        if (w4) launch_multi_w4_t<8, EXT>(M, g, shmem, stream);
        else launch_multi_t<8, EXT>(M, g, shmem, stream);
    } else if (maxd <= 16) {
        if (w4) launch_multi_w4_t<16, EXT>(M, g, shmem, stream);
        else launch_multi_t<16, EXT>(M, g, shmem, stream);
    } else {
        launch_multi_t<32, EXT>(M, g, shmem, stream);
    }
}

hipError_t rb_launch_multi(const DevModel* models, const void* args, const int* items, int nitems, int maxd,
                           int ext, int lds_floats, int lds_pad, int grid, int wpg, int waves, hipStream_t stream) {
    if (wpg < 1 || wpg > RB_MAX_WPG || grid < 1) return hipErrorInvalidValue;
    rbk::MultiArgs M;
    M.models = models;
    M.args = (const rbk::StepArgs*)args;
    M.items = items;
    M.nitems = nitems;
    M.wpg = wpg;
    M.lds_stride = lds_floats;
    size_t shmem = ((size_t)wpg * lds_floats + lds_pad) * sizeof(float);
    dim3 g((grid + wpg - 1) / wpg);   // grid counts worlds in flight, one wave each
    if (ext >= 4) launch_multi_b<4>(maxd, M, g, shmem, waves == 4, stream);
    else if (ext == 3) launch_multi_b<3>(maxd, M, g, shmem, waves == 4, stream);
    else if (ext == 2) launch_multi_b<2>(maxd, M, g, shmem, waves == 4, stream);
    else if (ext == 1) launch_multi_b<1>(maxd, M, g, shmem, waves == 4, stream);
    else launch_multi_b<0>(maxd, M, g, shmem, waves == 4, stream);
    return hipGetLastError();
}

template <bool TIMED, int EXT>
static void launch_step_d(const DevModel& m, const rbk::StepArgs& A, int n, size_t shmem, hipStream_t stream) {
    if (m.maxd <= 8) launch_step_t<8, TIMED, EXT>(m, A, n, shmem, stream);
    else if (m.maxd <= 16) launch_step_t<16, TIMED, EXT>(m, A, n, shmem, stream);
    else launch_step_t<32, TIMED, EXT>(m, A, n, shmem, stream);
}

template <int EXT>
static void launch_step_w4_d(const DevModel& m, const rbk::StepArgs& A, int n, size_t shmem, hipStream_t stream) {
    if (m.maxd <= 8) launch_step_w4_t<8, EXT>(m, A, n, shmem, stream);
    else launch_step_w4_t<16, EXT>(m, A, n, shmem, stream);
}

hipError_t rb_launch_step(const DevModel& m, int n, const float* ctrl, float* qpos, float* qvel, const DevWorlds& W,
                          const DevContactsOut* co, uint32_t* status_out, const DevTaps* taps, int waves,
                          hipStream_t stream) {
    rbk::StepArgs A;
    A.n = n;
    A.ctrl = ctrl;
    A.qpos = qpos;
    A.qvel = qvel;
    A.W = W;
    A.want_contacts = co != nullptr;
    if (co) A.co = *co; else A.co = DevContactsOut{};
    A.status_out = status_out;
    A.want_taps = taps != nullptr;
    if (taps) A.taps = *taps; else A.taps = DevTaps{};
    size_t shmem = (size_t)m.lds_floats * sizeof(float);
    const bool timed = taps != nullptr;   // every tap is served by the diagnostic instantiation
    const int lv = m.ext;   // the level of extended code the model needs
    if (timed) {
        if (lv >= 4) launch_step_d<true, 4>(m, A, n, shmem, stream);
        else if (lv == 3) launch_step_d<true, 3>(m, A, n, shmem, stream);
        else if (lv == 2) launch_step_d<true, 2>(m, A, n, shmem, stream);
        else if (lv == 1) launch_step_d<true, 1>(m, A, n, shmem, stream);
        else launch_step_d<true, 0>(m, A, n, shmem, stream);
    } else if (waves == 4 && m.maxd <= 16) {
        if (lv >= 4) launch_step_w4_d<4>(m, A, n, shmem, stream);
        else if (lv == 3) launch_step_w4_d<3>(m, A, n, shmem, stream);
        else if (lv == 2) launch_step_w4_d<2>(m, A, n, shmem, stream);
        else if (lv == 1) launch_step_w4_d<1>(m, A, n, shmem, stream);
        else launch_step_w4_d<0>(m, A, n, shmem, stream);
    } else {
        if (lv >= 4) launch_step_d<false, 4>(m, A, n, shmem, stream);
        else if (lv == 3) launch_step_d<false, 3>(m, A, n, shmem, stream);
        else if (lv == 2) launch_step_d<false, 2>(m, A, n, shmem, stream);
        else if (lv == 1) launch_step_d<false, 1>(m, A, n, shmem, stream);
        else launch_step_d<false, 0>(m, A, n, shmem, stream);
    }
    return hipGetLastError();
}
#endif  // RB_IN_PART(0)
