// Host runtime of librbstep: model validation and compilation into device tables, batches of
// world slots, and the C ABI declared in include/rbstep.h.
//
// The model pipeline mirrors the paper's scene path (section "Architecture", paragraph on
// the scene pipeline: a description is compiled on the CPU and transferred to the GPU): a
// host description is validated, flattened into structure-of-arrays tables (dof chains,
// tree levels, collision pairs, LDS layout) and uploaded once; every world shares them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rb_internal.h"
#include "rbstep.h"

hipError_t rb_launch_step(const DevModel& m, int n, const float* ctrl, float* qpos, float* qvel, const DevWorlds& W,
                          const DevContactsOut* co, uint32_t* status_out, const DevTaps* taps, int waves,
                          hipStream_t stream);
hipError_t rb_launch_reset(int nv, const int32_t* ids, int n, const float* qacc_ws, DevWorlds W, int capacity,
                           hipStream_t stream);
hipError_t rb_launch_fill(float* dst, float value, size_t count, hipStream_t stream);
hipError_t rb_launch_tile(float* dst, const float* src, size_t k, size_t copies, hipStream_t stream);
size_t rb_step_args_size();
void rb_fill_step_args(void* dst, int n, const float* ctrl, float* qpos, float* qvel, const DevWorlds& W,
                       const DevContactsOut* co, uint32_t* status_out);
hipError_t rb_launch_multi(const DevModel* models, const void* args, const int* items, int nitems, int maxd,
                           int ext, int lds_floats, int lds_pad, int grid, int wpg, int waves, hipStream_t stream);

namespace {

thread_local std::string g_err;
int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return RB_EHIP;
}

// ------------------------------------------------------------------ host-side double math
void qmul_d(const double* a, const double* b, double* o) {
    double t[4] = {a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                   a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                   a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                   a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]};
    std::memcpy(o, t, sizeof t);
}
void qmat_d(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
void mv_d(const double* R, const double* v, double* o) {
    double t[3];
    for (int i = 0; i < 3; i++) t[i] = R[3 * i] * v[0] + R[3 * i + 1] * v[1] + R[3 * i + 2] * v[2];
    std::memcpy(o, t, sizeof t);
}
void cross_d(const double* a, const double* b, double* o) {
    double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    std::memcpy(o, t, sizeof t);
}

// blob builder: 4-byte words, 8-byte aligned sections
struct Blob {
    std::vector<uint32_t> words;
    size_t add_i(const std::vector<int>& v) {
        align();
        size_t off = words.size();
        for (int x : v) words.push_back((uint32_t)x);
        if (v.empty()) words.push_back(0);
        return off;
    }
    size_t add_f(const std::vector<double>& v) {
        align();
        size_t off = words.size();
        for (double x : v) {
            float f = (float)x;
            uint32_t u;
            std::memcpy(&u, &f, 4);
            words.push_back(u);
        }
        if (v.empty()) words.push_back(0);
        return off;
    }
    size_t add_u64(const std::vector<uint64_t>& v) {
        align();
        size_t off = words.size();
        for (uint64_t x : v) {
            words.push_back((uint32_t)(x & 0xffffffffu));
            words.push_back((uint32_t)(x >> 32));
        }
        if (v.empty()) { words.push_back(0); words.push_back(0); }
        return off;
    }
    void align() {
        while (words.size() % 2) words.push_back(0);
    }
};

}  // namespace

struct rb_model {
    DevModel dm;
    void* blob = nullptr;
    int device = 0;
    int maxcon_static = 0;
    double meaninertia = 1.0;
    int nv_ = 0, nq_ = 0, nu_ = 0, nbody_ = 0, ngeom_ = 0;
};

struct rb_batch {
    const rb_model* model = nullptr;
    int capacity = 0;
    int waves = 0;          // resident waves per SIMD of the plain launch: 0 automatic, 3 or 4
    DevWorlds W{};
    DevModel dm;   // model copy with this batch's contact capacity
    void* mem = nullptr;
    void* field_mem[4] = {};   // model fields expanded per world (geom size, body pos, kp, kd)
    int version = 0;           // bumped when W changes (an expansion): plans re-bind
};

namespace {

// LDS sections from the pivot buffer on.  The pivot buffer holds one row per pivot of a height
// level at the stride of the kernel instantiation that runs the model (its chain bound + 4),
// so a model run by a deeper instantiation (a fused launch beside a deeper model) needs this
// tail laid out again for that bound.
void layout_tail(DevModel& m, int kernel_maxd) {
    auto r4 = [](int n) { return (n + 3) & ~3; };
    int o = m.o_piv + r4(m.maxpiv * (kernel_maxd + 4));
    m.o_rowadr = o;
    o += r4(m.nv);
    m.o_bb = o;
    o += r4(RB_BB_FLOATS * m.nbb);
    m.o_gr = o;
    o += r4(RB_GRF * (m.neqrow + m.nxmax));
    // dense Newton Hessian [nv, nv] and three direction vectors [3, nv] (two-body contacts)
    m.o_hd = o;
    if (m.nmm > 0) o += r4(m.nv * m.nv) + r4(3 * m.nv);
    m.lds_floats = o;
}

// Compile a description into host tables; returns RB_OK or RB_EINVAL with a message.
int compile_model(const rb_model_desc* d, rb_model* M) {
    const int nb = d->nbody, nj = d->njnt, ng = d->ngeom, nu = d->nu;
    if (nb < 2) return fail(RB_EINVAL, "model needs at least one body besides the world");
    if (nj < 1) return fail(RB_EINVAL, "model needs at least one joint");
    if (ng < 0 || nu < 0) return fail(RB_EINVAL, "negative sizes");
    // contact ids carry geom indices in 8-bit fields
    if (ng > RB_MAX_GEOM) return fail(RB_EINVAL, "more than 256 geoms");
    // every real number of the description must be finite
    auto finite = [](const double* x, int n) {
        for (int i = 0; i < n; i++)
            if (!std::isfinite(x[i])) return false;
        return true;
    };
    const struct { const double* x; int n; const char* what; } reals[] = {
        {d->body_pos, 3 * nb, "body pos"}, {d->body_quat, 4 * nb, "body quat"}, {d->body_ipos, 3 * nb, "body ipos"},
        {d->body_iquat, 4 * nb, "body iquat"}, {d->body_mass, nb, "body mass"}, {d->body_inertia, 3 * nb, "body inertia"},
        {d->jnt_pos, 3 * nj, "joint pos"}, {d->jnt_axis, 3 * nj, "joint axis"}, {d->jnt_armature, nj, "joint armature"},
        {d->geom_pos, 3 * ng, "geom pos"}, {d->geom_quat, 4 * ng, "geom quat"}, {d->geom_size, 3 * ng, "geom size"},
        {d->geom_friction, ng, "geom friction"}, {d->geom_margin, ng, "geom margin"}, {d->act_kp, nu, "actuator kp"},
        {d->act_kd, nu, "actuator kd"}, {d->act_gear, nu, "actuator gear"}, {&d->timestep, 1, "timestep"},
        {d->gravity, 3, "gravity"}, {&d->tolerance, 1, "tolerance"}, {d->solref, 2, "solref"}, {d->solimp, 5, "solimp"}};
    for (const auto& r : reals) {
        if (r.n > 0 && !r.x) return fail(RB_EINVAL, std::string("missing ") + r.what);
        if (r.n > 0 && !finite(r.x, r.n)) return fail(RB_EINVAL, std::string("non-finite ") + r.what);
    }
    auto P = [&](int b) { return d->body_parent[b]; };
    for (int b = 1; b < nb; b++)
        if (P(b) < 0 || P(b) >= b) return fail(RB_EINVAL, "body parent must precede the body");
    for (int b = 0; b < nb; b++) {
        const double* q = d->body_quat + 4 * b;
        double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (std::fabs(n - 1) > 1e-6) return fail(RB_EINVAL, "body quaternion is not unit");
        const double* iq = d->body_iquat + 4 * b;
        n = std::sqrt(iq[0] * iq[0] + iq[1] * iq[1] + iq[2] * iq[2] + iq[3] * iq[3]);
        if (b > 0 && std::fabs(n - 1) > 1e-6) return fail(RB_EINVAL, "inertia quaternion is not unit");
        if (b == 0) continue;
        if (!(d->body_mass[b] > 0)) return fail(RB_EINVAL, "body mass must be positive");
        const double* I = d->body_inertia + 3 * b;
        if (!(I[0] > 0 && I[1] > 0 && I[2] > 0)) return fail(RB_EINVAL, "principal inertias must be positive");
        const double tol = 1 + 1e-12;
        if (I[0] + I[1] < I[2] / tol || I[1] + I[2] < I[0] / tol || I[0] + I[2] < I[1] / tol)
            return fail(RB_EINVAL, "inertia violates the triangle inequality");
    }
    // joints
    std::vector<int> bjnt(nb, -1), jtype(nj), jbody(nj), jq(nj), jd(nj);
    int nq = 0, nv = 0, last = 0;
    for (int j = 0; j < nj; j++) {
        int b = d->jnt_body[j];
        if (b <= 0 || b >= nb) return fail(RB_EINVAL, "joint on an invalid body");
        if (bjnt[b] >= 0) return fail(RB_EINVAL, "more than one joint on a body");
        if (b < last) return fail(RB_EINVAL, "joints must be listed in body order");
        last = b;
        bjnt[b] = j;
        jtype[j] = d->jnt_type[j];
        jbody[j] = b;
        jq[j] = nq;
        jd[j] = nv;
        const double rlo = d->jnt_range ? d->jnt_range[2 * j] : 0.0, rhi = d->jnt_range ? d->jnt_range[2 * j + 1] : 0.0;
        const double damp = d->jnt_damping ? d->jnt_damping[j] : 0.0;
        if (!(std::isfinite(damp) && damp >= 0)) return fail(RB_EINVAL, "joint damping must be finite and >= 0");
        if (jtype[j] == RB_JNT_FREE) {
            if (P(b) != 0) return fail(RB_EINVAL, "a free joint must be on a child of the world");
            if (rlo != rhi) return fail(RB_EINVAL, "free joints take no range");
            if (damp != 0) return fail(RB_EINVAL, "free joints take no damping");
            nq += 7;
            nv += 6;
        } else if (jtype[j] == RB_JNT_HINGE) {
            const double* ax = d->jnt_axis + 3 * j;
            if (!(std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]) > 0))
                return fail(RB_EINVAL, "hinge axis is zero");
            if (!(std::isfinite(rlo) && std::isfinite(rhi)) || rlo > rhi)
                return fail(RB_EINVAL, "joint range must be finite with lower <= upper");
            nq += 1;
            nv += 1;
        } else {
            return fail(RB_EINVAL, "unknown joint type");
        }
    }
    if (nv > RB_MAX_DOF) return fail(RB_EINVAL, "more than 64 dofs");
    // dof tree
    std::vector<int> dof_body(nv), dof_parent(nv), dof_depth(nv), blast(nb, -1), bdepth(nb, 0);
    for (int b = 1; b < nb; b++) {
        int p = P(b);
        int parent_dof = blast[p];
        int j = bjnt[b];
        if (j >= 0) {
            int nd = jtype[j] == RB_JNT_FREE ? 6 : 1;
            for (int k = 0; k < nd; k++) {
                int i = jd[j] + k;
                dof_body[i] = b;
                dof_parent[i] = k == 0 ? parent_dof : i - 1;
                dof_depth[i] = dof_parent[i] < 0 ? 1 : dof_depth[dof_parent[i]] + 1;
            }
            blast[b] = jd[j] + nd - 1;
        } else {
            blast[b] = parent_dof;
        }
        bdepth[b] = blast[b] < 0 ? 0 : dof_depth[blast[b]];
    }
    int maxd = 0;
    for (int i = 0; i < nv; i++) maxd = std::max(maxd, dof_depth[i]);
    if (maxd > 32) return fail(RB_EINVAL, "dof chain deeper than 32");
    int tmaxd = maxd <= 8 ? 8 : (maxd <= 16 ? 16 : 32);
    std::vector<int> anc((size_t)nv * tmaxd, -1), rowadr(nv);
    int nM = 0;
    for (int i = 0; i < nv; i++) {
        rowadr[i] = nM;
        nM += dof_depth[i];
        for (int k = i, t = dof_depth[i] - 1; k >= 0; k = dof_parent[k], t--) anc[(size_t)i * tmaxd + t] = k;
    }
    std::vector<int> desc_start(nv + 1, 0), desc_list;
    for (int i = 0; i < nv; i++) {
        desc_start[i] = (int)desc_list.size();
        for (int k = i + 1; k < nv; k++)
            if (dof_depth[k] > dof_depth[i] && anc[(size_t)k * tmaxd + dof_depth[i] - 1] == i) desc_list.push_back(k);
    }
    desc_start[nv] = (int)desc_list.size();
    std::vector<int> dl_start(maxd + 2, 0), dl_dof;
    for (int lev = 0; lev <= maxd + 1; lev++) {
        dl_start[lev] = (int)dl_dof.size();
        for (int i = 0; i < nv; i++)
            if (dof_depth[i] == lev) dl_dof.push_back(i);
    }
    // body tree levels and children
    std::vector<int> blevel(nb, 0);
    int nblevel = 0;
    for (int b = 1; b < nb; b++) {
        blevel[b] = blevel[P(b)] + 1;
        nblevel = std::max(nblevel, blevel[b]);
    }
    std::vector<int> lv_start(nblevel + 2, 0), lv_body;
    for (int lev = 0; lev <= nblevel + 1; lev++) {
        lv_start[lev] = (int)lv_body.size();
        for (int b = 0; b < nb; b++)
            if (blevel[b] == lev) lv_body.push_back(b);
    }
    if (nb > 64) return fail(RB_EINVAL, "more than 64 bodies");
    std::vector<int> ch_start(nb + 1, 0), ch_list, bchild(nb, 0), bsize(nb, 1);
    for (int b = 0; b < nb; b++) {
        ch_start[b] = (int)ch_list.size();
        uint32_t packed = 0xffffffffu;
        int nc = 0;
        for (int c = b + 1; c < nb; c++)
            if (P(c) == b) {
                ch_list.push_back(c);
                if (b > 0 && nc >= 4) return fail(RB_EINVAL, "a body has more than 4 children");
                if (nc < 4) packed = (packed & ~(0xffu << (8 * nc))) | ((uint32_t)c << (8 * nc));
                nc++;
            }
        bchild[b] = (int)packed;
    }
    ch_start[nb] = (int)ch_list.size();
    for (int b = nb - 1; b >= 1; b--) bsize[P(b)] += bsize[b];
    for (int b = 1; b < nb; b++)       // subtrees must be contiguous: bodies listed depth first
        for (int c = b + 1; c < b + bsize[b]; c++) {
            int a = c;
            while (a > b) a = P(a);
            if (a != b) return fail(RB_EINVAL, "bodies must be listed in depth-first order");
        }
    // dof heights (0 for dofs without child dofs) and their level lists
    std::vector<int> height(nv, 0);
    for (int i = nv - 1; i >= 0; i--)
        if (dof_parent[i] >= 0) height[dof_parent[i]] = std::max(height[dof_parent[i]], height[i] + 1);
    int nhlevel = 0;
    for (int i = 0; i < nv; i++) nhlevel = std::max(nhlevel, height[i] + 1);
    std::vector<int> hl_start(nhlevel + 1, 0), hl_dof;
    int maxpiv = 0;
    for (int h = 0; h < nhlevel; h++) {
        hl_start[h] = (int)hl_dof.size();
        for (int i = nv - 1; i >= 0; i--)
            if (height[i] == h) hl_dof.push_back(i);
        maxpiv = std::max(maxpiv, (int)hl_dof.size() - hl_start[h]);
    }
    hl_start[nhlevel] = (int)hl_dof.size();
    std::vector<uint64_t> dmask(nv, 0);
    for (int i = 0; i < nv; i++)
        for (int c = desc_start[i]; c < desc_start[i + 1]; c++) dmask[i] |= 1ull << desc_list[c];
    std::vector<uint64_t> cmask(nb, 0);
    for (int b = 1; b < nb; b++) {
        if (blast[b] < 0) continue;
        for (int t = 0; t < bdepth[b]; t++) cmask[b] |= 1ull << anc[(size_t)blast[b] * tmaxd + t];
    }
    // actuators grouped by dof
    std::vector<std::vector<int>> by_dof(nv);
    std::vector<int> atype(nu), aqadr(nu);
    std::vector<double> akp(nu), akd(nu), agear(nu);
    for (int u = 0; u < nu; u++) {
        int j = d->act_joint[u];
        if (j < 0 || j >= nj) return fail(RB_EINVAL, "actuator on an invalid joint");
        if (jtype[j] != RB_JNT_HINGE) return fail(RB_EINVAL, "actuators drive hinge joints only");
        if (d->act_type[u] != RB_ACT_POSITION && d->act_type[u] != RB_ACT_MOTOR)
            return fail(RB_EINVAL, "unknown actuator type");
        atype[u] = d->act_type[u];
        aqadr[u] = jq[j];
        akp[u] = d->act_kp[u];
        akd[u] = d->act_kd[u];
        agear[u] = d->act_gear[u];
        by_dof[jd[j]].push_back(u);
    }
    std::vector<int> act_start(nv + 1, 0), act_list;
    for (int i = 0; i < nv; i++) {
        act_start[i] = (int)act_list.size();
        for (int u : by_dof[i]) act_list.push_back(u);
    }
    act_start[nv] = (int)act_list.size();
    // collision pairs
    std::vector<int> movable(nb, 0);
    for (int b = 1; b < nb; b++) movable[b] = movable[P(b)] || bjnt[b] >= 0;
    for (int g = 0; g < ng; g++) {
        int t = d->geom_type[g], b = d->geom_body[g];
        if (t < RB_GEOM_PLANE || t > RB_GEOM_HFIELD) return fail(RB_EINVAL, "unknown geom type");
        if (t == RB_GEOM_HFIELD) {
            if (movable[b]) return fail(RB_EINVAL, "a height field must be on a static body");
            if (!(d->geom_size[3 * g] > 0 && d->geom_size[3 * g + 1] > 0))
                return fail(RB_EINVAL, "height field extents must be positive");
            if (d->hfield_nrow < 2 || d->hfield_ncol < 2 || !d->hfield_data)
                return fail(RB_EINVAL, "height field geom without a grid (hfield_nrow, hfield_ncol >= 2, data)");
            for (long k = 0; k < (long)d->hfield_nrow * d->hfield_ncol; k++)
                if (!std::isfinite(d->hfield_data[k])) return fail(RB_EINVAL, "height field heights must be finite");
        }
        if (d->geom_condim && d->geom_condim[g] != 1 && d->geom_condim[g] != 3 && d->geom_condim[g] != 4 &&
            d->geom_condim[g] != 6)
            return fail(RB_EINVAL, "geom condim must be 1, 3, 4 or 6");
        const double fs = d->geom_friction_spin ? d->geom_friction_spin[g] : 0.0;
        const double fr = d->geom_friction_roll ? d->geom_friction_roll[g] : 0.0;
        if (!(fs >= 0 && fr >= 0 && std::isfinite(fs) && std::isfinite(fr)))
            return fail(RB_EINVAL, "torsional and rolling friction must be finite and >= 0");
        if (b < 0 || b >= nb) return fail(RB_EINVAL, "geom on an invalid body");
        if (t == RB_GEOM_PLANE && movable[b]) return fail(RB_EINVAL, "a plane must be on a static body");
        const double* q = d->geom_quat + 4 * g;
        if (std::fabs(std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) - 1) > 1e-6)
            return fail(RB_EINVAL, "geom quaternion is not unit");
    }
    struct Pair { int g1, g2; };
    std::vector<Pair> pairs;
    for (int a = 0; a < ng; a++)
        for (int b = a + 1; b < ng; b++) {
            int ba = d->geom_body[a], bb = d->geom_body[b];
            if (ba == bb) continue;
            if ((P(ba) == bb && bb != 0) || (P(bb) == ba && ba != 0)) continue;
            if (((d->geom_contype[a] & d->geom_conaffinity[b]) | (d->geom_contype[b] & d->geom_conaffinity[a])) == 0)
                continue;
            if (!movable[ba] && !movable[bb]) continue;
            int g1 = a, g2 = b;
            if (d->geom_type[g2] < d->geom_type[g1]) std::swap(g1, g2);
            // a height field takes the place of g1, as a plane does
            if (d->geom_type[g2] == RB_GEOM_HFIELD) std::swap(g1, g2);
            bool hfield_pair = d->geom_type[g1] == RB_GEOM_HFIELD && d->geom_type[g2] >= RB_GEOM_SPHERE &&
                               d->geom_type[g2] <= RB_GEOM_BOX;
            bool plane_pair = d->geom_type[g1] == RB_GEOM_PLANE && d->geom_type[g2] != RB_GEOM_PLANE &&
                              d->geom_type[g2] != RB_GEOM_HFIELD;
            bool box_pair = d->geom_type[g1] == RB_GEOM_BOX && d->geom_type[g2] == RB_GEOM_BOX;
            bool sphere_box = d->geom_type[g1] == RB_GEOM_SPHERE && d->geom_type[g2] == RB_GEOM_BOX;
            bool capsule_box = d->geom_type[g1] == RB_GEOM_CAPSULE && d->geom_type[g2] == RB_GEOM_BOX;
            auto round = [&](int g) { return d->geom_type[g] == RB_GEOM_SPHERE || d->geom_type[g] == RB_GEOM_CAPSULE; };
            bool round_pair = round(g1) && round(g2);
            if (!plane_pair && !box_pair && !sphere_box && !capsule_box && !hfield_pair && !round_pair)
                return fail(RB_EINVAL, "unsupported collision pair (only plane or height field vs sphere, capsule, "
                                       "box; box vs box; sphere or capsule vs box; sphere or capsule vs sphere or capsule)");
            pairs.push_back({g1, g2});
        }
    std::sort(pairs.begin(), pairs.end(), [](const Pair& x, const Pair& y) {
        return x.g1 != y.g1 ? x.g1 < y.g1 : x.g2 < y.g2;
    });
    int npair = (int)pairs.size();
    if (npair > RB_MAX_PAIR) return fail(RB_EINVAL, "more than 128 collision pairs");
    std::vector<int> pg1(npair), pg2(npair), ptype(npair), pbody(npair), pcap(npair), pslot(npair, -1);
    std::vector<int> pbody1(npair, 0);   // the second moving body of a pair (0: the other is static)
    int nmm = 0;                         // pairs of two moving bodies
    int nbb = 0;
    std::vector<double> psig(npair), pmu(npair), pmar(npair);
    std::vector<int> pfric0(npair, 0), pxr(npair, 0), pellx(npair, 0);
    const bool elliptic = d->cone == RB_CONE_ELLIPTIC;
    std::vector<double> pmus(npair, 0.0), pmur(npair, 0.0);
    int nxmax = 0;
    int maxcon = 0;
    for (int k = 0; k < npair; k++) {
        int g1 = pairs[k].g1, g2 = pairs[k].g2;
        pg1[k] = g1;
        pg2[k] = g2;
        const bool g2box = d->geom_type[g2] == RB_GEOM_BOX;
        ptype[k] = d->geom_type[g1] == RB_GEOM_BOX                ? RB_PAIR_BOXBOX
                   : (d->geom_type[g1] == RB_GEOM_SPHERE && g2box)  ? RB_PAIR_SPHEREBOX
                   : (d->geom_type[g1] == RB_GEOM_CAPSULE && g2box) ? RB_PAIR_CAPSULEBOX
                   : (d->geom_type[g1] == RB_GEOM_SPHERE || d->geom_type[g1] == RB_GEOM_CAPSULE) ? RB_PAIR_ROUND
                   : d->geom_type[g1] == RB_GEOM_HFIELD  ? RB_PAIR_HFIELD + d->geom_type[g2]
                                                         : d->geom_type[g2];
        if (ptype[k] == RB_PAIR_BOXBOX) pslot[k] = nbb++;
        bool mov2 = movable[d->geom_body[g2]];
        pbody[k] = mov2 ? d->geom_body[g2] : d->geom_body[g1];
        psig[k] = mov2 ? 1.0 : -1.0;
        if (mov2 && movable[d->geom_body[g1]]) {
            // both bodies move (box-box, sphere or capsule against box: planes and height
            // fields are static): rows of the relative velocity, g2's body minus g1's
            pbody1[k] = d->geom_body[g1];
            nmm++;
        }
        pmu[k] = std::max(d->geom_friction[g1], d->geom_friction[g2]);
        pmar[k] = std::max(d->geom_margin[g1], d->geom_margin[g2]);
        if (d->geom_condim) {
            // condim 4 adds the torsional row pair, 6 the two rolling pairs too
            const int cd = std::max(d->geom_condim[g1], d->geom_condim[g2]);
            pfric0[k] = cd == 1;
            // pyramidal: extra generic rows; elliptic: the spin row (condim 4) and the rolling
            // rows (6) join the contact's cone in its own lane
            pxr[k] = elliptic ? 0 : (cd == 4 ? 2 : (cd == 6 ? 6 : 0));
            pellx[k] = elliptic ? (cd == 4 ? 1 : (cd == 6 ? 3 : 0)) : 0;
            auto fmax = [&](const double* f, double dflt) { return f ? std::max(f[g1], f[g2]) : dflt; };
            pmus[k] = fmax(d->geom_friction_spin, 0.005);
            pmur[k] = fmax(d->geom_friction_roll, 0.0001);
        }
        const int shape = ptype[k] >= RB_PAIR_HFIELD ? ptype[k] - RB_PAIR_HFIELD : ptype[k];
        pcap[k] = (shape == RB_GEOM_SPHERE || shape == RB_PAIR_SPHEREBOX || shape == RB_PAIR_ROUND) ? 1
                  : (shape == RB_GEOM_CAPSULE || shape == RB_PAIR_CAPSULEBOX) ? 2
                                                                               : 8;
        maxcon += pcap[k];
        nxmax += pcap[k] * pxr[k];
    }
    // options
    if (!(d->timestep > 0) || d->nsubsteps < 1 || d->iterations < 0) return fail(RB_EINVAL, "bad options");
    if (d->cone != RB_CONE_PYRAMIDAL && d->cone != RB_CONE_ELLIPTIC)
        return fail(RB_EINVAL, "cone must be RB_CONE_PYRAMIDAL or RB_CONE_ELLIPTIC");
    const double impratio = d->impratio == 0 ? 1.0 : d->impratio;
    if (!(impratio > 0) || !std::isfinite(impratio)) return fail(RB_EINVAL, "impratio must be positive");
    if (nmm > 0) {
        if (d->cone == RB_CONE_ELLIPTIC)
            return fail(RB_EINVAL, "contacts between two moving bodies take pyramidal cones");
        for (int k = 0; k < npair; k++)
            if (pbody1[k] > 0 && pxr[k] > 0)
                return fail(RB_EINVAL, "contacts between two moving bodies take condim 1 or 3");
    }
    double dmax = std::min(std::max(d->solimp[1], 1e-4), 0.9999);
    double tc = std::max(d->solref[0], 2 * d->timestep), zeta = d->solref[1];
    // mean diagonal inertia at the reference configuration: composite inertias in double
    double meaninertia;
    {
        std::vector<double> xp(3 * nb, 0), xq(4 * nb, 0), R(9 * nb, 0);
        xq[0] = 1;
        qmat_d(&xq[0], &R[0]);
        for (int b = 1; b < nb; b++) {
            int p = P(b);
            double off[3];
            mv_d(&R[9 * p], d->body_pos + 3 * b, off);
            for (int i = 0; i < 3; i++) xp[3 * b + i] = xp[3 * p + i] + off[i];
            qmul_d(&xq[4 * p], d->body_quat + 4 * b, &xq[4 * b]);
            qmat_d(&xq[4 * b], &R[9 * b]);
        }
        // composite mass, first moment and rotational inertia about the world origin
        std::vector<double> cm(nb, 0), ch(3 * nb, 0), cI(9 * nb, 0);
        for (int b = nb - 1; b >= 1; b--) {
            double Ri[9], RR[9], c[3];
            qmat_d(d->body_iquat + 4 * b, Ri);
            for (int i = 0; i < 3; i++)
                for (int k = 0; k < 3; k++)
                    RR[3 * i + k] = R[9 * b + 3 * i] * Ri[k] + R[9 * b + 3 * i + 1] * Ri[3 + k] + R[9 * b + 3 * i + 2] * Ri[6 + k];
            mv_d(&R[9 * b], d->body_ipos + 3 * b, c);
            for (int i = 0; i < 3; i++) c[i] += xp[3 * b + i];
            double m = d->body_mass[b];
            cm[b] += m;
            for (int i = 0; i < 3; i++) ch[3 * b + i] += m * c[i];
            double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            for (int i = 0; i < 3; i++)
                for (int k = 0; k < 3; k++) {
                    double Ic = 0;
                    for (int l = 0; l < 3; l++) Ic += RR[3 * i + l] * d->body_inertia[3 * b + l] * RR[3 * k + l];
                    cI[9 * b + 3 * i + k] += Ic + m * ((i == k) * cc - c[i] * c[k]);
                }
            int p = P(b);
            cm[p] += cm[b];
            for (int i = 0; i < 3; i++) ch[3 * p + i] += ch[3 * b + i];
            for (int i = 0; i < 9; i++) cI[9 * p + i] += cI[9 * b + i];
        }
        double tr = 0;
        for (int j = 0; j < nj; j++) {
            int b = jbody[j];
            const double* I = &cI[9 * b];
            const double* h = &ch[3 * b];
            if (jtype[j] == RB_JNT_FREE) {
                tr += 3 * cm[b];
                // body axes through the body origin x: I_x = I_O - m(|x|^2 - x x') - cross terms
                const double* x = &xp[3 * b];
                for (int a = 0; a < 3; a++) {
                    double u[3] = {R[9 * b + a], R[9 * b + 3 + a], R[9 * b + 6 + a]};
                    double Iu[3];
                    mv_d(I, u, Iu);
                    double val = u[0] * Iu[0] + u[1] * Iu[1] + u[2] * Iu[2];
                    // shift the axis from the origin to x: + m |u x x|^2 - 2 (u x x).(u x h)
                    double ux[3], uh[3];
                    cross_d(u, x, ux);
                    cross_d(u, h, uh);
                    val += cm[b] * (ux[0] * ux[0] + ux[1] * ux[1] + ux[2] * ux[2]) -
                           2 * (ux[0] * uh[0] + ux[1] * uh[1] + ux[2] * uh[2]);
                    tr += val;
                }
            } else {
                double u[3], o[3], Iu[3];
                mv_d(&R[9 * b], d->jnt_axis + 3 * j, u);
                double nrm = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                for (int i = 0; i < 3; i++) u[i] /= nrm;
                mv_d(&R[9 * b], d->jnt_pos + 3 * j, o);
                for (int i = 0; i < 3; i++) o[i] += xp[3 * b + i];
                mv_d(I, u, Iu);
                double val = u[0] * Iu[0] + u[1] * Iu[1] + u[2] * Iu[2];
                double uo[3], uh[3];
                cross_d(u, o, uo);
                cross_d(u, h, uh);
                val += cm[b] * (uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2]) -
                       2 * (uo[0] * uh[0] + uo[1] * uh[1] + uo[2] * uh[2]);
                tr += val + d->jnt_armature[j];
            }
        }
        meaninertia = tr / nv;
    }
    // body tables
    std::vector<int> bjt(nb, -1), bq(nb, 0), bd(nb, 0);
    std::vector<double> jpos(3 * nb, 0), jax(3 * nb, 0), arm(nv, 0);
    for (int b = 1; b < nb; b++) {
        int j = bjnt[b];
        if (j < 0) continue;
        bjt[b] = jtype[j];
        bq[b] = jq[j];
        bd[b] = jd[j];
        if (jtype[j] == RB_JNT_HINGE) {
            const double* ax = d->jnt_axis + 3 * j;
            double n = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
            for (int i = 0; i < 3; i++) {
                jax[3 * b + i] = ax[i] / n;
                jpos[3 * b + i] = d->jnt_pos[3 * j + i];
            }
            arm[jd[j]] = d->jnt_armature[j];
        }
    }
    // joint damping per dof (hinges only)
    std::vector<double> ddamp(nv, 0.0);
    int ndamp = 0;
    for (int j = 0; j < nj && d->jnt_damping; j++)
        if (jtype[j] == RB_JNT_HINGE && d->jnt_damping[j] > 0) {
            ddamp[jd[j]] = d->jnt_damping[j];
            ndamp++;
        }
    // joint limits per dof: the hinge's qpos index (-1 when unlimited) and its bounds
    std::vector<int> limq(nv, -1);
    std::vector<double> limlo(nv, 0.0), limhi(nv, 0.0);
    int nlim = 0;
    for (int j = 0; j < nj && d->jnt_range; j++)
        if (jtype[j] == RB_JNT_HINGE && d->jnt_range[2 * j] < d->jnt_range[2 * j + 1]) {
            limq[jd[j]] = jq[j];
            limlo[jd[j]] = d->jnt_range[2 * j];
            limhi[jd[j]] = d->jnt_range[2 * j + 1];
            nlim++;
        }
    // equality constraints: per constraint body, anchor, target point and orientation; per row
    // its constraint and axis (k < 3 translational, 3..5 rotational)
    if (d->neq < 0 || (d->neq > 0 && (!d->eq_type || !d->eq_body || !d->eq_anchor || !d->eq_target)))
        return fail(RB_EINVAL, "equality constraints missing");
    std::vector<int> eqb, eqr_q, eqr_k;
    std::vector<double> eqa, eqp, eqm;
    for (int q = 0; q < d->neq; q++) {
        const int t = d->eq_type[q], b = d->eq_body[q];
        if (t != RB_EQ_CONNECT && t != RB_EQ_WELD) return fail(RB_EINVAL, "unknown equality type");
        if (b <= 0 || b >= nb || !movable[b]) return fail(RB_EINVAL, "an equality constraint needs a moving body");
        if (!finite(d->eq_anchor + 3 * q, 3) || !finite(d->eq_target + 7 * q, 7))
            return fail(RB_EINVAL, "equality constraint values must be finite");
        const double* tq = d->eq_target + 7 * q + 3;
        const double qn = std::sqrt(tq[0] * tq[0] + tq[1] * tq[1] + tq[2] * tq[2] + tq[3] * tq[3]);
        if (t == RB_EQ_WELD && std::fabs(qn - 1) > 1e-6) return fail(RB_EINVAL, "weld target quaternion is not unit");
        eqb.push_back(b);
        for (int i = 0; i < 3; i++) {
            eqa.push_back(d->eq_anchor[3 * q + i]);
            eqp.push_back(d->eq_target[7 * q + i]);
        }
        double Rt[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (t == RB_EQ_WELD) qmat_d(tq, Rt);
        eqm.insert(eqm.end(), Rt, Rt + 9);
        for (int k = 0; k < (t == RB_EQ_WELD ? 6 : 3); k++) {
            eqr_q.push_back(q);
            eqr_k.push_back(k);
        }
    }
    const int neqrow = (int)eqr_q.size();
    // generic rows, one lane each: equality rows and the torsional / rolling rows that the
    // contacts can produce
    nxmax = std::min(nxmax, 6 * RB_MAX_CON);
    if (neqrow + nxmax > RB_MAX_GROW)
        return fail(RB_EINVAL, "more than 64 equality and torsional / rolling friction rows (condim 4 and 6 "
                               "pairs count 2 and 6 rows for every contact they can produce)");

    // ---- upload
    Blob B;
    DevModel& m = M->dm;
    std::memset(&m, 0, sizeof m);
    struct Fix { size_t off; const void** field; };
    std::vector<Fix> fx;
    auto I = [&](const std::vector<int>& v, const int** f) { fx.push_back({B.add_i(v), (const void**)f}); };
    auto F = [&](const std::vector<double>& v, const float** f) { fx.push_back({B.add_f(v), (const void**)f}); };
    std::vector<int> parent(nb);
    for (int b = 0; b < nb; b++) parent[b] = b == 0 ? -1 : P(b);
    I(parent, &m.body_parent); I(bjt, &m.body_jtype); I(bq, &m.body_qadr); I(bd, &m.body_dadr);
    I(blast, &m.body_lastdof); I(bdepth, &m.body_depth); I(blevel, &m.body_level);
    F(std::vector<double>(d->body_pos, d->body_pos + 3 * nb), &m.body_pos);
    F(std::vector<double>(d->body_quat, d->body_quat + 4 * nb), &m.body_quat);
    F(std::vector<double>(d->body_ipos, d->body_ipos + 3 * nb), &m.body_ipos);
    F(std::vector<double>(d->body_iquat, d->body_iquat + 4 * nb), &m.body_iquat);
    F(std::vector<double>(d->body_mass, d->body_mass + nb), &m.body_mass);
    F(std::vector<double>(d->body_inertia, d->body_inertia + 3 * nb), &m.body_inertia);
    F(jpos, &m.body_jpos); F(jax, &m.body_jaxis);
    size_t off_mask = B.add_u64(cmask);
    size_t off_dmask = B.add_u64(dmask);
    I(lv_start, &m.level_start); I(lv_body, &m.level_body); I(ch_start, &m.child_start); I(ch_list, &m.child_list);
    I(dof_body, &m.dof_body); I(dof_depth, &m.dof_depth); I(rowadr, &m.dof_rowadr); I(anc, &m.dof_anc);
    I(desc_start, &m.desc_start); I(desc_list, &m.desc_list); I(dl_start, &m.dlevel_start); I(dl_dof, &m.dlevel_dof);
    I(height, &m.dof_height); I(hl_start, &m.hlevel_start); I(hl_dof, &m.hlevel_dof); I(bsize, &m.body_size); I(bchild, &m.body_children);
    F(arm, &m.dof_armature);
    I(limq, &m.dof_limq); F(limlo, &m.dof_limlo); F(limhi, &m.dof_limhi); F(ddamp, &m.dof_damping);
    I(act_start, &m.act_start); I(act_list, &m.act_list); I(atype, &m.act_type); I(aqadr, &m.act_qadr);
    F(akp, &m.act_kp); F(akd, &m.act_kd); F(agear, &m.act_gear);
    I(jtype, &m.jnt_type); I(jq, &m.jnt_qadr); I(jd, &m.jnt_dadr);
    I(pg1, &m.pair_g1); I(pg2, &m.pair_g2); I(ptype, &m.pair_type); I(pbody, &m.pair_body); I(pcap, &m.pair_cap);
    if (nmm > 0) I(pbody1, &m.pair_body1);
    I(pslot, &m.pair_slot);
    F(psig, &m.pair_sigma); F(pmu, &m.pair_mu); F(pmar, &m.pair_margin); I(pfric0, &m.pair_frictionless);
    I(std::vector<int>(d->geom_body, d->geom_body + ng), &m.geom_body);
    I(std::vector<int>(d->geom_type, d->geom_type + ng), &m.geom_type);
    F(std::vector<double>(d->geom_pos, d->geom_pos + 3 * ng), &m.geom_pos);
    F(std::vector<double>(d->geom_quat, d->geom_quat + 4 * ng), &m.geom_quat);
    F(std::vector<double>(d->geom_size, d->geom_size + 3 * ng), &m.geom_size);
    if (nxmax > 0 || elliptic) {
        I(pxr, &m.pair_xrows); F(pmus, &m.pair_mu_spin); F(pmur, &m.pair_mu_roll); I(pellx, &m.pair_ellrows);
    }
    if (neqrow > 0) {
        I(eqb, &m.eq_body); F(eqa, &m.eq_anchor); F(eqp, &m.eq_tpos); F(eqm, &m.eq_tmat);
        I(eqr_q, &m.eqrow_eq); I(eqr_k, &m.eqrow_k);
    }
    const bool has_hf = std::count(d->geom_type, d->geom_type + ng, RB_GEOM_HFIELD) > 0;
    if (has_hf) {
        F(std::vector<double>(d->hfield_data, d->hfield_data + (size_t)d->hfield_nrow * d->hfield_ncol), &m.hf_data);
        m.hf_nrow = d->hfield_nrow;
        m.hf_ncol = d->hfield_ncol;
    }
    void* dev = nullptr;
    size_t bytes = B.words.size() * 4;
    hipError_t e = hipMalloc(&dev, bytes);
    if (e != hipSuccess) return fail(RB_ENOMEM, std::string("hipMalloc(model): ") + hipGetErrorString(e));
    e = hipMemcpy(dev, B.words.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "hipMemcpy(model)");
    }
    char* base = (char*)dev;
    for (auto& f : fx) *f.field = base + 4 * f.off;
    m.body_chainmask = (const uint64_t*)(base + 4 * off_mask);
    m.dof_descmask = (const uint64_t*)(base + 4 * off_dmask);
    // sizes and options
    m.nbody = nb; m.nv = nv; m.nq = nq; m.nu = nu; m.njnt = nj; m.npair = npair; m.nbb = nbb; m.ngeom = ng;
    m.maxd = tmaxd; m.nblevel = nblevel; m.ndlevel = maxd; m.nhlevel = nhlevel; m.maxpiv = maxpiv; m.K = d->nsubsteps; m.maxiter = d->iterations;
    m.fr_pw = d->friction_per_world != 0; m.ms_pw = d->mass_scale_per_world != 0; m.nM = nM;
    m.nlim = nlim;
    m.ndamp = ndamp;
    m.neq = d->neq; m.neqrow = neqrow; m.nxmax = nxmax;
    m.cone = d->cone == RB_CONE_ELLIPTIC && npair > 0 ? 1 : 0;
    m.impratio = (float)impratio;
    m.rsqrt_impratio = (float)(1.0 / std::sqrt(impratio));
    // level 2: equality rows, torsional / rolling rows, elliptic cones up to condim 4; level 1:
    // the rest; level 3: pairs of two moving bodies (a dense Newton Hessian); level 4: elliptic
    // cones with condim 6 (the rolling rows)
    bool ell6 = false;
    for (int k = 0; k < npair; k++) ell6 = ell6 || pellx[k] == 3;
    const int ext2 = nmm > 0 ? 3 : (ell6 ? 4 : ((neqrow > 0 || nxmax > 0 || m.cone) ? 2 : 0));
    m.nmm = nmm;
    m.ext = ext2 ? ext2 : (nbb > 0 || nlim > 0 || ndamp > 0 || npair > RB_WAVE ||
             std::count(ptype.begin(), ptype.end(), RB_PAIR_SPHEREBOX) > 0 ||
             std::count(ptype.begin(), ptype.end(), RB_PAIR_CAPSULEBOX) > 0 ||
             std::count(ptype.begin(), ptype.end(), RB_PAIR_ROUND) > 0 ||
             std::count_if(ptype.begin(), ptype.end(), [](int t) { return t >= RB_PAIR_HFIELD; }) > 0 ||
             std::count(pfric0.begin(), pfric0.end(), 1) > 0) ? 1 : 0;
    m.dt = (float)d->timestep;
    for (int i = 0; i < 3; i++) m.grav[i] = (float)d->gravity[i];
    m.tol_scale = (float)(d->tolerance * meaninertia * nv);
    m.bref = (float)(2.0 / (dmax * tc));
    m.kref = (float)(1.0 / (dmax * dmax * tc * tc * zeta * zeta));
    m.dmin = (float)d->solimp[0]; m.dmax = (float)d->solimp[1]; m.width = (float)d->solimp[2];
    m.mid = (float)d->solimp[3]; m.power = (float)d->solimp[4];
    // LDS layout, 4-float aligned sections
    int o = 0;
    auto sec = [&](int nfl) { int r = o; o += (nfl + 3) & ~3; return r; };
    m.o_q = sec(nq); m.o_v = sec(nv); m.o_ctrl = sec(nu); m.o_aws = sec(nv); m.o_mscale = sec(nb);
    m.o_xpos = sec(3 * nb);
    // sections that are dead at the same time share space (world counts per CU depend on it):
    // the Newton vectors g, p, Mp, tmp (and, with joint limits, the limit rows' signed D and
    // residual) live in the rotation matrices' space (dead from the end of collision to the next
    // substep's kinematics); the bias pass's body forces in M's (consumed before M's rows are
    // written); the composite inertias in M's factor's (dead once M is built, before it is
    // factored)
    const int r4nv = (nv + 3) & ~3;
    m.o_xmat = sec(std::max(9 * nb, (nlim > 0 ? 6 : 4) * r4nv));
    m.o_g = m.o_xmat; m.o_p = m.o_g + r4nv; m.o_Mp = m.o_p + r4nv; m.o_tmp = m.o_Mp + r4nv;
    m.o_lD = m.o_tmp + r4nv; m.o_ljar = m.o_lD + r4nv;
    m.o_cinert = sec(10 * nb); m.o_cdof = sec(6 * nv); m.o_cvel = sec(6 * nb); m.o_bvec = sec(6 * nb);
    m.o_tau = sec(nv); m.o_bias = sec(nv); m.o_a0 = sec(nv); m.o_a = sec(nv); m.o_Ma = sec(nv);
    m.o_M = sec(std::max(nM, 6 * nb)); m.o_bvec2 = m.o_M;
    m.o_H = sec(std::max(nM, 10 * nb)); m.o_crb = m.o_H;
    m.o_piv = o;
    layout_tail(m, tmaxd);
    m.ncap = std::min(maxcon, RB_MAX_CON);
    M->blob = dev;
    M->maxcon_static = maxcon;
    M->meaninertia = meaninertia;
    M->nv_ = nv; M->nq_ = nq; M->nu_ = nu; M->nbody_ = nb; M->ngeom_ = ng;
    (void)hipGetDevice(&M->device);
    return RB_OK;
}

}  // namespace

int rb_record_error(int code, const char* msg) { return fail(code, msg); }

// ====================================================================================== ABI
// ---------------------------------------------------------------------------------------
// the fixed per-device array of rb_step_noalloc
// ---------------------------------------------------------------------------------------
// One array per device, held until the process ends.  In host code its name stands for a
// host-side symbol, not a device address: the device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is used.
static __device__ __align__(256) float scratch[RB_NOALLOC_MAX_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array, looked up on first use on the device.
int scratch_address(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RB_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RB_OK;
}
}  // namespace


extern "C" {

const char* rb_last_error(void) { return g_err.c_str(); }

int rb_model_create(const rb_model_desc* desc, rb_model** out) {
    if (!desc || !out) return fail(RB_EINVAL, "null argument");
    *out = nullptr;
    rb_model* m = new rb_model();
    int rc = compile_model(desc, m);
    if (rc != RB_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return RB_OK;
}

void rb_model_destroy(rb_model* m) {
    if (!m) return;
    if (m->blob) (void)hipFree(m->blob);
    delete m;
}

int rb_model_info_get(const rb_model* m, rb_model_info* out) {
    if (!m || !out) return fail(RB_EINVAL, "null argument");
    out->nq = m->nq_; out->nv = m->nv_; out->nu = m->nu_; out->nbody = m->nbody_; out->ngeom = m->ngeom_;
    out->npair = m->dm.npair; out->maxcon = m->maxcon_static; out->max_depth = m->dm.ndlevel;
    out->lds_bytes = m->dm.lds_floats * 4; out->meaninertia = m->meaninertia;
    // a batch slot: warm start [nv], status, friction, mass scales [nbody] (rb_batch_create)
    out->bytes_per_world = 4 * (m->nv_ + 2 + m->nbody_);
    return RB_OK;
}

int rb_batch_create(const rb_model* model, int32_t capacity, int32_t contact_capacity, rb_batch** out) {
    if (!model || !out || capacity <= 0) return fail(RB_EINVAL, "bad arguments to rb_batch_create");
    if (contact_capacity > RB_MAX_CON) return fail(RB_EINVAL, "contact capacity above 64");
    *out = nullptr;
    rb_batch* b = new rb_batch();
    b->model = model;
    b->capacity = capacity;
    b->dm = model->dm;
    int cap = contact_capacity > 0 ? contact_capacity : std::min(model->maxcon_static, RB_MAX_CON);
    b->dm.ncap = std::max(cap, 1);
    const int nv = model->nv_, nb = model->nbody_;
    size_t s_ws = (size_t)capacity * nv * 4, s_st = (size_t)capacity * 4, s_fr = (size_t)capacity * 4,
           s_ms = (size_t)capacity * nb * 4;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t total = al(s_ws) + al(s_st) + al(s_fr) + al(s_ms);
    hipError_t e = hipMalloc(&b->mem, total);
    if (e != hipSuccess) {
        delete b;
        return fail(RB_ENOMEM, std::string("hipMalloc(batch): ") + hipGetErrorString(e));
    }
    char* p = (char*)b->mem;
    b->W.qacc_ws = (float*)p; p += al(s_ws);
    b->W.status = (uint32_t*)p; p += al(s_st);
    b->W.friction = (float*)p; p += al(s_fr);
    b->W.mass_scale = (float*)p;
    e = hipMemset(b->W.qacc_ws, 0, s_ws);
    if (e == hipSuccess) e = hipMemset(b->W.status, 0, s_st);
    if (e == hipSuccess) e = rb_launch_fill(b->W.friction, 1.0f, (size_t)capacity, nullptr);
    if (e == hipSuccess) e = rb_launch_fill(b->W.mass_scale, 1.0f, (size_t)capacity * nb, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(b->mem);
        delete b;
        return hip_fail(e, "batch init");
    }
    *out = b;
    return RB_OK;
}

void rb_batch_destroy(rb_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->mem) (void)hipFree(b->mem);
    for (void* f : b->field_mem)
        if (f) (void)hipFree(f);
    delete b;
}

int32_t rb_batch_contact_capacity(const rb_batch* b) { return b ? b->dm.ncap : 0; }

// Expand a model field to one value per world slot: a [capacity, k] array initialised with the
// model's values in every slot.  Returns the array (already expanded: the same one).
static int expand_field(rb_batch* b, int field, float** out) {
    const DevModel& m = b->dm;
    const int idx = field - RB_PARAM_GEOM_SIZE;
    float** slot = idx == 0 ? &b->W.geom_size : idx == 1 ? &b->W.body_pos : idx == 2 ? &b->W.act_kp : &b->W.act_kd;
    const float* src = idx == 0 ? m.geom_size : idx == 1 ? m.body_pos : idx == 2 ? m.act_kp : m.act_kd;
    const size_t k = idx == 0 ? 3 * (size_t)m.ngeom : idx == 1 ? 3 * (size_t)m.nbody : (size_t)m.nu;
    if (!*slot) {
        if (k == 0) return fail(RB_EINVAL, "the model has no values of this field");
        void* mem = nullptr;
        hipError_t e = hipMalloc(&mem, k * b->capacity * sizeof(float));
        if (e != hipSuccess) return fail(RB_ENOMEM, std::string("hipMalloc(field): ") + hipGetErrorString(e));
        e = rb_launch_tile(static_cast<float*>(mem), src, k, (size_t)b->capacity, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return hip_fail(e, "expanding a model field");
        }
        b->field_mem[idx] = mem;
        *slot = static_cast<float*>(mem);
        b->version++;
    }
    *out = *slot;
    return RB_OK;
}

int rb_batch_set_params_at(rb_batch* b, int32_t field, int32_t first, int32_t n, const float* vals, void* stream) {
    if (!b || n < 0 || first < 0 || first > b->capacity || n > b->capacity - first || (n > 0 && !vals))
        return fail(RB_EINVAL, "bad arguments to rb_batch_set_params");
    hipError_t e = hipSuccess;
    if (field >= RB_PARAM_GEOM_SIZE && field <= RB_PARAM_ACT_KD) {
        float* dst = nullptr;
        int rc = expand_field(b, field, &dst);
        if (rc != RB_OK) return rc;
        const DevModel& m = b->dm;
        const size_t k = field == RB_PARAM_GEOM_SIZE ? 3 * (size_t)m.ngeom
                         : field == RB_PARAM_BODY_POS ? 3 * (size_t)m.nbody : (size_t)m.nu;
        if (n) e = hipMemcpyAsync(dst + (size_t)first * k, vals, (size_t)n * k * 4, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    } else if (field == RB_PARAM_FRICTION) {
        if (!b->dm.fr_pw) return fail(RB_EINVAL, "model does not have per-world friction");
        if (n) e = hipMemcpyAsync(b->W.friction + first, vals, (size_t)n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    } else if (field == RB_PARAM_MASS_SCALE) {
        if (!b->dm.ms_pw) return fail(RB_EINVAL, "model does not have per-world mass scale");
        const size_t nb = (size_t)b->dm.nbody;
        if (n) e = hipMemcpyAsync(b->W.mass_scale + (size_t)first * nb, vals, (size_t)n * nb * 4, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    } else {
        return fail(RB_EINVAL, "unknown parameter field");
    }
    return e == hipSuccess ? RB_OK : hip_fail(e, "rb_batch_set_params");
}

int rb_batch_set_params(rb_batch* b, int32_t field, int32_t n, const float* vals, void* stream) {
    if (!vals && n > 0) return fail(RB_EINVAL, "bad arguments to rb_batch_set_params");
    return rb_batch_set_params_at(b, field, 0, n, vals, stream);
}

int rb_batch_set_waves(rb_batch* b, int32_t waves) {
    if (!b || (waves != 0 && waves != 3 && waves != 4)) return fail(RB_EINVAL, "waves must be 0, 3 or 4");
    b->waves = waves;
    return RB_OK;
}

int rb_world_reset(rb_batch* b, const int32_t* ids, int32_t n, const float* qacc_ws, void* stream) {
    if (!b || n < 0 || (n > 0 && !ids)) return fail(RB_EINVAL, "bad arguments to rb_world_reset");
    if (n == 0) return RB_OK;
    hipError_t e = rb_launch_reset(b->dm.nv, ids, n, qacc_ws, b->W, b->capacity, (hipStream_t)stream);
    return e == hipSuccess ? RB_OK : hip_fail(e, "rb_world_reset");
}

int rb_get_state(const rb_batch* b, int32_t n, float* ws, uint32_t* st, void* stream) {
    if (!b || n < 0 || n > b->capacity) return fail(RB_EINVAL, "bad arguments to rb_get_state");
    hipError_t e = hipSuccess;
    if (ws && n)
        e = hipMemcpyAsync(ws, b->W.qacc_ws, (size_t)n * b->dm.nv * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e == hipSuccess && st && n)
        e = hipMemcpyAsync(st, b->W.status, (size_t)n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? RB_OK : hip_fail(e, "rb_get_state");
}

// Resident waves per SIMD for a plain launch of n worlds: the batch's setting, or
// automatically 4 when the model's LDS lets 16 worlds share a compute unit, its chain bound is
// at most 16 and n is more than one round of the 3-wave kernel; otherwise 3.
static int auto_waves(const DevModel& m, int setting, int n) {
    if (setting == 3 || m.maxd > 16) return 3;
    if (setting == 4) return 4;
    static int ncu = 0, lds_cu = 0;
    if (ncu == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 3;
        ncu = prop.multiProcessorCount;
        lds_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    }
    const bool lds_ok = (long)m.lds_floats * 4 * 16 <= (long)lds_cu;
    return lds_ok && n > 12 * ncu ? 4 : 3;
}
static int plain_waves(const rb_batch* b, int n) { return auto_waves(b->dm, b->waves, n); }

static int step_impl(rb_batch* b, int32_t n, const float* ctrl, float* qpos, float* qvel, const rb_contacts* c,
                     uint32_t* status, const DevTaps* taps, void* stream) {
    if (!b) return fail(RB_EINVAL, "null batch");
    if (n < 0 || n > b->capacity) return fail(RB_EINVAL, "world count outside the batch capacity");
    if (n == 0) return RB_OK;
    if (!qpos || !qvel) return fail(RB_EINVAL, "qpos and qvel are required");
    if (b->dm.nu > 0 && !ctrl) return fail(RB_EINVAL, "ctrl is required for a model with actuators");
    hipError_t pending = hipGetLastError();
    if (pending != hipSuccess) return hip_fail(pending, "earlier asynchronous error");
    DevContactsOut co{};
    if (c) {
        co.ncon = c->ncon; co.geom = c->geom; co.feature = c->feature; co.dist = c->dist;
        co.pos = c->pos; co.frame = c->frame; co.force = c->force;
    }
    hipError_t e = rb_launch_step(b->dm, n, ctrl, qpos, qvel, b->W, c ? &co : nullptr, status, taps,
                                  plain_waves(b, n), (hipStream_t)stream);
    return e == hipSuccess ? RB_OK : hip_fail(e, "step launch");
}

int rb_step(rb_batch* b, int32_t n, const float* ctrl, float* qpos, float* qvel, const rb_contacts* c,
            uint32_t* status, void* stream) {
    return step_impl(b, n, ctrl, qpos, qvel, c, status, nullptr, stream);
}

int rb_step_taps(rb_batch* b, int32_t n, const float* ctrl, float* qpos, float* qvel, const rb_contacts* c,
                 uint32_t* status, float* M, float* bias, float* a0, float* qacc, float* efc, int32_t* stats,
                 void* stream) {
    DevTaps t{M, bias, a0, qacc, efc, stats};
    return step_impl(b, n, ctrl, qpos, qvel, c, status, &t, stream);
}

// ---------------------------------------------------------------------------------------
// the step without allocation: per-world working state in a fixed device array
// ---------------------------------------------------------------------------------------
int rb_step_noalloc(const rb_model* model, int32_t n, const float* ctrl, float* qpos, float* qvel,
                    const float* friction, const float* mass_scale, const rb_contacts* c, uint32_t* status,
                    void* stream) {
    if (!model) return fail(RB_EINVAL, "null model");
    if (n < 0) return fail(RB_EINVAL, "negative world count");
    if (n == 0) return RB_OK;
    if (!qpos || !qvel) return fail(RB_EINVAL, "qpos and qvel are required");
    if (model->dm.nu > 0 && !ctrl) return fail(RB_EINVAL, "ctrl is required for a model with actuators");
    const size_t nv = (size_t)model->nv_, nb = (size_t)model->nbody_;
    const size_t need = (size_t)n * (nv + 2 + nb);
    if (need > (size_t)RB_NOALLOC_MAX_FLOATS)
        return fail(RB_EINVAL, "rb_step_noalloc: n * (nv + 2 + nbody) = " + std::to_string(need) +
                                   " floats exceeds RB_NOALLOC_MAX_FLOATS (" + std::to_string(RB_NOALLOC_MAX_FLOATS) +
                                   "); use a batch (rb_batch_create) or fewer worlds per call");
    hipError_t pending = hipGetLastError();
    if (pending != hipSuccess) return hip_fail(pending, "earlier asynchronous error");
    float* base = nullptr;
    int rc = scratch_address(&base);
    if (rc != RB_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    // every call starts as a freshly reset batch: zero warm start and status, per-world
    // friction and mass scale 1 unless the caller passes them
    DevWorlds W{};
    W.qacc_ws = base;
    W.status = reinterpret_cast<uint32_t*>(base + (size_t)n * nv);
    float* fr = base + (size_t)n * (nv + 1);
    float* ms = base + (size_t)n * (nv + 2);
    hipError_t e = rb_launch_fill(base, 0.0f, (size_t)n * (nv + 1), s);   // 0.0f is the zero status word too
    W.friction = friction ? const_cast<float*>(friction) : fr;
    W.mass_scale = mass_scale ? const_cast<float*>(mass_scale) : ms;
    if (e == hipSuccess && !friction && model->dm.fr_pw) e = rb_launch_fill(fr, 1.0f, (size_t)n, s);
    if (e == hipSuccess && !mass_scale && model->dm.ms_pw) e = rb_launch_fill(ms, 1.0f, (size_t)n * nb, s);
    if (e != hipSuccess) return hip_fail(e, "rb_step_noalloc: clearing the scratch array");
    DevModel dm = model->dm;
    dm.ncap = std::max(std::min(model->maxcon_static, RB_MAX_CON), 1);   // a batch's default capacity
    DevContactsOut co{};
    if (c) {
        co.ncon = c->ncon; co.geom = c->geom; co.feature = c->feature; co.dist = c->dist;
        co.pos = c->pos; co.frame = c->frame; co.force = c->force;
    }
    e = rb_launch_step(dm, n, ctrl, qpos, qvel, W, c ? &co : nullptr, status, nullptr, auto_waves(dm, 0, n), s);
    return e == hipSuccess ? RB_OK : hip_fail(e, "rb_step_noalloc launch");
}

// ---------------------------------------------------------------------------------------
// mixed-model batching
// ---------------------------------------------------------------------------------------
struct BindRec {
    int n = -1;
    const float* ctrl = nullptr;
    float *qpos = nullptr, *qvel = nullptr;
    DevContactsOut co{};
    bool has_co = false;
    uint32_t* status = nullptr;
    int version = 0;          // the batch's version the argument block was written from
};

struct rb_multi {
    std::vector<rb_batch*> batches;
    std::vector<int> bound_n;
    std::vector<BindRec> bind;
    std::vector<char> args_host;   // nbatch step-argument blocks
    DevModel* d_models = nullptr;
    void* d_args = nullptr;
    int* d_items = nullptr;
    int nitems = 0, grid = 0, maxd = 0, lds_floats = 0;
    int boxbox = 0;                            // highest level of extended code a model needs
    bool scheduled = false;                    // a work list was set (possibly empty)
    int items_cap = 0;                         // capacity of d_items
    int lds_pad = 0;                           // extra LDS floats per workgroup (occupancy cap)
    int occ = 0;                               // requested waves per SIMD (0 automatic)
    int wpg = 1;                               // worlds (waves) per workgroup
    // pinned staging ring for rb_multi_set_items (a slot is reused once its copy is done)
    static constexpr int RING = 4;
    int32_t* stage[RING] = {};
    hipEvent_t stage_ev[RING] = {};
    bool stage_used[RING] = {};
    int stage_cap = 0, stage_next = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void multi_free_graph(rb_multi* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

int rb_multi_create(rb_batch* const* batches, int32_t nbatch, rb_multi** out) {
    if (!batches || nbatch <= 0 || nbatch > 127 || !out) return fail(RB_EINVAL, "bad arguments to rb_multi_create");
    *out = nullptr;
    rb_multi* p = new rb_multi();
    std::vector<DevModel> models(nbatch);
    for (int i = 0; i < nbatch; i++) {
        if (!batches[i]) {
            delete p;
            return fail(RB_EINVAL, "null batch");
        }
        p->batches.push_back(batches[i]);
        models[i] = batches[i]->dm;
        p->maxd = std::max(p->maxd, models[i].maxd);
        p->boxbox = std::max(p->boxbox, models[i].ext);   // the extended code the models need
    }
    // every batch runs in its own model's instantiation, with its own LDS layout
    for (int i = 0; i < nbatch; i++) p->lds_floats = std::max(p->lds_floats, models[i].lds_floats);
    p->bound_n.assign(nbatch, -1);
    p->bind.assign(nbatch, BindRec{});
    p->args_host.assign(rb_step_args_size() * nbatch, 0);
    hipError_t e = hipMalloc((void**)&p->d_models, sizeof(DevModel) * nbatch);
    if (e == hipSuccess) e = hipMalloc(&p->d_args, rb_step_args_size() * nbatch);
    if (e == hipSuccess) e = hipMemcpy(p->d_models, models.data(), sizeof(DevModel) * nbatch, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_models) (void)hipFree(p->d_models);
        if (p->d_args) (void)hipFree(p->d_args);
        delete p;
        return hip_fail(e, "rb_multi_create");
    }
    *out = p;
    return RB_OK;
}

void rb_multi_destroy(rb_multi* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    multi_free_graph(p);
    if (p->d_models) (void)hipFree(p->d_models);
    if (p->d_args) (void)hipFree(p->d_args);
    if (p->d_items) (void)hipFree(p->d_items);
    for (int r = 0; r < rb_multi::RING; r++) {
        if (p->stage[r]) (void)hipHostFree(p->stage[r]);
        if (p->stage_ev[r]) (void)hipEventDestroy(p->stage_ev[r]);
    }
    delete p;
}

int rb_multi_bind(rb_multi* p, int32_t i, int32_t n, const float* ctrl, float* qpos, float* qvel, const rb_contacts* c,
                  uint32_t* status) {
    if (!p || i < 0 || i >= (int)p->batches.size()) return fail(RB_EINVAL, "bad batch index");
    rb_batch* b = p->batches[i];
    if (n < 0 || n > b->capacity) return fail(RB_EINVAL, "world count outside the batch capacity");
    if (n > 0 && (!qpos || !qvel)) return fail(RB_EINVAL, "qpos and qvel are required");
    if (n > 0 && b->dm.nu > 0 && !ctrl) return fail(RB_EINVAL, "ctrl is required for a model with actuators");
    DevContactsOut co{};
    if (c) {
        co.ncon = c->ncon; co.geom = c->geom; co.feature = c->feature; co.dist = c->dist;
        co.pos = c->pos; co.frame = c->frame; co.force = c->force;
    }
    size_t sz = rb_step_args_size();
    rb_fill_step_args(p->args_host.data() + sz * i, n, ctrl, qpos, qvel, b->W, c ? &co : nullptr, status);
    hipError_t e = hipMemcpy((char*)p->d_args + sz * i, p->args_host.data() + sz * i, sz, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "rb_multi_bind");
    p->bound_n[i] = n;
    BindRec& r = p->bind[i];
    r.n = n; r.ctrl = ctrl; r.qpos = qpos; r.qvel = qvel; r.co = co; r.has_co = c != nullptr; r.status = status;
    r.version = b->version;
    multi_free_graph(p);
    return RB_OK;
}

// A batch that expanded a model field since it was bound has new per-world arrays: rewrite its
// argument block (on the stream, before the launch that reads it).  The blocks live in device
// memory and launches (captured graphs included) read them at run time, so a captured graph
// picks up the new arrays without being captured again.
static int multi_refresh(rb_multi* p, hipStream_t stream) {
    const size_t sz = rb_step_args_size();
    for (size_t i = 0; i < p->batches.size(); i++) {
        BindRec& r = p->bind[i];
        rb_batch* b = p->batches[i];
        if (r.n < 0 || r.version == b->version) continue;
        rb_fill_step_args(p->args_host.data() + sz * i, r.n, r.ctrl, r.qpos, r.qvel, b->W, r.has_co ? &r.co : nullptr,
                          r.status);
        hipError_t e = hipMemcpyAsync((char*)p->d_args + sz * i, p->args_host.data() + sz * i, sz,
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);   // the host block is rewritten on the next refresh
        if (e != hipSuccess) return hip_fail(e, "re-binding a batch with expanded fields");
        r.version = b->version;
    }
    return RB_OK;
}

int rb_multi_set_schedule(rb_multi* p, int32_t order, int32_t grid, const float* cost) {
    if (!p) return fail(RB_EINVAL, "null plan");
    const int nb = (int)p->batches.size();
    for (int i = 0; i < nb; i++)
        if (p->bound_n[i] < 0) return fail(RB_ESTATE, "every batch must be bound before scheduling");
    std::vector<double> w(nb);
    for (int i = 0; i < nb; i++) {
        const DevModel& m = p->batches[i]->dm;
        w[i] = cost ? (double)cost[i] : (double)m.K * (m.nM + 8.0 * m.ncap + 4.0 * m.nbody);
    }
    std::vector<int> items;
    if (order == RB_ORDER_BATCH || order == RB_ORDER_HEAVY_FIRST) {
        std::vector<int> idx(nb);
        for (int i = 0; i < nb; i++) idx[i] = i;
        if (order == RB_ORDER_HEAVY_FIRST)
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] > w[b]; });
        for (int i : idx)
            for (int k = 0; k < p->bound_n[i]; k++) items.push_back(i << 24 | k);
    } else if (order == RB_ORDER_INTERLEAVE) {
        // each batch advances through its worlds at a rate proportional to its world count
        std::vector<int> next(nb, 0);
        int total = 0;
        for (int i = 0; i < nb; i++) total += p->bound_n[i];
        for (int t = 0; t < total; t++) {
            int best = -1;
            double bestf = 2.0;
            for (int i = 0; i < nb; i++) {
                if (next[i] >= p->bound_n[i]) continue;
                double f = (next[i] + 0.5) / p->bound_n[i];
                if (f < bestf) { bestf = f; best = i; }
            }
            items.push_back(best << 24 | next[best]++);
        }
    } else {
        return fail(RB_EINVAL, "unknown order");
    }
    if (p->d_items) (void)hipFree(p->d_items);
    p->d_items = nullptr;
    p->nitems = (int)items.size();
    p->scheduled = true;
    if (p->nitems > 0) {
        hipError_t e = hipMalloc((void**)&p->d_items, sizeof(int) * items.size());
        if (e == hipSuccess) e = hipMemcpy(p->d_items, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "rb_multi_set_schedule");
    }
    p->items_cap = p->nitems;
    p->grid = grid > 0 ? std::min(grid, std::max(p->nitems, 1)) : p->nitems;
    multi_free_graph(p);
    return RB_OK;
}

int rb_multi_set_items(rb_multi* p, const int32_t* items, int32_t n, int32_t grid, void* stream) {
    if (!p || n < 0 || (n > 0 && !items)) return fail(RB_EINVAL, "bad arguments to rb_multi_set_items");
    const int nb = (int)p->batches.size();
    for (int k = 0; k < n; k++) {
        const int b = (int)((uint32_t)items[k] >> 24), w = items[k] & 0xffffff;
        if (b >= nb || p->bound_n[b] < 0 || w >= p->bound_n[b])
            return fail(RB_EINVAL, "work item outside the bound batches");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (n > p->items_cap) {
        // launches queued on the stream may still read the old list
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "rb_multi_set_items");
        if (p->d_items) (void)hipFree(p->d_items);
        p->d_items = nullptr;
        p->items_cap = 0;
        const int cap = std::max(n, 1024);
        e = hipMalloc((void**)&p->d_items, sizeof(int32_t) * cap);
        if (e != hipSuccess) return hip_fail(e, "rb_multi_set_items");
        p->items_cap = cap;
    }
    if (n > p->stage_cap) {
        for (int r = 0; r < rb_multi::RING; r++) {
            if (p->stage_used[r]) (void)hipEventSynchronize(p->stage_ev[r]);
            if (p->stage[r]) (void)hipHostFree(p->stage[r]);
            p->stage[r] = nullptr;
            p->stage_used[r] = false;
        }
        p->stage_cap = 0;
        const int cap = std::max(n, 1024);
        for (int r = 0; r < rb_multi::RING && e == hipSuccess; r++) {
            e = hipHostMalloc((void**)&p->stage[r], sizeof(int32_t) * cap, hipHostMallocDefault);
            if (e == hipSuccess && !p->stage_ev[r]) e = hipEventCreateWithFlags(&p->stage_ev[r], hipEventDisableTiming);
        }
        if (e != hipSuccess) return hip_fail(e, "rb_multi_set_items");
        p->stage_cap = cap;
    }
    if (n > 0) {
        const int r = p->stage_next;
        p->stage_next = (r + 1) % rb_multi::RING;
        if (p->stage_used[r]) {
            e = hipEventSynchronize(p->stage_ev[r]);
            if (e != hipSuccess) return hip_fail(e, "rb_multi_set_items");
        }
        std::memcpy(p->stage[r], items, sizeof(int32_t) * n);
        e = hipMemcpyAsync(p->d_items, p->stage[r], sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(p->stage_ev[r], s);
        if (e != hipSuccess) return hip_fail(e, "rb_multi_set_items");
        p->stage_used[r] = true;
    }
    p->nitems = n;
    p->scheduled = true;
    p->grid = grid > 0 ? std::min(grid, std::max(n, 1)) : n;
    multi_free_graph(p);
    return RB_OK;
}

static void device_cu(int* ncu, int* lds_cu) {
    static int n = 0, l = 0;
    if (n == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            n = prop.multiProcessorCount;
            l = (int)prop.maxSharedMemoryPerMultiProcessor;
        }
    }
    *ncu = n;
    *lds_cu = l;
}

// whether the plan's models fit the 4-wave fused kernel (chain bound and LDS)
static bool multi_fits_w4(const rb_multi* p) {
    int ncu, lds_cu;
    device_cu(&ncu, &lds_cu);
    return p->maxd <= 16 && (long)p->lds_floats * 4 * 16 <= (long)lds_cu;
}

// waves per SIMD of the fused launch: as requested, or automatically 4 when the models fit and
// the work list is more than one round of the 3-wave kernel
static int multi_waves(const rb_multi* p) {
    if (p->occ == 4) return 4;
    if (p->occ != 0) return 3;
    int ncu, lds_cu;
    device_cu(&ncu, &lds_cu);
    return multi_fits_w4(p) && p->nitems > 12 * ncu ? 4 : 3;
}

// The LDS of one fused workgroup: wpg world sections, plus the padding that enforces an
// occupancy cap of w < 3 waves per SIMD.  Four SIMDs per CU and wpg waves per workgroup: the CU
// is capped at 4 w / wpg workgroups by making each one need more than 1 / (4 w / wpg + 1) of
// the CU's LDS.
static int multi_layout(rb_multi* p, int occ, int wpg, const char* who) {
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, who);
    const long sections = (long)wpg * p->lds_floats;   // floats
    if (sections * 4 > (long)prop.sharedMemPerBlock)
        return fail(RB_EINVAL, "the worlds of one workgroup need more LDS than a workgroup may use");
    int pad = 0;
    if (occ > 0 && occ < 3) {
        const long per_cu = (long)prop.maxSharedMemoryPerMultiProcessor;
        const long need = per_cu / (4 * occ / wpg + 1) / 4 + 1;   // floats
        if (need * 4 > (long)prop.sharedMemPerBlock) return fail(RB_EINVAL, "occupancy cap needs more LDS than a workgroup may use");
        pad = (int)std::max(0L, need - sections);
    }
    p->occ = occ;
    p->wpg = wpg;
    p->lds_pad = pad;
    multi_free_graph(p);
    return RB_OK;
}

int rb_multi_set_occupancy(rb_multi* p, int32_t waves_per_simd) {
    if (!p || waves_per_simd < 0 || waves_per_simd > 4) return fail(RB_EINVAL, "bad arguments to rb_multi_set_occupancy");
    if (waves_per_simd == 4 && !multi_fits_w4(p)) return fail(RB_EINVAL, "the plan's models do not fit 4 waves per SIMD");
    return multi_layout(p, waves_per_simd, p->wpg, "rb_multi_set_occupancy");
}

int rb_multi_set_group(rb_multi* p, int32_t worlds_per_workgroup) {
    const int g = worlds_per_workgroup;
    if (!p || (g != 1 && g != 2 && g != 4)) return fail(RB_EINVAL, "bad arguments to rb_multi_set_group (1, 2 or 4 worlds)");
    return multi_layout(p, p->occ, g, "rb_multi_set_group");
}

int rb_multi_step(rb_multi* p, void* stream) {
    if (!p) return fail(RB_EINVAL, "null plan");
    if (!p->scheduled) return fail(RB_ESTATE, "no schedule: set one (rb_multi_set_schedule or rb_multi_set_items) after binding");
    if (p->nitems == 0) return RB_OK;
    int rc = multi_refresh(p, (hipStream_t)stream);
    if (rc != RB_OK) return rc;
    hipError_t e = rb_launch_multi(p->d_models, p->d_args, p->d_items, p->nitems, p->maxd, p->boxbox, p->lds_floats,
                                   p->lds_pad, p->grid, p->wpg, multi_waves(p), (hipStream_t)stream);
    return e == hipSuccess ? RB_OK : hip_fail(e, "rb_multi_step");
}

int rb_multi_graph_capture(rb_multi* p, int32_t nsteps, void* stream) {
    if (!p || nsteps <= 0) return fail(RB_EINVAL, "bad arguments to rb_multi_graph_capture");
    if (!stream) return fail(RB_EINVAL, "graph capture needs a non-default stream");
    if (!p->scheduled || !p->d_items) return fail(RB_ESTATE, "no schedule");
    multi_free_graph(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    for (int k = 0; k < nsteps && e == hipSuccess; k++)
        e = rb_launch_multi(p->d_models, p->d_args, p->d_items, p->nitems, p->maxd, p->boxbox, p->lds_floats,
                            p->lds_pad, p->grid, p->wpg, multi_waves(p), s);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture");
    }
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    p->graph = g;
    return RB_OK;
}

int rb_multi_graph_launch(rb_multi* p, void* stream) {
    if (!p) return fail(RB_EINVAL, "null plan");
    if (!p->exec) return fail(RB_ESTATE, "nothing captured");
    int rc = multi_refresh(p, (hipStream_t)stream);
    if (rc != RB_OK) return rc;
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    return e == hipSuccess ? RB_OK : hip_fail(e, "hipGraphLaunch");
}

}  // extern "C"
