// rb_model_create_json: a model description as JSON text (the same fields as rb_model_desc,
// grouped per body / joint / geom / actuator), parsed on the host into an rb_model_desc.
//
// {"opt": {"timestep", "nsubsteps", "gravity": [3], "iterations", "tolerance",
//          "solref": [2], "solimp": [5], "cone": "pyramidal"|"elliptic", "impratio" (optional)},
//  "bodies": [{"parent", "pos": [3], "quat": [4], "ipos": [3], "iquat": [4], "mass",
//              "inertia": [3]}, ...],                    body 0 is the world
//  "joints": [{"type": "free"|"hinge", "body", "pos": [3], "axis": [3], "armature",
//              "range": [2], "damping" (both optional)}, ...],
//  "geoms": [{"type": "plane"|"sphere"|"capsule"|"box"|"hfield", "body", "pos": [3], "quat": [4],
//             "size": [3], "friction", "contype", "conaffinity", "margin", "condim", "friction_spin",
//             "friction_roll" (the last three optional)}, ...],
//  "actuators": [{"type": "position"|"motor", "joint", "kp", "kd", "gear"}, ...],
//  "per_world": {"friction": bool, "mass_scale": bool},      optional, default false
//  "hfield": {"nrow", "ncol", "data": [nrow * ncol]},         required with hfield geoms
//  "equality": [{"type": "connect"|"weld", "body", "anchor": [3], "target": [3],
//                "quat": [4] (welds)}, ...]}                  optional
//
// Other keys (names, comments) are ignored.  Every listed field is required except a joint's
// range and damping, a geom's condim, friction_spin and friction_roll, per_world, hfield and
// equality; a missing or mistyped field is RB_EINVAL with the field named.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "rbstep.h"

namespace {

struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::map<std::string, JVal> obj;
};

struct Parser {
    const char* s;
    size_t i = 0;
    std::string err;

    explicit Parser(const char* text) : s(text) {}
    void ws() {
        while (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r') i++;
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = m + " at offset " + std::to_string(i);
        return false;
    }
    bool lit(const char* w) {
        size_t n = std::strlen(w);
        if (std::strncmp(s + i, w, n) != 0) return fail(std::string("expected ") + w);
        i += n;
        return true;
    }
    bool string(std::string& out) {
        if (s[i] != '"') return fail("expected a string");
        i++;
        out.clear();
        while (s[i] && s[i] != '"') {
            if (s[i] == '\\') {
                i++;
                char c = s[i];
                if (c == 'n') out += '\n';
                else if (c == 't') out += '\t';
                else if (c == 'u') {
                    // keep the escape as text: names are not used
                    for (int k = 0; k < 5 && s[i]; k++) out += s[i++];
                    continue;
                } else if (c) out += c;
                else return fail("unterminated escape");
                i++;
            } else {
                out += s[i++];
            }
        }
        if (s[i] != '"') return fail("unterminated string");
        i++;
        return true;
    }
    bool value(JVal& v, int depth) {
        if (depth > 64) return fail("nesting too deep");
        ws();
        char c = s[i];
        if (c == '{') {
            v.kind = JVal::OBJ;
            i++;
            ws();
            if (s[i] == '}') { i++; return true; }
            for (;;) {
                ws();
                std::string key;
                if (!string(key)) return false;
                ws();
                if (s[i] != ':') return fail("expected ':'");
                i++;
                JVal child;
                if (!value(child, depth + 1)) return false;
                v.obj[key] = std::move(child);
                ws();
                if (s[i] == ',') { i++; continue; }
                if (s[i] == '}') { i++; return true; }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v.kind = JVal::ARR;
            i++;
            ws();
            if (s[i] == ']') { i++; return true; }
            for (;;) {
                JVal child;
                if (!value(child, depth + 1)) return false;
                v.arr.push_back(std::move(child));
                ws();
                if (s[i] == ',') { i++; continue; }
                if (s[i] == ']') { i++; return true; }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (c == 't') { v.kind = JVal::BOOL; v.b = true; return lit("true"); }
        if (c == 'f') { v.kind = JVal::BOOL; v.b = false; return lit("false"); }
        if (c == 'n') { v.kind = JVal::NUL; return lit("null"); }
        if (c == '-' || (c >= '0' && c <= '9')) {
            char* end = nullptr;
            v.kind = JVal::NUM;
            v.num = std::strtod(s + i, &end);
            if (end == s + i) return fail("bad number");
            // JSON numbers are finite; strtod would also take "-inf" and "-nan"
            if (!std::isfinite(v.num)) return fail("non-finite number");
            i = (size_t)(end - s);
            return true;
        }
        return fail("unexpected character");
    }
};

struct Reader {
    std::string err;
    bool fail(const std::string& m) {
        if (err.empty()) err = m;
        return false;
    }
    const JVal* field(const JVal& o, const char* key, const std::string& where) {
        if (o.kind != JVal::OBJ) { fail(where + " is not an object"); return nullptr; }
        auto it = o.obj.find(key);
        if (it == o.obj.end()) { fail(where + ": missing \"" + key + "\""); return nullptr; }
        return &it->second;
    }
    bool num(const JVal& o, const char* key, const std::string& where, double* out) {
        const JVal* v = field(o, key, where);
        if (!v) return false;
        if (v->kind != JVal::NUM) return fail(where + ": \"" + key + "\" is not a number");
        *out = v->num;
        return true;
    }
    bool integer(const JVal& o, const char* key, const std::string& where, int32_t* out) {
        double d;
        if (!num(o, key, where, &d)) return false;
        if (d != std::floor(d) || std::fabs(d) > 2e9) return fail(where + ": \"" + key + "\" is not an integer");
        *out = (int32_t)d;
        return true;
    }
    bool vec(const JVal& o, const char* key, const std::string& where, int n, double* out) {
        const JVal* v = field(o, key, where);
        if (!v) return false;
        if (v->kind != JVal::ARR || (int)v->arr.size() != n)
            return fail(where + ": \"" + key + "\" is not an array of " + std::to_string(n) + " numbers");
        for (int k = 0; k < n; k++) {
            if (v->arr[k].kind != JVal::NUM) return fail(where + ": \"" + key + "\" holds a non-number");
            out[k] = v->arr[k].num;
        }
        return true;
    }
    bool choice(const JVal& o, const char* key, const std::string& where, const char* const* names, int n,
                int32_t* out) {
        const JVal* v = field(o, key, where);
        if (!v) return false;
        if (v->kind != JVal::STR) return fail(where + ": \"" + key + "\" is not a string");
        for (int k = 0; k < n; k++)
            if (v->str == names[k]) { *out = k; return true; }
        return fail(where + ": unknown " + key + " \"" + v->str + "\"");
    }
    const std::vector<JVal>* list(const JVal& root, const char* key) {
        const JVal* v = field(root, key, "model");
        if (!v) return nullptr;
        if (v->kind != JVal::ARR) { fail(std::string("model: \"") + key + "\" is not an array"); return nullptr; }
        return &v->arr;
    }
};

}  // namespace

// records the message rb_last_error returns (runtime.hip)
int rb_record_error(int code, const char* msg);

extern "C" {

int rb_model_create_json(const char* json, rb_model** out) {
    if (!json || !out) return rb_record_error(RB_EINVAL, "null argument to rb_model_create_json");
    *out = nullptr;
    Parser P(json);
    JVal root;
    if (!P.value(root, 0)) return rb_record_error(RB_EINVAL, ("model JSON: " + P.err).c_str());
    P.ws();
    if (P.s[P.i]) return rb_record_error(RB_EINVAL, "model JSON: trailing characters");
    Reader R;
    const std::vector<JVal>* bodies = R.list(root, "bodies");
    const std::vector<JVal>* joints = bodies ? R.list(root, "joints") : nullptr;
    const std::vector<JVal>* geoms = joints ? R.list(root, "geoms") : nullptr;
    const std::vector<JVal>* acts = geoms ? R.list(root, "actuators") : nullptr;
    const JVal* opt = acts ? R.field(root, "opt", "model") : nullptr;
    if (!opt) return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
    const int nb = (int)bodies->size(), nj = (int)joints->size(), ng = (int)geoms->size(), nu = (int)acts->size();
    // one spare element each, so that an empty list still hands over a valid pointer
    const int b1 = nb + 1, j1 = nj + 1, g1 = ng + 1, u1 = nu + 1;
    std::vector<int32_t> bpar(b1), jtype(j1), jbody(j1), gtype(g1), gbody(g1), gct(g1), gca(g1), atype(u1), ajnt(u1),
        gdim(g1, 3);
    std::vector<double> bpos(3 * b1), bquat(4 * b1), bipos(3 * b1), biquat(4 * b1), bmass(b1), binert(3 * b1);
    std::vector<double> jpos(3 * j1), jaxis(3 * j1), jarm(j1), jrange(2 * j1, 0.0), jdamp(j1, 0.0);
    std::vector<double> gpos(3 * g1), gquat(4 * g1), gsize(3 * g1), gfric(g1), gmarg(g1), gspin(g1, 0.005),
        groll(g1, 0.0001);
    std::vector<double> akp(u1), akd(u1), agear(u1);
    bool ok = true;
    for (int b = 0; b < nb && ok; b++) {
        const JVal& o = (*bodies)[b];
        const std::string w = "body " + std::to_string(b);
        ok = R.integer(o, "parent", w, &bpar[b]) && R.vec(o, "pos", w, 3, &bpos[3 * b]) &&
             R.vec(o, "quat", w, 4, &bquat[4 * b]) && R.vec(o, "ipos", w, 3, &bipos[3 * b]) &&
             R.vec(o, "iquat", w, 4, &biquat[4 * b]) && R.num(o, "mass", w, &bmass[b]) &&
             R.vec(o, "inertia", w, 3, &binert[3 * b]);
    }
    static const char* const jnames[] = {"free", "hinge"};
    for (int j = 0; j < nj && ok; j++) {
        const JVal& o = (*joints)[j];
        const std::string w = "joint " + std::to_string(j);
        ok = R.choice(o, "type", w, jnames, 2, &jtype[j]) && R.integer(o, "body", w, &jbody[j]) &&
             R.vec(o, "pos", w, 3, &jpos[3 * j]) && R.vec(o, "axis", w, 3, &jaxis[3 * j]) &&
             R.num(o, "armature", w, &jarm[j]);
        if (ok && o.obj.count("range")) ok = R.vec(o, "range", w, 2, &jrange[2 * j]);
        if (ok && o.obj.count("damping")) ok = R.num(o, "damping", w, &jdamp[j]);
    }
    static const char* const gnames[] = {"plane", "sphere", "capsule", "box", "hfield"};
    for (int g = 0; g < ng && ok; g++) {
        const JVal& o = (*geoms)[g];
        const std::string w = "geom " + std::to_string(g);
        ok = R.choice(o, "type", w, gnames, 5, &gtype[g]) && R.integer(o, "body", w, &gbody[g]) &&
             R.vec(o, "pos", w, 3, &gpos[3 * g]) && R.vec(o, "quat", w, 4, &gquat[4 * g]) &&
             R.vec(o, "size", w, 3, &gsize[3 * g]) && R.num(o, "friction", w, &gfric[g]) &&
             R.integer(o, "contype", w, &gct[g]) && R.integer(o, "conaffinity", w, &gca[g]) &&
             R.num(o, "margin", w, &gmarg[g]);
        if (ok && o.obj.count("condim")) ok = R.integer(o, "condim", w, &gdim[g]);
        if (ok && o.obj.count("friction_spin")) ok = R.num(o, "friction_spin", w, &gspin[g]);
        if (ok && o.obj.count("friction_roll")) ok = R.num(o, "friction_roll", w, &groll[g]);
    }
    static const char* const anames[] = {"position", "motor"};
    for (int u = 0; u < nu && ok; u++) {
        const JVal& o = (*acts)[u];
        const std::string w = "actuator " + std::to_string(u);
        ok = R.choice(o, "type", w, anames, 2, &atype[u]) && R.integer(o, "joint", w, &ajnt[u]) &&
             R.num(o, "kp", w, &akp[u]) && R.num(o, "kd", w, &akd[u]) && R.num(o, "gear", w, &agear[u]);
    }
    rb_model_desc d;
    std::memset(&d, 0, sizeof d);
    double nsub = 0, iters = 0;
    ok = ok && R.num(*opt, "timestep", "opt", &d.timestep) && R.num(*opt, "nsubsteps", "opt", &nsub) &&
         R.vec(*opt, "gravity", "opt", 3, d.gravity) && R.num(*opt, "iterations", "opt", &iters) &&
         R.num(*opt, "tolerance", "opt", &d.tolerance) && R.vec(*opt, "solref", "opt", 2, d.solref) &&
         R.vec(*opt, "solimp", "opt", 5, d.solimp);
    if (!ok) return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
    if (nsub != std::floor(nsub) || iters != std::floor(iters) || std::fabs(nsub) > 1e9 || std::fabs(iters) > 1e9)
        return rb_record_error(RB_EINVAL, "model JSON: opt nsubsteps and iterations must be integers");
    d.nsubsteps = (int32_t)nsub;
    d.iterations = (int32_t)iters;
    d.impratio = 1.0;
    if (opt->obj.count("cone")) {
        static const char* const cnames[] = {"pyramidal", "elliptic"};
        if (!R.choice(*opt, "cone", "opt", cnames, 2, &d.cone))
            return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
    }
    if (opt->obj.count("impratio") && !R.num(*opt, "impratio", "opt", &d.impratio))
        return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
    auto pw = root.obj.find("per_world");
    if (pw != root.obj.end() && pw->second.kind == JVal::OBJ) {
        auto f = pw->second.obj.find("friction");
        auto s = pw->second.obj.find("mass_scale");
        d.friction_per_world = f != pw->second.obj.end() && f->second.kind == JVal::BOOL && f->second.b;
        d.mass_scale_per_world = s != pw->second.obj.end() && s->second.kind == JVal::BOOL && s->second.b;
    }
    std::vector<double> hfdata;
    auto hf = root.obj.find("hfield");
    if (hf != root.obj.end()) {
        double nr = 0, nc = 0;
        ok = R.num(hf->second, "nrow", "hfield", &nr) && R.num(hf->second, "ncol", "hfield", &nc);
        if (ok && (nr != std::floor(nr) || nc != std::floor(nc) || nr < 2 || nc < 2 || nr * nc > 1e7))
            return rb_record_error(RB_EINVAL, "model JSON: hfield nrow and ncol must be integers >= 2");
        if (ok) {
            hfdata.assign((size_t)(nr * nc), 0.0);
            ok = R.vec(hf->second, "data", "hfield", (int)(nr * nc), hfdata.data());
        }
        if (!ok) return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
        d.hfield_nrow = (int32_t)nr;
        d.hfield_ncol = (int32_t)nc;
        d.hfield_data = hfdata.data();
    }
    std::vector<int32_t> etype, ebody;
    std::vector<double> eanchor, etarget;
    auto eq = root.obj.find("equality");
    if (eq != root.obj.end()) {
        if (eq->second.kind != JVal::ARR) return rb_record_error(RB_EINVAL, "model JSON: \"equality\" is not an array");
        static const char* const enames[] = {"connect", "weld"};
        const int ne = (int)eq->second.arr.size();
        etype.assign(ne, 0); ebody.assign(ne, 0); eanchor.assign(3 * ne, 0.0); etarget.assign(7 * ne, 0.0);
        for (int q = 0; q < ne && ok; q++) {
            const JVal& o = eq->second.arr[q];
            const std::string w = "equality " + std::to_string(q);
            ok = R.choice(o, "type", w, enames, 2, &etype[q]) && R.integer(o, "body", w, &ebody[q]) &&
                 R.vec(o, "anchor", w, 3, &eanchor[3 * q]) && R.vec(o, "target", w, 3, &etarget[7 * q]);
            etarget[7 * q + 3] = 1.0;
            if (ok && etype[q] == RB_EQ_WELD) ok = R.vec(o, "quat", w, 4, &etarget[7 * q + 3]);
        }
        if (!ok) return rb_record_error(RB_EINVAL, ("model JSON: " + R.err).c_str());
        d.neq = ne;
        if (ne > 0) {
            d.eq_type = etype.data(); d.eq_body = ebody.data();
            d.eq_anchor = eanchor.data(); d.eq_target = etarget.data();
        }
    }
    d.nbody = nb; d.njnt = nj; d.ngeom = ng; d.nu = nu;
    d.body_parent = bpar.data(); d.body_pos = bpos.data(); d.body_quat = bquat.data();
    d.body_ipos = bipos.data(); d.body_iquat = biquat.data(); d.body_mass = bmass.data(); d.body_inertia = binert.data();
    d.jnt_type = jtype.data(); d.jnt_body = jbody.data(); d.jnt_pos = jpos.data(); d.jnt_axis = jaxis.data();
    d.jnt_armature = jarm.data();
    d.jnt_range = jrange.data();
    d.jnt_damping = jdamp.data();
    d.geom_condim = gdim.data();
    d.geom_friction_spin = gspin.data();
    d.geom_friction_roll = groll.data();
    d.geom_type = gtype.data(); d.geom_body = gbody.data(); d.geom_contype = gct.data(); d.geom_conaffinity = gca.data();
    d.geom_pos = gpos.data(); d.geom_quat = gquat.data(); d.geom_size = gsize.data(); d.geom_friction = gfric.data();
    d.geom_margin = gmarg.data();
    d.act_type = atype.data(); d.act_joint = ajnt.data(); d.act_kp = akp.data(); d.act_kd = akd.data();
    d.act_gear = agear.data();
    return rb_model_create(&d, out);
}

}  // extern "C"
