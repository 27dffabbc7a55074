// extern "C" entry points of include/wavefd.h: argument checks, then the
// runtime. No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "runtime.h"

using namespace wf;

#define ABI_GUARD_BEGIN try {
#define ABI_GUARD_END                                                         \
    }                                                                         \
    catch (const std::bad_alloc&) {                                           \
        return fail(WF_E_NOMEM, "host allocation failed");                    \
    }                                                                         \
    catch (...) {                                                             \
        return fail(WF_E_STATE, "internal error");                            \
    }

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

Model* as_model(wf_model* m) { return static_cast<Model*>(m); }

wf_status check_series(int nt, int npts, const void* series, const char* what) {
    if (npts < 0) return fail(WF_E_ARG, "%s: negative point count", what);
    if (npts > 0 && !series) return fail(WF_E_ARG, "%s: device array is NULL", what);
    if ((int64_t)nt * npts > ((int64_t)1 << 40)) return fail(WF_E_ARG, "%s: too large", what);
    return WF_OK;
}

}  // namespace

extern "C" {

const char* wf_last_error(void) { return last_error(); }

int wf_version(void) { return 10000; }

double wf_critical_dt(const wf_geom* geom, double vmax) {
    if (check_geom(geom) != WF_OK) return -1.0;
    if (!(vmax > 0.0) || !std::isfinite(vmax)) {
        fail(WF_E_ARG, "vmax must be > 0");
        return -1.0;
    }
    return critical_dt(geom, vmax);
}

wf_status wf_geom_shape(const wf_geom* geom, int64_t shape_out[3], int64_t* npoints_out) {
    wf_status st = check_geom(geom);
    if (st != WF_OK) return st;
    int64_t x, y, z;
    comp_shape(geom, &x, &y, &z);
    if (shape_out) {
        shape_out[0] = x;
        shape_out[1] = geom->ndim == 3 ? y : z;
        shape_out[2] = geom->ndim == 3 ? z : 1;
    }
    if (npoints_out) *npoints_out = x * y * z;
    return WF_OK;
}

wf_status wf_model_create(const wf_geom* geom, const float* m_dev, void* stream, wf_model** out) {
    ABI_GUARD_BEGIN
    if (!out) return fail(WF_E_ARG, "out is NULL");
    *out = nullptr;
    wf_status st = check_geom(geom);
    if (st != WF_OK) return st;
    if (!m_dev) return fail(WF_E_ARG, "m is NULL");
    Model* md = new Model();
    st = md->init(geom, m_dev, as_stream(stream));
    if (st != WF_OK) {
        delete md;
        return st;
    }
    *out = md;
    return WF_OK;
    ABI_GUARD_END
}

wf_status wf_model_set_m(wf_model* model, const float* m_dev, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    return as_model(model)->set_m(m_dev, as_stream(stream));
    ABI_GUARD_END
}

int64_t wf_model_bytes(const wf_model* model) {
    if (!model) return -1;
    return static_cast<const Model*>(model)->bytes();
}

wf_status wf_model_trim(wf_model* model) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    wf_status st = hip_check(hipStreamSynchronize(md.last_stream), "sync");
    if (st != WF_OK) return st;
    md.ws.reset();
    md.ws_clean = false;
    md.d_u2[0].reset();
    md.d_u2[1].reset();
    return WF_OK;
    ABI_GUARD_END
}

wf_status wf_model_ghost_nonzero(wf_model* model, int64_t* count) {
    ABI_GUARD_BEGIN
    if (!model || !count) return fail(WF_E_ARG, "NULL argument");
    return count_ghost_nonzero(*as_model(model), count);
    ABI_GUARD_END
}

wf_status wf_validate_enable(int on) {
    set_validation(on != 0);
    return WF_OK;
}

wf_status wf_graph_enable(int on) {
    set_graphs_enabled(on != 0);
    return WF_OK;
}

wf_status wf_two_step_enable(int mode) {
    if (mode < 0 || mode > 2) return fail(WF_E_ARG, "two-step mode must be 0, 1 or 2");
    set_two_step_mode(mode);
    return WF_OK;
}

int64_t wf_model_graph_launches(const wf_model* model) {
    if (!model) return -1;
    return static_cast<const Model*>(model)->graph_launches;
}

wf_status wf_model_destroy(wf_model* model) {
    ABI_GUARD_BEGIN
    delete as_model(model);
    return WF_OK;
    ABI_GUARD_END
}

wf_status wf_forward(wf_model* model, double dt, int nt, int nsrc, const double* src_xyz,
                     const float* src_wav, int nrec, const double* rec_xyz, float* rec_out,
                     float* u_save, int save_every, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
    wf_status st;
    if ((st = md.check_dt(dt)) != WF_OK) return st;
    if ((st = check_series(nt, nsrc, src_wav, "src_wav")) != WF_OK) return st;
    if ((st = check_series(nt, nrec, rec_out, "rec_out")) != WF_OK) return st;
    if (u_save && save_every < 1) return fail(WF_E_ARG, "save_every must be >= 1");
    const PointSet *src = nullptr, *rec = nullptr;
    if ((st = md.points(nsrc, src_xyz, &src)) != WF_OK) return st;
    if ((st = md.points(nrec, rec_xyz, &rec)) != WF_OK) return st;
    hipStream_t s = as_stream(stream);
    st = run_forward(md, dt, nt, *src, src_wav, *rec, rec_out, u_save, save_every, s);
    if (st == WF_OK && validation_enabled()) {
        st = md.check_finite(rec_out, (int64_t)nt * nrec, "rec_out", s);
        if (st == WF_OK && u_save)
            st = md.check_finite(u_save, ((int64_t)(nt - 1) / save_every + 1) * md.L.npoints, "u_save", s);
    }
    return st;
    ABI_GUARD_END
}

wf_status wf_adjoint(wf_model* model, double dt, int nt, int nrec, const double* rec_xyz,
                     const float* rec_in, int nsrc, const double* src_xyz, float* src_out,
                     void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
    wf_status st;
    if ((st = md.check_dt(dt)) != WF_OK) return st;
    if ((st = check_series(nt, nrec, rec_in, "rec_in")) != WF_OK) return st;
    if ((st = check_series(nt, nsrc, src_out, "src_out")) != WF_OK) return st;
    const PointSet *src = nullptr, *rec = nullptr;
    if ((st = md.points(nsrc, src_xyz, &src)) != WF_OK) return st;
    if ((st = md.points(nrec, rec_xyz, &rec)) != WF_OK) return st;
    hipStream_t s = as_stream(stream);
    st = run_adjoint(md, dt, nt, *rec, rec_in, *src, src_out, s);
    if (st == WF_OK && validation_enabled()) st = md.check_finite(src_out, (int64_t)nt * nsrc, "src_out", s);
    return st;
    ABI_GUARD_END
}

wf_status wf_gradient(wf_model* model, double dt, int nt, int nsrc, const double* src_xyz,
                      const float* src_wav, int nrec, const double* rec_xyz, const float* residual,
                      float* grad_out, int n_checkpoints, int64_t hbm_budget_bytes, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
    if (!grad_out) return fail(WF_E_ARG, "grad_out is NULL");
    if (n_checkpoints < -2) return fail(WF_E_ARG, "n_checkpoints must be >= -2");
    if (hbm_budget_bytes < 0) return fail(WF_E_ARG, "negative budget");
    wf_status st;
    if ((st = md.check_dt(dt)) != WF_OK) return st;
    if ((st = check_series(nt, nsrc, src_wav, "src_wav")) != WF_OK) return st;
    if ((st = check_series(nt, nrec, residual, "residual")) != WF_OK) return st;
    const PointSet *src = nullptr, *rec = nullptr;
    if ((st = md.points(nsrc, src_xyz, &src)) != WF_OK) return st;
    if ((st = md.points(nrec, rec_xyz, &rec)) != WF_OK) return st;
    hipStream_t s = as_stream(stream);
    st = run_gradient(md, dt, nt, *src, src_wav, *rec, residual, grad_out, n_checkpoints, hbm_budget_bytes, s);
    if (st == WF_OK && validation_enabled()) st = md.check_finite(grad_out, md.L.npoints, "grad_out", s);
    return st;
    ABI_GUARD_END
}

wf_status wf_born(wf_model* model, double dt, int nt, int nsrc, const double* src_xyz,
                  const float* src_wav, const float* dm, int nrec, const double* rec_xyz,
                  float* drec_out, float* rec_out, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
    if (!dm) return fail(WF_E_ARG, "dm is NULL");
    wf_status st;
    if ((st = md.check_dt(dt)) != WF_OK) return st;
    if ((st = check_series(nt, nsrc, src_wav, "src_wav")) != WF_OK) return st;
    if ((st = check_series(nt, nrec, drec_out, "drec_out")) != WF_OK) return st;
    const PointSet *src = nullptr, *rec = nullptr;
    if ((st = md.points(nsrc, src_xyz, &src)) != WF_OK) return st;
    if ((st = md.points(nrec, rec_xyz, &rec)) != WF_OK) return st;
    hipStream_t s = as_stream(stream);
    st = run_born(md, dt, nt, *src, src_wav, dm, *rec, drec_out, rec_out, s);
    if (st == WF_OK && validation_enabled()) {
        st = md.check_finite(drec_out, (int64_t)nt * nrec, "drec_out", s);
        if (st == WF_OK) st = md.check_finite(rec_out, (int64_t)nt * nrec, "rec_out", s);
    }
    return st;
    ABI_GUARD_END
}

wf_status wf_fwi_gradient(wf_model* model, double dt, int nt, int nshots, const wf_shot* shots,
                          float* grad_out, double* misfit_out, int n_checkpoints,
                          int64_t hbm_budget_bytes, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    Model& md = *as_model(model);
    if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
    if (nshots < 1 || !shots) return fail(WF_E_ARG, "at least one shot is needed");
    if (!grad_out) return fail(WF_E_ARG, "grad_out is NULL");
    if (n_checkpoints < -2) return fail(WF_E_ARG, "n_checkpoints must be >= -2");
    if (hbm_budget_bytes < 0) return fail(WF_E_ARG, "negative budget");
    wf_status st;
    if ((st = md.check_dt(dt)) != WF_OK) return st;
    std::vector<FwiShot> v((size_t)nshots);
    for (int i = 0; i < nshots; ++i) {
        const wf_shot& sh = shots[i];
        if ((st = check_series(nt, sh.nsrc, sh.src_wav, "src_wav")) != WF_OK) return st;
        if ((st = check_series(nt, sh.nrec, sh.d_obs, "d_obs")) != WF_OK) return st;
        if (sh.nsrc > 0 && !sh.src_xyz) return fail(WF_E_ARG, "shot %d: src_xyz is NULL", i);
        if (sh.nrec > 0 && !sh.rec_xyz) return fail(WF_E_ARG, "shot %d: rec_xyz is NULL", i);
        // every coordinate is checked before any work is enqueued
        const PointSet* ps = nullptr;
        if ((st = md.points(sh.nsrc, sh.src_xyz, &ps)) != WF_OK) return st;
        if ((st = md.points(sh.nrec, sh.rec_xyz, &ps)) != WF_OK) return st;
        v[(size_t)i] = FwiShot{sh.nsrc, sh.src_xyz, sh.src_wav, sh.nrec, sh.rec_xyz, sh.d_obs, sh.d_pred};
    }
    hipStream_t s = as_stream(stream);
    double phi = 0.0;
    st = run_fwi_gradient(md, dt, nt, v, grad_out, &phi, n_checkpoints, hbm_budget_bytes, s);
    if (st == WF_OK && misfit_out) *misfit_out = phi;
    if (st == WF_OK && validation_enabled()) {
        st = md.check_finite(grad_out, md.L.npoints, "grad_out", s);
        for (int i = 0; i < nshots && st == WF_OK; ++i)
            st = md.check_finite(shots[i].d_pred, (int64_t)nt * shots[i].nrec, "d_pred", s);
        if (st == WF_OK && !std::isfinite(phi)) st = fail(WF_E_NONFINITE, "the misfit is not finite");
    }
    return st;
    ABI_GUARD_END
}

wf_status wf_model_update(wf_model* model, const float* grad, double alpha, double m_lo,
                          double m_hi, float* m_out, void* stream) {
    ABI_GUARD_BEGIN
    if (!model) return fail(WF_E_ARG, "model is NULL");
    return as_model(model)->update(grad, alpha, m_lo, m_hi, m_out, as_stream(stream));
    ABI_GUARD_END
}

int64_t wf_revolve_forward_steps(int64_t steps, int snaps) { return revolve_cost(steps, snaps); }

}  // extern "C"
