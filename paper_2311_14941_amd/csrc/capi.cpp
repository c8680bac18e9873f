// C ABI of libstiffchem (declared in include/stiffchem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <tuple>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "devmech.hpp"
#include "mech.hpp"
#include "stiffchem.h"

struct sc_mech {
    sc::Mech m;
};

struct sc_plan {
    sc::Mech m;  // private copy: the plan does not depend on the sc_mech's lifetime
    sc_options opt;
    int device = 0;
    int np = 0;
    scdev::DevMech dm{};
    bool sparse = false;  // sparse linear algebra kernels
    int vpl = 1;          // state components per lane of the sparse kernels
    scdev::DevSparse ds{};
    std::vector<void *> allocs;
    unsigned long long *queue = nullptr;
    int capacity = 0;
    void *order_ws = nullptr;  // cell-ordering workspace (grown on demand)
    size_t order_ws_bytes = 0;
    int adj_capacity = 0;        // resident waves of the adjoint kernel
    void *adj_ws = nullptr;      // adjoint per-wave slots (grown on demand)
    size_t adj_ws_bytes = 0;
    void *gcell_ws = nullptr;    // per-cell parameter adjoints when the caller passes none
    size_t gcell_ws_bytes = 0;
    bool mapping = false;        // sc_plan_set_mapping has been called
    scdev::MapParams mp{};       // its weights and zone table (device), band sizes
};

namespace {

thread_local std::string g_err;

sc_status fail(sc_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

sc_status hip_fail(hipError_t e, const char *what)
{
    return fail(SC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
bool upload(sc_plan *p, const std::vector<T> &v, const T **out)
{
    size_t bytes = sizeof(T) * (v.empty() ? 1 : v.size());
    void *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return false;
    p->allocs.push_back(d);
    if (!v.empty() && hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
        return false;
    *out = static_cast<const T *>(d);
    return true;
}

void release(sc_plan *p)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    for (void *d : p->allocs) (void)hipFree(d);
    p->allocs.clear();
    for (void **w : {&p->order_ws, &p->adj_ws, &p->gcell_ws})
        if (*w) (void)hipFree(*w);
    p->order_ws = p->adj_ws = p->gcell_ws = nullptr;
    p->order_ws_bytes = p->adj_ws_bytes = p->gcell_ws_bytes = 0;
    (void)hipSetDevice(cur);
}

struct DeviceGuard {
    int prev = 0;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard()
    {
        if (ok) (void)hipSetDevice(prev);
    }
};

// Grow a plan-owned device workspace to at least `need` bytes.
hipError_t grow(void **ws, size_t *have, size_t need)
{
    if (*have >= need) return hipSuccess;
    if (*ws) (void)hipFree(*ws);
    *ws = nullptr;
    *have = 0;
    hipError_t e = hipMalloc(ws, need);
    if (e == hipSuccess) *have = need;
    return e;
}

scdev::Opts dev_opts(const sc_options &o)
{
    return scdev::Opts{o.rtol, o.atol, o.hmax_frac, o.max_steps, o.fixed_step};
}

sc_status check_common(sc_plan *plan, int64_t n, int64_t ld, std::initializer_list<const void *> ptrs)
{
    if (!plan) return fail(SC_EINVAL, "plan is NULL");
    if (n < 0) return fail(SC_EINVAL, "n must be >= 0");
    if (n > INT_MAX) return fail(SC_EINVAL, "n exceeds 2^31-1 cells");
    if (n == 0) return SC_OK;
    if (ld < n) return fail(SC_EINVAL, "ld must be >= n");
    for (const void *q : ptrs)
        if (!q) return fail(SC_EINVAL, "required array pointer is NULL");
    return SC_OK;
}

}  // namespace

extern "C" {

const char *sc_last_error(void) { return g_err.c_str(); }

void sc_default_options(sc_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->rtol = 1e-6;
    opt->atol = 1e-12;
    opt->max_steps = 100000;
    opt->mode = SC_MODE_PLAIN;
    opt->tile = 1;
    opt->grid = 0;
    opt->order = 0;
    opt->reactor = SC_REACTOR_CONST_P;
    opt->method = SC_METHOD_ROS4;
    opt->thermo_tol = 0.0;
    opt->thermo_Tmin = 250.0;
    opt->thermo_Tmax = 4000.0;
    opt->thermo_degree = 0;
}

sc_status sc_mech_load(const char *text, size_t len, sc_mech **out)
{
    if (!out) return fail(SC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!text) return fail(SC_EINVAL, "text is NULL");
    try {
        auto *h = new sc_mech{sc::load_mechanism(std::string(text, len))};
        *out = h;
        return SC_OK;
    } catch (const sc::Unsupported &e) {
        return fail(SC_EUNSUPPORTED, e.what());
    } catch (const sc::ParseError &e) {
        return fail(SC_EPARSE, e.what());
    } catch (const std::bad_alloc &) {
        return fail(SC_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SC_EPARSE, e.what());
    }
}

void sc_mech_free(sc_mech *mech) { delete mech; }

sc_status sc_mech_info_get(const sc_mech *mech, sc_mech_info *out)
{
    if (!mech || !out) return fail(SC_EINVAL, "NULL argument");
    const sc::Mech &m = mech->m;
    std::memset(out, 0, sizeof *out);
    out->n_species = m.N;
    out->n_reactions = m.R;
    out->n_third_body = m.n_third;
    out->n_troe = m.n_troe;
    out->n_elements = m.E;
    out->n_state = m.N + 1;
    out->n_padded = m.n_padded;
    out->nnz_jac = m.cnt.nnz_jac;
    out->nnz_lu = m.cnt.nnz_lu;
    out->n_stages = 4;
    out->rhs_evals_per_step = 3;
    out->exp_per_rhs = m.cnt.exp_per_rhs;
    out->flops_rhs = m.cnt.flops_rhs;
    out->flops_jac = m.cnt.flops_jac;
    out->flops_lu = m.cnt.flops_lu;
    out->flops_solve = m.cnt.flops_solve;
    out->flops_step = m.cnt.flops_step;
    out->nnz_a_sparse = (int32_t)m.sp.nnz_a;
    out->nnz_lu_sparse = m.sp.nnz;
    out->lu_levels = (int32_t)m.sp.lu_b_lvl.size() - 1;
    out->solve_levels = (int32_t)(m.sp.fw_lvl.size() + m.sp.bw_lvl.size()) - 2;
    out->lu_updates_sparse = m.sp.updates;
    out->flops_lu_sparse = m.cnt_sparse.flops_lu;
    out->flops_solve_sparse = m.cnt_sparse.flops_solve;
    out->flops_step_sparse = m.cnt_sparse.flops_step;
    out->lu_tail_sparse = m.sp.n - m.sp.tail0;
    return SC_OK;
}

sc_status sc_mech_thermo_fit(const sc_mech *mech, double Tmin, double Tmax, double tol, int32_t degree,
                             int32_t *degree_out, int32_t *nint_out, double *max_err_out, double *coef,
                             size_t *ncoef)
{
    if (!mech) return fail(SC_EINVAL, "mech is NULL");
    sc::ThermoFit f;
    try {
        f = sc::fit_thermo(mech->m, Tmin, Tmax, tol, degree);
    } catch (const std::exception &e) {
        return fail(SC_EINVAL, std::string("thermo interpolation: ") + e.what());
    }
    if (degree_out) *degree_out = f.degree;
    if (nint_out) *nint_out = f.nint;
    if (max_err_out) *max_err_out = f.max_err;
    if (ncoef) {
        if (coef) std::copy_n(f.coef.begin(), std::min(*ncoef, f.coef.size()), coef);
        *ncoef = f.coef.size();
    }
    return SC_OK;
}

sc_status sc_mech_sparse_array(const sc_mech *mech, const char *name, void *out, size_t *bytes)
{
    if (!mech || !name || !bytes) return fail(SC_EINVAL, "NULL argument");
    const sc::SparseLU &s = mech->m.sp;
    const void *src = nullptr;
    size_t sz = 0;
    auto take = [&](const auto &v) {
        src = v.data();
        sz = v.size() * sizeof(v[0]);
    };
    const std::string k(name);
    if (k == "perm") take(s.perm);
    else if (k == "pattern") take(mech->m.pattern);
    else if (k == "apat") take(s.apat);
    else if (k == "erow") take(s.erow);
    else if (k == "ecol") take(s.ecol);
    else if (k == "lu_b_lvl") take(s.lu_b_lvl);
    else if (k == "lu_c_lvl") take(s.lu_c_lvl);
    else if (k == "lu_b") take(s.lu_b);
    else if (k == "lu_c") take(s.lu_c);
    else if (k == "lu_u") take(s.lu_u);
    else if (k == "diag") take(s.diag);
    else if (k == "fw_lvl") take(s.fw_lvl);
    else if (k == "bw_lvl") take(s.bw_lvl);
    else if (k == "tfw_lvl") take(s.tfw_lvl);
    else if (k == "tbw_lvl") take(s.tbw_lvl);
    else if (k == "fw") take(s.fw);
    else if (k == "bw") take(s.bw);
    else if (k == "tfw") take(s.tfw);
    else if (k == "tbw") take(s.tbw);
    else if (k == "rxi") take(s.rxi);
    else if (k == "cstart") take(s.cstart);
    else if (k == "cmask") take(s.cmask);
    else if (k == "sweep_f") take(s.sweep_f);
    else if (k == "sweep_b") take(s.sweep_b);
    else if (k == "sweep_fi") take(s.sweep_fi);
    else if (k == "sweep_bi") take(s.sweep_bi);
    else return fail(SC_EINVAL, "unknown sparse array " + k);
    if (out && sz) std::memcpy(out, src, std::min(sz, *bytes));
    *bytes = sz;
    return SC_OK;
}

sc_status sc_species_index(const sc_mech *mech, const char *name, int32_t *idx)
{
    if (!mech || !name || !idx) return fail(SC_EINVAL, "NULL argument");
    int k = mech->m.species(name);
    if (k < 0) return fail(SC_EINVAL, std::string("unknown species ") + name);
    *idx = k;
    return SC_OK;
}

sc_status sc_plan_create(const sc_mech *mech, int device, const sc_options *opt, sc_plan **out)
{
    if (!out) return fail(SC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mech) return fail(SC_EINVAL, "mech is NULL");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(SC_EHIP, "no HIP device");
    if (device < 0 || device >= ndev) return fail(SC_EINVAL, "device index out of range");
    sc_options o;
    sc_default_options(&o);
    if (opt) o = *opt;
    if (!(o.rtol > 0) || !(o.atol > 0) || !std::isfinite(o.rtol) || !std::isfinite(o.atol))
        return fail(SC_EINVAL, "rtol and atol must be positive and finite");
    if (o.max_steps <= 0) return fail(SC_EINVAL, "max_steps must be positive");
    if (o.mode != SC_MODE_PLAIN && o.mode != SC_MODE_PERSISTENT && o.mode != SC_MODE_STATIC)
        return fail(SC_EINVAL, "unknown mode");
    if (o.order < SC_ORDER_NONE || o.order > SC_ORDER_COST) return fail(SC_EINVAL, "unknown cell order");
    if (o.tile <= 0) o.tile = 1;
    if (o.grid < 0) return fail(SC_EINVAL, "grid must be >= 0");
    if (o.fixed_step != 0 && o.fixed_step != 1) return fail(SC_EINVAL, "fixed_step must be 0 or 1");
    if (!(o.hmax_frac >= 0.0) || !std::isfinite(o.hmax_frac)) return fail(SC_EINVAL, "hmax_frac must be >= 0");
    if (o.reactor != SC_REACTOR_CONST_P && o.reactor != SC_REACTOR_CONST_V) return fail(SC_EINVAL, "unknown reactor");
    if (o.method != SC_METHOD_ROS4 && o.method != SC_METHOD_EXTRAP) return fail(SC_EINVAL, "unknown method");
    if (o.linalg != SC_LINALG_AUTO && o.linalg != SC_LINALG_DENSE && o.linalg != SC_LINALG_SPARSE)
        return fail(SC_EINVAL, "unknown linalg");
    const int nstate = mech->m.N + 1;
    const bool sparse = o.linalg == SC_LINALG_SPARSE || (o.linalg == SC_LINALG_AUTO && nstate > sc::MAX_STATE);
    if (!sparse && nstate > sc::MAX_STATE)
        return fail(SC_EUNSUPPORTED, "the dense linear algebra supports up to " + std::to_string(sc::MAX_STATE - 1) +
                                         " species; use the sparse one (linalg = SC_LINALG_SPARSE or AUTO)");
    if (sparse && o.method != SC_METHOD_ROS4)
        return fail(SC_EUNSUPPORTED, "the extrapolation baseline runs with the dense linear algebra only");
    if (!(o.thermo_tol >= 0.0) || !std::isfinite(o.thermo_tol)) return fail(SC_EINVAL, "thermo_tol must be >= 0");
    if (o.thermo_tol > 0.0 && !sparse)
        return fail(SC_EUNSUPPORTED, "interpolated thermodynamics run with the sparse linear algebra only");
    sc::ThermoFit fit;
    if (o.thermo_tol > 0.0) {
        try {
            fit = sc::fit_thermo(mech->m, o.thermo_Tmin, o.thermo_Tmax, o.thermo_tol, o.thermo_degree);
        } catch (const std::exception &e) {
            return fail(SC_EINVAL, std::string("thermo interpolation: ") + e.what());
        }
    }
    const sc::SparseLU &S = mech->m.sp;
    // the sparse kernels' vectors hold every position of the bordered
    // system (N + 2 of them) in one or two slots per lane
    const int vpl = S.n <= 64 ? 1 : 2;
    // cells per wave: each cell's group of 64 / cpw lanes must hold the N + 2 positions
    const int cpw_max = !sparse ? 1 : S.n <= 16 ? 4 : S.n <= 32 ? 2 : 1;
    if (o.cells_per_wave != 0 && o.cells_per_wave != 1 && o.cells_per_wave != 2 && o.cells_per_wave != 4)
        return fail(SC_EINVAL, "cells_per_wave must be 0, 1, 2 or 4");
    if (o.cells_per_wave > cpw_max)
        return fail(SC_EINVAL, "cells_per_wave " + std::to_string(o.cells_per_wave) + " needs the sparse linear "
                               "algebra and N + 2 <= " + std::to_string(64 / o.cells_per_wave) + " positions");
    const int cpw = o.cells_per_wave ? o.cells_per_wave : cpw_max;
    scdev::DevSparse ds{};
    if (sparse) {
        const int NV = 64 / cpw * vpl;
        ds.cpw = cpw;
        ds.n = S.n;
        ds.nnz = S.nnz;
        ds.nl_lu = (int)S.lu_b_lvl.size() - 1;
        ds.nl_fw = (int)S.fw_lvl.size() - 1;
        ds.nl_bw = (int)S.bw_lvl.size() - 1;
        ds.n_u = (int)S.lu_u.size();
        ds.tail0 = S.tail0;
        ds.NV = NV;
        ds.E = 0;
        ds.C = S.nnz + 1;  // E[nnz]: a slot kept at zero (the table sweeps' entry for rows without one)
        ds.G = ds.C + NV;
        ds.H = ds.G + NV;
        ds.WD = ds.H + NV;
        ds.UA = ds.WD + NV;
        ds.U = ds.UA + NV;
        ds.X = ds.U + 4 * NV;
        ds.DINV = ds.X + S.n;
        ds.size = ds.DINV + S.n;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(SC_EHIP, "hipGetDeviceProperties failed");
        // the register tail: at most sparse_tail_max(n) rows, and no more than a cell's lanes
        if (S.n - S.tail0 > std::min(sc::sparse_tail_max(S.n), 64 / cpw))
            return fail(SC_EUNSUPPORTED, "dense LU tail wider than a cell's lanes");
        if (sizeof(double) * (size_t)ds.size * cpw > prop.sharedMemPerBlock)
            return fail(SC_EUNSUPPORTED, "the sparse factors of this mechanism need " +
                                             std::to_string(sizeof(double) * ds.size) +
                                             " bytes of LDS per cell; the device has " +
                                             std::to_string(prop.sharedMemPerBlock));
    }
    DeviceGuard g(device);
    if (!g.ok) return fail(SC_EHIP, "hipSetDevice failed");
    sc_plan *p = nullptr;
    try {
        p = new sc_plan();
        p->m = mech->m;
    } catch (...) {
        delete p;
        return fail(SC_ENOMEM, "host allocation failed");
    }
    p->opt = o;
    p->device = device;
    p->np = p->m.n_padded;
    const sc::Tables &t = p->m.tab;
    scdev::DevMech &d = p->dm;
    d.N = t.N;
    d.R = t.R;
    d.nt = t.n_troe;
    d.cv = o.reactor == SC_REACTOR_CONST_V ? 1 : 0;
    d.Rgas = t.Rgas;
    d.lnp0R = std::log(t.p0 / t.Rgas);
    // species table, reaction records, Troe records
    std::vector<double> spv;
    spv.reserve(9 * (size_t)t.N);
    spv.insert(spv.end(), t.W.begin(), t.W.end());
    spv.insert(spv.end(), t.invW.begin(), t.invW.end());
    spv.insert(spv.end(), t.nasa.begin(), t.nasa.end());
    // execution order: plain, third-body, Troe; then by side sizes, so that
    // the 64 reactions of a pass take the same branches (the original index
    // is kept for per-reaction inputs)
    std::vector<int> order(t.R);
    for (int j = 0; j < t.R; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        auto key = [&](int j) { return std::make_tuple(t.kind[j], t.neff[j] > 0, t.nr[j] + t.np[j]); };
        return key(x) < key(y);
    });
    std::vector<scdev::RxRec> rx(t.R);
    for (int q = 0; q < t.R; ++q) {
        const int j = order[q];
        scdev::RxRec &r = rx[q];
        std::memset(&r, 0, sizeof r);
        r.lnA = t.lnA[j];
        r.b = t.b[j];
        r.EaR = t.EaR[j];
        r.kind = t.kind[j];
        r.nr = t.nr[j];
        r.np = t.np[j];
        r.dnu = t.dnu[j];
        r.neff = t.neff[j];
        r.tix = t.tix[j];
        for (int i = 0; i < sc::MAXSIDE; ++i) {
            r.rsp[i] = t.rsp[i * t.R + j];
            r.rnu[i] = t.rnu[i * t.R + j];
            r.psp[i] = t.psp[i * t.R + j];
            r.pnu[i] = t.pnu[i * t.R + j];
        }
        for (int e = 0; e < sc::MAXENH; ++e) {
            r.esp[e] = t.esp[e * t.R + j];
            r.eam1[e] = t.eam1[e * t.R + j];
        }
        r.orig = j;
    }
    std::vector<scdev::TroeRec> tr(t.n_troe > 0 ? t.n_troe : 1);
    for (int k = 0; k < t.n_troe; ++k) {
        const int nt = t.n_troe;
        tr[k] = scdev::TroeRec{t.troe[0 * nt + k], t.troe[1 * nt + k], t.troe[2 * nt + k], t.troe[3 * nt + k],
                               t.troe[4 * nt + k], t.troe[5 * nt + k], t.troe[6 * nt + k], 0.0};
    }
    bool ok = upload(p, spv, &d.sp) && upload(p, rx, &d.rx) && upload(p, tr, &d.troe);
    if (ok && fit.nint > 0) {
        // the table in the records' execution order: the 64 lanes of a pass
        // read 64 consecutive coefficient blocks of the cell's interval
        const int nc = 2 * (fit.degree + 1);
        std::vector<double> tab(fit.coef.size());
        for (int iv = 0; iv < fit.nint; ++iv)
            for (int q = 0; q < t.R; ++q)
                std::copy_n(&fit.coef[((size_t)iv * t.R + order[q]) * nc], nc, &tab[((size_t)iv * t.R + q) * nc]);
        ok = upload(p, tab, &ds.itab);
        ds.ideg = fit.degree;
        ds.inint = fit.nint;
        ds.iu0 = fit.u0;
        ds.iinvdu = 1.0 / fit.du;
    }
    p->sparse = sparse;
    p->vpl = vpl;
    p->ds = ds;
    if (ok && sparse) {
        const int N = t.N;
        // per-reaction entry indices in the execution order of the records
        std::vector<uint16_t> rxi((size_t)t.R * sc::RXI_SIZE);
        for (int q = 0; q < t.R; ++q)
            std::memcpy(&rxi[(size_t)q * sc::RXI_SIZE], &S.rxi[(size_t)order[q] * sc::RXI_SIZE],
                        sizeof(uint16_t) * sc::RXI_SIZE);
        std::vector<int32_t> comp((size_t)scdev::CMP * (N + 1), -1);
        for (int k = 0; k < N; ++k) {
            int32_t *c = &comp[(size_t)scdev::CMP * k];
            c[0] = S.pos[k];
            c[1] = S.e_kk[k];
            c[2] = S.e_kT[k];
            c[3] = S.e_kS[k];
            c[4] = S.e_Tk[k];
            c[5] = S.e_Sk[k];
        }
        comp[(size_t)scdev::CMP * N] = S.pos[N];
        comp[(size_t)scdev::CMP * N + 1] = S.e_TT;
        comp[(size_t)scdev::CMP * N + 2] = S.e_SS;
        std::vector<uint16_t> emap(S.emap.size());
        for (size_t i = 0; i < emap.size(); ++i) emap[i] = S.emap[i] < 0 ? sc::NOENT : (uint16_t)S.emap[i];
        scdev::DevSparse &q = p->ds;
        std::vector<uint64_t> lu_b(S.lu_b.begin(), S.lu_b.end());
        ok = upload(p, S.lu_b_lvl, &q.lu_b_lvl) && upload(p, S.lu_c_lvl, &q.lu_c_lvl) &&
             upload(p, S.fw_lvl, &q.fw_lvl) && upload(p, S.bw_lvl, &q.bw_lvl) && upload(p, lu_b, &q.lu_b) &&
             upload(p, S.lu_u, &q.lu_u) && upload(p, S.diag, &q.diag) && upload(p, S.lu_c, &q.lu_c) &&
             upload(p, S.fw, &q.fw) && upload(p, S.bw, &q.bw) && upload(p, rxi, &q.rxi) &&
             upload(p, comp, &q.comp) && upload(p, emap, &q.emap) && upload(p, S.cstart, &q.cstart) &&
             upload(p, S.cmask, &q.cmask) && upload(p, S.sweep_f, &q.swf) && upload(p, S.sweep_b, &q.swb) &&
             upload(p, S.sweep_fi, &q.swfi) && upload(p, S.sweep_bi, &q.swbi);
    }
    if (ok) {
        void *q = nullptr;
        ok = hipMalloc(&q, sizeof(unsigned long long)) == hipSuccess;
        if (ok) {
            p->allocs.push_back(q);
            p->queue = static_cast<unsigned long long *>(q);
        }
    }
    if (!ok) {
        release(p);
        delete p;
        return fail(SC_ENOMEM, "device allocation/upload failed");
    }
    p->capacity = sparse ? scdev::persistent_capacity_sp(vpl, p->ds, device) : scdev::persistent_capacity(p->np, device);
    p->adj_capacity = nstate <= sc::MAX_STATE ? scdev::adjoint_capacity(p->np, d.R, device) : 0;
    *out = p;
    return SC_OK;
}

void sc_plan_free(sc_plan *plan)
{
    if (!plan) return;
    release(plan);
    delete plan;
}

sc_status sc_rhs(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y, int64_t ld,
                 const double *dlnA, double *fT, double *fY, void *stream)
{
    sc_status s = check_common(plan, n, ld, {T, p, Y, fT, fY});
    if (s != SC_OK || n == 0) return s;
    DeviceGuard g(plan->device);
    hipError_t e =
        plan->sparse
            ? scdev::launch_rhs_sp(plan->vpl, plan->dm, plan->ds, n, T, p, Y, ld, dlnA, fT, fY, (hipStream_t)stream)
            : scdev::launch_rhs(plan->np, plan->dm, n, T, p, Y, ld, dlnA, fT, fY, (hipStream_t)stream);
    return e == hipSuccess ? SC_OK : hip_fail(e, "rhs launch");
}

sc_status sc_jacobian(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y, int64_t ld,
                      const double *dlnA, double *J, void *stream)
{
    sc_status s = check_common(plan, n, ld, {T, p, Y, J});
    if (s != SC_OK || n == 0) return s;
    DeviceGuard g(plan->device);
    hipError_t e = plan->sparse
                       ? scdev::launch_jac_sp(plan->vpl, plan->dm, plan->ds, n, T, p, Y, ld, dlnA, J,
                                              (hipStream_t)stream)
                       : scdev::launch_jac(plan->np, plan->dm, n, T, p, Y, ld, dlnA, J, (hipStream_t)stream);
    return e == hipSuccess ? SC_OK : hip_fail(e, "jacobian launch");
}

sc_status sc_linsolve(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y, int64_t ld,
                      const double *dlnA, const double *hg, const double *b, double *x, void *stream)
{
    sc_status s = check_common(plan, n, ld, {T, p, Y, hg, b, x});
    if (s != SC_OK || n == 0) return s;
    DeviceGuard g(plan->device);
    hipError_t e = plan->sparse ? scdev::launch_linsolve_sp(plan->vpl, plan->dm, plan->ds, n, T, p, Y, ld, dlnA, hg,
                                                            b, x, (hipStream_t)stream)
                                : scdev::launch_linsolve(plan->np, plan->dm, n, T, p, Y, ld, dlnA, hg, b, x,
                                                         (hipStream_t)stream);
    return e == hipSuccess ? SC_OK : hip_fail(e, "linsolve launch");
}

// sc_integrate and its allocation-free variant: with `noalloc` the queue
// counter and the ordering workspace come from the library's fixed device
// scratch instead of the plan's allocations.
// With `ref`, the cells whose ref is another cell are skipped (mapped
// afterwards by the caller).
static sc_status integrate_impl(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0, int64_t ld,
                         const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                         int32_t *cell_status, int32_t *n_acc, int32_t *n_rej, void *stream, bool noalloc,
                         const int32_t *ref = nullptr)
{
    sc_status s = check_common(plan, n, ld, {T0, p, Y0, dt, T1, Y1, cell_status});
    if (s != SC_OK || n == 0) return s;
    if (plan->opt.fixed_step && !h_io) return fail(SC_EINVAL, "fixed_step needs h_io (the step of each cell)");
    if (plan->opt.mode == SC_MODE_PERSISTENT && plan->opt.order == SC_ORDER_COST && (!n_acc || !n_rej))
        return fail(SC_EINVAL, "cost ordering needs the previous n_acc and n_rej");
    DeviceGuard g(plan->device);
    const scdev::Opts o = dev_opts(plan->opt);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    unsigned long long *queue = plan->queue;
    char *ows = nullptr;  // ordering workspace in the fixed scratch
    size_t ows_bytes = 0;
    if (noalloc && plan->opt.mode == SC_MODE_PERSISTENT) {
        void *base = nullptr;
        size_t bytes = 0;
        int64_t max_cells = 0;
        e = scdev::noalloc_scratch(plan->device, &base, &bytes, &max_cells);
        if (e != hipSuccess) return hip_fail(e, "device scratch address");
        if (n > max_cells)
            return fail(SC_EINVAL, "sc_integrate_noalloc: n = " + std::to_string(n) + " exceeds its limit of " +
                                       std::to_string(max_cells) + " cells");
        queue = static_cast<unsigned long long *>(base);
        ows = static_cast<char *>(base) + 256;
        ows_bytes = bytes - 256;
        if (plan->opt.order != SC_ORDER_NONE) {
            size_t need = 0;
            e = scdev::order_ws_need(plan->opt.order, n, &need, st);
            if (e != hipSuccess) return hip_fail(e, "ordering workspace size");
            if (need > ows_bytes)
                return fail(SC_EINVAL, "sc_integrate_noalloc: the cell ordering of n = " + std::to_string(n) +
                                           " cells needs more than the fixed scratch holds");
        }
    }
    if (plan->opt.mode == SC_MODE_PERSISTENT) {
        const int tile = plan->opt.tile;
        const int64_t per_pull = (int64_t)tile * (plan->sparse ? plan->ds.cpw : 1);  // cells one wave takes per pull
        int64_t tiles = (n + per_pull - 1) / per_pull;
        int grid = plan->opt.grid > 0 ? plan->opt.grid : plan->capacity;
        if (grid <= 0) grid = 1;
        if (grid > tiles) grid = (int)tiles;
        int32_t *perm = nullptr;
        if (plan->opt.order != SC_ORDER_NONE) {
            if (noalloc)
                e = scdev::order_cells_in(plan->opt.order, n, dt, n_acc, n_rej, ows, ows_bytes, &perm, st);
            else
                e = scdev::order_cells(plan->opt.order, n, dt, n_acc, n_rej, &plan->order_ws, &plan->order_ws_bytes,
                                       &perm, st);
            if (e != hipSuccess) return hip_fail(e, "cell ordering");
        }
        e = scdev::launch_zero_u64(queue, st);
        if (e == hipSuccess && plan->sparse)
            e = scdev::launch_integrate_sp_persistent(plan->vpl, plan->dm, plan->ds, o, n, T0, p, Y0, ld, dt, dlnA,
                                                      h_io, T1, Y1, cell_status, n_acc, n_rej, queue, perm, tile,
                                                      grid, ref, st);
        else if (e == hipSuccess)
            e = scdev::launch_integrate_persistent(plan->np, plan->dm, o, plan->opt.method, n, T0, p, Y0, ld, dt,
                                                   dlnA, h_io, T1, Y1, cell_status, n_acc, n_rej, queue, perm, tile,
                                                   grid, ref, st);
    } else if (plan->opt.mode == SC_MODE_STATIC) {
        int grid = plan->opt.grid > 0 ? plan->opt.grid : plan->capacity;
        if (grid <= 0) grid = 1;
        if (grid > n) grid = (int)n;
        if (plan->sparse)
            e = scdev::launch_integrate_sp_static(plan->vpl, plan->dm, plan->ds, o, n, T0, p, Y0, ld, dt, dlnA, h_io,
                                                  T1, Y1, cell_status, n_acc, n_rej, grid, ref, st);
        else
            e = scdev::launch_integrate_static(plan->np, plan->dm, o, plan->opt.method, n, T0, p, Y0, ld, dt, dlnA,
                                               h_io, T1, Y1, cell_status, n_acc, n_rej, grid, ref, st);
    } else if (plan->sparse) {
        e = scdev::launch_integrate_sp(plan->vpl, plan->dm, plan->ds, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1,
                                       cell_status, n_acc, n_rej, ref, st);
    } else {
        e = scdev::launch_integrate(plan->np, plan->dm, o, plan->opt.method, n, T0, p, Y0, ld, dt, dlnA, h_io, T1,
                                    Y1, cell_status, n_acc, n_rej, ref, st);
    }
    return e == hipSuccess ? SC_OK : hip_fail(e, "integrate launch");
}

sc_status sc_integrate(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0, int64_t ld,
                       const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                       int32_t *cell_status, int32_t *n_acc, int32_t *n_rej, void *stream)
{
    return integrate_impl(plan, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, cell_status, n_acc, n_rej, stream, false);
}

sc_status sc_integrate_noalloc(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0,
                               int64_t ld, const double *dt, const double *dlnA, double *h_io, double *T1,
                               double *Y1, int32_t *cell_status, int32_t *n_acc, int32_t *n_rej, void *stream)
{
    return integrate_impl(plan, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, cell_status, n_acc, n_rej, stream, true);
}

sc_status sc_plan_set_mapping(sc_plan *plan, const double *Y_fuel, const double *Y_ox, const sc_mapping *opt)
{
    if (!plan || !Y_fuel || !Y_ox || !opt) return fail(SC_EINVAL, "NULL argument");
    const sc::Mech &m = plan->m;
    const int N = m.N;
    if (!std::isfinite(opt->z_tol)) return fail(SC_EINVAL, "z_tol must be finite");
    if (!(opt->dT > 0.0) || !std::isfinite(opt->dT)) return fail(SC_EINVAL, "dT must be positive");
    if (!(opt->dlnp >= 0.0) || !std::isfinite(opt->dlnp)) return fail(SC_EINVAL, "dlnp must be >= 0");
    for (int k = 0; k < N; ++k)
        if (!std::isfinite(Y_fuel[k]) || !std::isfinite(Y_ox[k]))
            return fail(SC_EINVAL, "stream compositions must be finite");
    // Bilger's coupling function per unit mass: carbon 2, hydrogen 1/2,
    // oxygen -1 mole per mole of atoms; other elements do not count
    std::vector<double> w(N, 0.0);
    for (int e = 0; e < m.E; ++e) {
        const std::string &el = m.elements[e];
        const double a = el == "C" ? 2.0 : el == "H" ? 0.5 : el == "O" ? -1.0 : 0.0;
        if (a != 0.0)
            for (int k = 0; k < N; ++k) w[k] += a * m.comp[(size_t)k * m.E + e];
    }
    for (int k = 0; k < N; ++k) w[k] /= m.W[k];
    double bf = 0.0, bo = 0.0;
    for (int k = 0; k < N; ++k) {
        const double tf = w[k] * Y_fuel[k];
        bf = bf + tf;
        const double to = w[k] * Y_ox[k];
        bo = bo + to;
    }
    if (!(bf != bo) || !std::isfinite(bf - bo))
        return fail(SC_EINVAL, "fuel and oxidiser streams have the same coupling function");
    const double nT = std::ceil(SC_MAP_T_MAX / opt->dT);
    const double np = opt->dlnp > 0.0 ? std::ceil(std::log(SC_MAP_P_MAX) / opt->dlnp) : 1.0;
    if (nT * np > (double)(1 << 24))
        return fail(SC_EINVAL, "dT and dlnp give more than 2^24 zones");
    DeviceGuard g(plan->device);
    if (!plan->mapping) {
        // weights and the largest table, allocated once per plan
        void *dw = nullptr, *dt = nullptr;
        if (hipMalloc(&dw, sizeof(double) * (size_t)N) != hipSuccess) return fail(SC_ENOMEM, "mapping weights");
        plan->allocs.push_back(dw);
        if (hipMalloc(&dt, sizeof(int32_t) << 24) != hipSuccess) return fail(SC_ENOMEM, "mapping zone table");
        plan->allocs.push_back(dt);
        plan->mp.w = static_cast<const double *>(dw);
        plan->mp.table = static_cast<int32_t *>(dt);
    }
    if (hipMemcpy(const_cast<double *>(plan->mp.w), w.data(), sizeof(double) * (size_t)N, hipMemcpyHostToDevice) !=
        hipSuccess)
        return fail(SC_EHIP, "mapping weights upload");
    plan->mp.beta_ox = bo;
    plan->mp.dbeta = bf - bo;
    plan->mp.z_tol = opt->z_tol;
    plan->mp.dT = opt->dT;
    plan->mp.dlnp = opt->dlnp;
    plan->mp.nT = (int)nT;
    plan->mp.np = (int)np;
    plan->mapping = true;
    return SC_OK;
}

sc_status sc_integrate_mapped(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0,
                              int64_t ld, const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                              int32_t *cell_status, int32_t *n_acc, int32_t *n_rej, int32_t *ref, void *stream)
{
    sc_status s = check_common(plan, n, ld, {T0, p, Y0, dt, T1, Y1, cell_status, ref});
    if (s != SC_OK) return s;
    if (!plan->mapping) return fail(SC_EINVAL, "sc_plan_set_mapping has not been called on this plan");
    if (T1 == T0 || Y1 == Y0)
        return fail(SC_EINVAL, "the mapped integration needs T1, Y1 apart from T0, Y0 (mapped cells add the "
                               "reference's change to their inputs)");
    if (n == 0) return SC_OK;
    DeviceGuard g(plan->device);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = scdev::launch_map_classify(plan->mp, plan->m.N, n, T0, p, Y0, ld, dt, ref, st);
    if (e != hipSuccess) return hip_fail(e, "mapping classification");
    s = integrate_impl(plan, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, cell_status, n_acc, n_rej, stream, false, ref);
    if (s != SC_OK) return s;
    e = scdev::launch_map_apply(plan->m.N, n, ref, T0, Y0, ld, dt, T1, Y1, cell_status, n_acc, n_rej, st);
    return e == hipSuccess ? SC_OK : hip_fail(e, "mapping");
}

sc_status sc_vjp(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y, int64_t ld,
                 const double *dlnA, const double *wT, const double *wY, double *gT, double *gY,
                 double *g_dlnA_cell, void *stream)
{
    sc_status s = check_common(plan, n, ld, {T, p, Y, wT, wY, gT, gY});
    if (s != SC_OK) return s;
    if (plan->dm.cv) return fail(SC_EUNSUPPORTED, "the VJP supports the constant-pressure reactor only");
    if (plan->ds.itab)
        return fail(SC_EUNSUPPORTED, "the VJP follows the exact thermodynamics: create the plan with thermo_tol = 0");
    if (plan->m.N + 1 > sc::MAX_STATE)
        return fail(SC_EUNSUPPORTED, "the VJP supports up to " + std::to_string(sc::MAX_STATE - 1) + " species");
    if (n == 0) return SC_OK;
    DeviceGuard g(plan->device);
    hipError_t e = scdev::launch_vjp(plan->np, plan->dm, n, T, p, Y, ld, dlnA, wT, wY, gT, gY, g_dlnA_cell,
                                     (hipStream_t)stream);
    return e == hipSuccess ? SC_OK : hip_fail(e, "vjp launch");
}

size_t sc_adjoint_slot_bytes(const sc_plan *plan)
{
    if (!plan) return 0;
    const int64_t hcap = ((int64_t)plan->opt.max_steps + 31) / 32 * 32;
    const int nck = scdev::adjoint_slot_checkpoints();
    int64_t kmax = 1;
    while ((int64_t)nck * kmax < plan->opt.max_steps) kmax *= 2;
    return sizeof(double) * (size_t)(hcap + (int64_t)(nck + kmax - 1) * 64);
}

sc_status sc_adjoint(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0, int64_t ld,
                     const double *dt, const double *dlnA, const double *h0, const double *gT1, const double *gY1,
                     double *gT0, double *gY0, double *g_dlnA, double *g_dlnA_cell, const int32_t *cost,
                     double *T1, double *Y1, int32_t *cell_status, int32_t *n_acc, size_t budget_bytes,
                     size_t *peak_bytes, void *stream)
{
    if (peak_bytes) *peak_bytes = 0;
    sc_status s = check_common(plan, n, ld, {T0, p, Y0, dt, gT1, gY1, gT0, gY0, cell_status});
    if (s != SC_OK) return s;
    if (plan->dm.cv) return fail(SC_EUNSUPPORTED, "the adjoint supports the constant-pressure reactor only");
    if (plan->ds.itab)
        return fail(SC_EUNSUPPORTED, "the adjoint follows the exact thermodynamics: create the plan with thermo_tol = 0");
    if (plan->opt.method != SC_METHOD_ROS4)
        return fail(SC_EUNSUPPORTED, "the adjoint supports the Rosenbrock method only");
    if (plan->m.N + 1 > sc::MAX_STATE)
        return fail(SC_EUNSUPPORTED, "the adjoint supports up to " + std::to_string(sc::MAX_STATE - 1) + " species");
    const int R = plan->dm.R;
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard g(plan->device);
    if (n == 0) {
        if (g_dlnA && R > 0) {  // an empty sum: zeros, written by a kernel
            hipError_t e = scdev::launch_sum_cells(nullptr, 0, R, g_dlnA, st);
            if (e != hipSuccess) return hip_fail(e, "clear g_dlnA");
        }
        return SC_OK;
    }
    if (plan->opt.fixed_step && !h0) return fail(SC_EINVAL, "fixed_step needs h0 (the step of each cell)");
    if (budget_bytes == 0) budget_bytes = (size_t)8 << 30;
    const scdev::Opts o = dev_opts(plan->opt);
    // per-cell parameter adjoints: the caller's array, else a plan workspace
    double *gcell = g_dlnA_cell;
    size_t used = 0;
    const size_t gcell_bytes = sizeof(double) * (size_t)R * (size_t)n;
    if (!gcell && g_dlnA && R > 0) used += gcell_bytes;
    const size_t slot = sc_adjoint_slot_bytes(plan);
    if (used + slot > budget_bytes)
        return fail(SC_EBUDGET, "adjoint workspace of one wave (" + std::to_string(slot) +
                                    " bytes) exceeds the budget; lower max_steps or raise the budget");
    int grid = plan->adj_capacity > 0 ? plan->adj_capacity : 1;
    if (plan->opt.grid > 0 && plan->opt.grid < grid) grid = plan->opt.grid;
    if (grid > n) grid = (int)n;
    const size_t fit = (budget_bytes - used) / slot;
    if ((size_t)grid > fit) grid = (int)fit;
    hipError_t e = grow(&plan->adj_ws, &plan->adj_ws_bytes, slot * (size_t)grid);
    if (e != hipSuccess) return hip_fail(e, "adjoint workspace");
    used += slot * (size_t)grid;
    if (!gcell && g_dlnA && R > 0) {
        e = grow(&plan->gcell_ws, &plan->gcell_ws_bytes, gcell_bytes);
        if (e != hipSuccess) return hip_fail(e, "parameter-adjoint workspace");
        gcell = static_cast<double *>(plan->gcell_ws);
    }
    int32_t *perm = nullptr;
    if (cost) {
        e = scdev::order_cells(SC_ORDER_COST, n, dt, cost, nullptr, &plan->order_ws, &plan->order_ws_bytes, &perm,
                               st);
        if (e != hipSuccess) return hip_fail(e, "cell ordering");
        used += plan->order_ws_bytes;
    }
    e = scdev::launch_zero_u64(plan->queue, st);
    if (e != hipSuccess) return hip_fail(e, "queue reset");
    const int64_t hcap = ((int64_t)plan->opt.max_steps + 31) / 32 * 32;
    e = scdev::launch_adjoint(plan->np, plan->dm, o, n, T0, p, Y0, ld, dt, dlnA, h0, gT1, gY1, gT0, gY0, gcell,
                              cell_status, n_acc, T1, Y1, static_cast<double *>(plan->adj_ws),
                              (int64_t)(slot / sizeof(double)), (int)hcap, plan->queue, perm, grid, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    if (g_dlnA && R > 0) {
        e = scdev::launch_sum_cells(gcell, n, R, g_dlnA, st);
        if (e != hipSuccess) return hip_fail(e, "parameter-adjoint reduction");
    }
    if (peak_bytes) *peak_bytes = used;
    return SC_OK;
}

sc_status sc_transport2d(int32_t nx, int32_t ny, int32_t ncomp, const double *in, int64_t ld, const double *u,
                         const double *dt, double dx, double diffusivity, const double *inflow, double *out,
                         void *stream)
{
    if (nx <= 0 || ny <= 0 || ncomp <= 0) return fail(SC_EINVAL, "nx, ny and ncomp must be positive");
    // one thread per value in 256-thread blocks on a one-dimensional grid,
    // whose x dimension holds at most 2^31 - 1 blocks
    if ((int64_t)nx * ny * ncomp > (((int64_t)1 << 31) - 1) * 256)
        return fail(SC_EINVAL, "nx * ny * ncomp too large for one launch");
    if (ld < (int64_t)nx * ny) return fail(SC_EINVAL, "ld must be >= nx * ny");
    if (!in || !u || !dt || !inflow || !out) return fail(SC_EINVAL, "required array pointer is NULL");
    if (in == out) return fail(SC_EINVAL, "out must not alias in");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(SC_EINVAL, "dx must be positive");
    if (!(diffusivity >= 0.0) || !std::isfinite(diffusivity)) return fail(SC_EINVAL, "diffusivity must be >= 0");
    hipError_t e = scdev::launch_transport2d(nx, ny, ncomp, in, ld, u, dt, dx, diffusivity, inflow, out,
                                             (hipStream_t)stream);
    return e == hipSuccess ? SC_OK : hip_fail(e, "transport launch");
}

}  // extern "C"
