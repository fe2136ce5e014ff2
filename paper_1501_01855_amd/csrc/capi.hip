// extern "C" entry points (include/ovl.h): argument checks, layout packing
// between the canonical complex128 layout and the internal planes, error
// translation.  No exception crosses this boundary.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <thread>
#include <vector>

#include "context.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {
const char *last_error();
}

using namespace ovl;

struct ovl_context : public ovl::Context {};

template <class F>
static ovl_status guard(F &&f)
{
    try {
        f();
        return OVL_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return OVL_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return OVL_ERR_ARG;
    }
}

static void check_prec(int prec, bool allow_half = false)
{
    OVL_REQUIRE(prec == OVL_F64 || prec == OVL_F32 || (allow_half && prec == OVL_HALF), OVL_ERR_ARG,
                "precision must be OVL_F64 or OVL_F32" + std::string(allow_half ? " or OVL_HALF" : ""));
}

static void check_ctx(ovl_context *ctx) { OVL_REQUIRE(ctx != nullptr, OVL_ERR_ARG, "null context"); }

static void check_zolo(const ovl_zolo *z)
{
    OVL_REQUIRE(z != nullptr, OVL_ERR_ARG, "null Zolotarev coefficients");
    OVL_REQUIRE(z->n_z >= 1 && z->n_z <= OVL_MAX_NZ, OVL_ERR_ARG, "n_z out of range");
    for (int l = 0; l < z->n_z; ++l)
        OVL_REQUIRE(z->omega[l] > 0.0 && z->sigma[l] > 0.0 && std::isfinite(z->omega[l]) &&
                        std::isfinite(z->sigma[l]),
                    OVL_ERR_ARG, "Zolotarev omega and sigma must be positive and finite");
}

static constexpr int MAX_NRHS = 16;
static constexpr int MAX_SOLVE_THREADS = 32;   // host threads driving instances at once

extern "C" {

const char *ovl_last_error(void) { return ovl::last_error(); }

void ovl_solver_defaults(ovl_solver_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->rho = 1.4;
    p->mu = 0.05;
    p->tol = 1e-10;
    p->eta_tilde = 1e-3;
    p->relax_floor = 1e-2;
    p->f32_threshold = 1e-6;
    p->half_threshold = 2.0;
    p->norm_restart = 0.1;
    p->max_outer = 16;
    p->max_middle = 2000;
    p->max_mscg = 20000;
    p->use_deflation = 0;
    p->eig_calc = 0;
    p->n_eig = 20;
    p->m_eig = 60;
    p->k_recalc = 25;
    p->verbose = 0;
    p->eig_eps = 1e-4;
    p->delta_split = 0.1;
    p->middle_cg = 0;
}

ovl_status ovl_create(const int32_t dims[4], void *hip_stream, ovl_context **out)
{
    return guard([&] {
        OVL_REQUIRE(dims != nullptr && out != nullptr, OVL_ERR_ARG, "null argument");
        int64_t V = 1;
        for (int m = 0; m < 4; ++m) {
            OVL_REQUIRE(dims[m] >= 2 && dims[m] <= 4096, OVL_ERR_ARG, "lattice extents must be in [2, 4096]");
            V *= dims[m];
        }
        OVL_REQUIRE(V < (int64_t)1 << 30, OVL_ERR_ARG, "lattice volume must be below 2^30 sites");
        auto *c = new ovl_context();
        c->g = make_geom(dims);
        c->stream = (hipStream_t)hip_stream;
        hipError_t e = hipGetDevice(&c->device);
        if (e != hipSuccess) {
            delete c;
            throw Error{OVL_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)};
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
            c->num_cu = ncu;
        noalloc_scratch_init(c->device);   // once per device, with it current
        *out = c;
    });
}

ovl_status ovl_destroy(ovl_context *ctx)
{
    return guard([&] { delete ctx; });
}

int64_t ovl_device_bytes(const ovl_context *ctx) { return ctx ? ctx->bytes_held : 0; }

ovl_status ovl_gauge_load(ovl_context *ctx, const double *U_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(U_dev != nullptr, OVL_ERR_ARG, "null gauge field");
        pack_gauge(*ctx, U_dev);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_gauge_generate(ovl_context *ctx, uint64_t seed, double eps, double *U_out_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(std::isfinite(eps), OVL_ERR_ARG, "eps must be finite");
        gauge_generate(*ctx, seed, eps, U_out_dev);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_source_generate(ovl_context *ctx, int kind, uint64_t seed, int64_t site, int32_t spin,
                               int32_t colour, double *out_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(out_dev != nullptr, OVL_ERR_ARG, "null output");
        OVL_REQUIRE(kind == OVL_SRC_POINT || kind == OVL_SRC_GAUSS || kind == OVL_SRC_Z2, OVL_ERR_ARG,
                    "unknown source kind");
        if (kind == OVL_SRC_POINT)
            OVL_REQUIRE(site >= 0 && site < ctx->g.V && spin >= 0 && spin < 4 && colour >= 0 && colour < 3,
                        OVL_ERR_ARG, "point source index out of range");
        source_generate(*ctx, kind, seed, site, spin, colour, out_dev);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_wilson_dslash(ovl_context *ctx, const double *in_dev, double *out_dev, int32_t nrhs, int32_t prec)
{
    return guard([&] {
        check_ctx(ctx);
        check_prec(prec, true);
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, prec) * nrhs;
        void *a = ctx->buf("api_a", FB);
        void *b = ctx->buf("api_b", FB);
        pack_spinor(*ctx, in_dev, a, nrhs, prec);
        launch_hop(*ctx, a, b, nrhs, prec);
        unpack_spinor(*ctx, b, out_dev, nrhs, prec);
        ctx->prof_collect();
    });
}

ovl_status ovl_wilson_dslash_noalloc(ovl_context *ctx, const double *in_dev, double *out_dev, int32_t nrhs,
                                     int32_t prec)
{
    return guard([&] {
        check_ctx(ctx);
        check_prec(prec, true);
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t FB = up(field_bytes(ctx->g, prec) * nrhs);
        const size_t TB = prec == OVL_F64 ? 0 : up(field_bytes(ctx->g, OVL_F64) * nrhs);
        OVL_REQUIRE(2 * FB + TB <= (size_t)OVL_NOALLOC_SCRATCH_BYTES, OVL_ERR_ARG,
                    "fields too large for the fixed scratch: " + std::to_string(2 * FB + TB) + " bytes needed, " +
                        std::to_string((size_t)OVL_NOALLOC_SCRATCH_BYTES) + " available");
        unsigned char *base = (unsigned char *)noalloc_scratch(ctx->device);
        void *a = base;
        void *b = base + FB;
        double2 *tmp = TB ? (double2 *)(base + 2 * FB) : nullptr;
        struct Scope {
            Context &c;
            bool prev;
            explicit Scope(Context &cc) : c(cc), prev(cc.no_alloc) { c.no_alloc = true; }
            ~Scope() { c.no_alloc = prev; }
        } scope(*ctx);
        pack_spinor(*ctx, in_dev, a, nrhs, prec, tmp);
        launch_hop(*ctx, a, b, nrhs, prec);
        unpack_spinor(*ctx, b, out_dev, nrhs, prec, tmp);
    });
}

ovl_status ovl_kernel_K_apply(ovl_context *ctx, double rho, const double *in_dev, double *out_dev, int32_t nrhs,
                              int32_t prec)
{
    return guard([&] {
        check_ctx(ctx);
        check_prec(prec, true);
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(std::isfinite(rho), OVL_ERR_ARG, "rho must be finite");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, prec) * nrhs;
        void *a = ctx->buf("api_a", FB);
        void *b = ctx->buf("api_b", FB);
        pack_spinor(*ctx, in_dev, a, nrhs, prec);
        launch_K(*ctx, rho, a, b, nrhs, prec);
        unpack_spinor(*ctx, b, out_dev, nrhs, prec);
        ctx->prof_collect();
    });
}

ovl_status ovl_zolotarev_coeffs(int32_t n_z, double a, double b, ovl_zolo *out_host)
{
    return guard([&] {
        OVL_REQUIRE(out_host != nullptr, OVL_ERR_ARG, "null output");
        zolotarev(n_z, a, b, *out_host);
    });
}

ovl_status ovl_kernel_interval(ovl_context *ctx, double rho, int32_t max_iter, double *lmin_host,
                               double *lmin_err_host, double *lmax_host)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(std::isfinite(rho), OVL_ERR_ARG, "rho must be finite");
        OVL_REQUIRE(max_iter >= 2 && max_iter <= 2000, OVL_ERR_ARG, "max_iter must be in [2, 2000]");
        OVL_REQUIRE(lmin_host != nullptr, OVL_ERR_ARG, "null lmin output");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        kernel_interval(*ctx, rho, max_iter, lmin_host, lmin_err_host, lmax_host);
    });
}

ovl_status ovl_lowmodes_compute(ovl_context *ctx, double rho, int32_t n_low, double tol, double *evals_host,
                                double *lmax_host)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(n_low >= 1 && n_low <= 256, OVL_ERR_ARG, "n_low must be in [1, 256]");
        OVL_REQUIRE(tol > 0.0, OVL_ERR_ARG, "tol must be positive");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        lowmodes_compute(*ctx, rho, n_low, tol, evals_host, lmax_host);
    });
}

ovl_status ovl_lowmodes_set(ovl_context *ctx, int32_t n, const double *evals_host, const double *evecs_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(n >= 0 && n <= 256, OVL_ERR_ARG, "n must be in [0, 256]");
        if (n > 0) OVL_REQUIRE(evals_host && evecs_dev, OVL_ERR_ARG, "null low-mode data");
        ctx->lowmodes_changed();
        if (ctx->low) {
            OVL_HIP(hipStreamSynchronize(ctx->stream));
            OVL_HIP(hipFree(ctx->low));
            ctx->bytes_held -= (int64_t)field_bytes(ctx->g, OVL_F64) * ctx->n_low;
            ctx->low = nullptr;
        }
        ctx->n_low = 0;
        ctx->low_evals.clear();
        if (n == 0) return;
        const size_t FB = field_bytes(ctx->g, OVL_F64);
        OVL_HIP(hipMalloc(&ctx->low, FB * n));
        ctx->bytes_held += (int64_t)FB * n;
        pack_spinor(*ctx, evecs_dev, ctx->low, n, OVL_F64);
        ctx->low_evals.assign(evals_host, evals_host + n);
        ctx->n_low = n;
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_lowmodes_get(ovl_context *ctx, double *evecs_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(evecs_dev != nullptr, OVL_ERR_ARG, "null output");
        if (ctx->n_low > 0) unpack_spinor(*ctx, ctx->low, evecs_dev, ctx->n_low, OVL_F64);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_sign_zolotarev_mscg(ovl_context *ctx, double rho, const ovl_zolo *zolo, const double *in_dev,
                                   double *out_dev, int32_t nrhs, double eta, int32_t prec, ovl_stats *stats_host)
{
    return guard([&] {
        check_ctx(ctx);
        check_prec(prec, true);
        check_zolo(zolo);
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(eta > 0.0 && std::isfinite(rho), OVL_ERR_ARG, "eta must be positive, rho finite");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, prec) * nrhs;
        void *a = ctx->buf("api_a", FB);
        void *b = ctx->buf("api_b", FB);
        pack_spinor(*ctx, in_dev, a, nrhs, prec);
        sign_mscg(*ctx, rho, *zolo, a, b, nrhs, eta, prec, 100000, stats_host);
        unpack_spinor(*ctx, b, out_dev, nrhs, prec);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof_collect();
    });
}

ovl_status ovl_sign_lanczos(ovl_context *ctx, double rho, const ovl_zolo *zolo, const double *in_dev,
                            double *out_dev, int32_t nrhs, double eta, ovl_stats *stats_host)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(zolo != nullptr && zolo->a > 0.0 && zolo->b > zolo->a && std::isfinite(zolo->b), OVL_ERR_ARG,
                    "need the interval 0 < a < b of |K| (zolo->a, zolo->b)");
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(std::isfinite(rho) && eta > 0.0 && eta < 1.0, OVL_ERR_ARG, "need finite rho and 0 < eta < 1");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        ovl_stats st{};
        const auto t0 = std::chrono::steady_clock::now();
        const size_t FB = field_bytes(ctx->g, OVL_F64) * nrhs;
        double2 *a = (double2 *)ctx->buf("api_a", FB);
        double2 *b = (double2 *)ctx->buf("api_b", FB);
        pack_spinor(*ctx, in_dev, a, nrhs, OVL_F64);
        sign_lanczos(*ctx, rho, *zolo, a, b, nrhs, eta, 20000, &st);
        unpack_spinor(*ctx, b, out_dev, nrhs, OVL_F64);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats_host) *stats_host = st;
    });
}

ovl_status ovl_overlap_apply(ovl_context *ctx, double rho, double mu, const ovl_zolo *zolo, const double *in_dev,
                             double *out_dev, int32_t nrhs, double eta, int32_t prec, ovl_stats *stats_host)
{
    return guard([&] {
        check_ctx(ctx);
        check_prec(prec, true);
        check_zolo(zolo);
        OVL_REQUIRE(in_dev && out_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(eta > 0.0 && std::isfinite(rho) && mu >= 0.0 && mu < 1.0, OVL_ERR_ARG,
                    "need eta > 0, finite rho, 0 <= mu < 1");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, OVL_F64) * nrhs;
        double2 *a = (double2 *)ctx->buf("api_a64", FB);
        double2 *b = (double2 *)ctx->buf("api_b64", FB);
        pack_spinor(*ctx, in_dev, a, nrhs, OVL_F64);
        overlap_f64(*ctx, rho, mu, *zolo, a, b, nrhs, eta, prec, 100000, stats_host);
        unpack_spinor(*ctx, b, out_dev, nrhs, OVL_F64);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof_collect();
    });
}

ovl_status ovl_overlap_adjoint(ovl_context *ctx, double rho, double mu, const ovl_zolo *zolo,
                               const double *psi_dev, const double *chi_dev, int32_t nrhs, double eta,
                               int32_t prec, double *dS_dpsi_dev, double *dS_dU_dev, ovl_stats *stats_host)
{
    return guard([&] {
        check_ctx(ctx);
        check_zolo(zolo);
        OVL_REQUIRE(prec == OVL_F64 || prec == OVL_F32, OVL_ERR_UNSUPPORTED, "the adjoint runs in FP64 or FP32");
        OVL_REQUIRE(chi_dev && nrhs >= 1 && nrhs <= MAX_NRHS && (dS_dpsi_dev || dS_dU_dev) &&
                        (psi_dev || !dS_dU_dev),
                    OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(eta > 0.0 && std::isfinite(rho) && mu >= 0.0 && mu < 1.0, OVL_ERR_ARG,
                    "need eta > 0, finite rho, 0 <= mu < 1");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, OVL_F64) * nrhs;
        double2 *chi = (double2 *)ctx->buf("api_a64", FB);
        double2 *psi = dS_dU_dev ? (double2 *)ctx->buf("api_c64", FB) : nullptr;
        double2 *dpsi = dS_dpsi_dev ? (double2 *)ctx->buf("api_b64", FB) : nullptr;
        pack_spinor(*ctx, chi_dev, chi, nrhs, OVL_F64);
        if (psi) pack_spinor(*ctx, psi_dev, psi, nrhs, OVL_F64);
        if (stats_host) std::memset(stats_host, 0, sizeof(ovl_stats));
        overlap_adjoint(*ctx, rho, mu, *zolo, psi, chi, dpsi, (double2 *)dS_dU_dev, nrhs, eta, prec, 100000,
                        stats_host);
        if (dpsi) unpack_spinor(*ctx, dpsi, dS_dpsi_dev, nrhs, OVL_F64);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof_collect();
    });
}

ovl_status ovl_sumr_gmresr_solve(ovl_context *ctx, const ovl_zolo *zolo, const ovl_solver_params *params,
                                 const double *b_dev, double *x_dev, int32_t nrhs, ovl_stats *stats_host)
{
    ovl_status worst = OVL_OK;
    ovl_status st = guard([&] {
        check_ctx(ctx);
        check_zolo(zolo);
        OVL_REQUIRE(params != nullptr && b_dev && x_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG,
                    "bad solver arguments");
        const ovl_solver_params &p = *params;
        OVL_REQUIRE(p.mu >= 0.0 && p.mu < 1.0 && p.tol > 0.0 && p.eta_tilde > 0.0 && p.relax_floor > 0.0 &&
                        p.max_outer >= 1 && p.max_middle >= 1 && p.max_mscg >= 1 && p.norm_restart > 0.0,
                    OVL_ERR_ARG, "invalid solver parameters");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        const size_t FB = field_bytes(ctx->g, OVL_F64);
        if (stats_host) std::memset(stats_host, 0, sizeof(ovl_stats) * nrhs);
        // calculating (eigSUMR / eigCG) solves run one right-hand side after
        // another unless they collect as a block; otherwise all right-hand
        // sides are solved together
        OVL_REQUIRE(!(p.eig_block && p.middle_cg), OVL_ERR_UNSUPPORTED, "block collection needs the relSUMR middle solve");
        const int batch = (p.eig_calc && !p.eig_block) ? 1 : nrhs;
        double2 *b = (double2 *)ctx->buf("api_b64", FB * batch);
        double2 *x = (double2 *)ctx->buf("api_x64", FB * batch);
        for (int f0 = 0; f0 < nrhs; f0 += batch) {
            const int nb = std::min(batch, nrhs - f0);
            pack_spinor(*ctx, b_dev + (size_t)f0 * ctx->g.V * 24, b, nb, OVL_F64);
            const ovl_status r = solve_batch(*ctx, *zolo, p, b, x, nb, stats_host ? stats_host + f0 : nullptr);
            unpack_spinor(*ctx, x, x_dev + (size_t)f0 * ctx->g.V * 24, nb, OVL_F64);
            if (r != OVL_OK && worst == OVL_OK) worst = r;
        }
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof_collect();
        if (worst != OVL_OK) set_error("solver: iteration limit reached");
    });
    return st != OVL_OK ? st : worst;
}

ovl_status ovl_eigspace_info(ovl_context *ctx, int32_t *n_held, int32_t cap, double *ritz_host,
                             double *resid_host, int32_t *n_diag)
{
    return guard([&] {
        check_ctx(ctx);
        const EigSpace &e = ctx->eig;
        if (n_held) *n_held = e.k;
        if (n_diag) *n_diag = e.ndiag;
        for (int i = 0; i < cap && i < (int)e.ritz.size(); ++i) {
            if (ritz_host) ritz_host[i] = e.ritz[i];
            if (resid_host) resid_host[i] = e.resid[i];
        }
    });
}

ovl_status ovl_eigspace_get(ovl_context *ctx, double *v_dev, double *vD_dev)
{
    return guard([&] {
        check_ctx(ctx);
        const EigSpace &e = ctx->eig;
        if (e.k > 0) {
            if (v_dev) unpack_spinor(*ctx, e.V, v_dev, e.k, OVL_F64);
            if (vD_dev) unpack_spinor(*ctx, e.VD, vD_dev, e.k, OVL_F64);
        }
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_eigspace_set(ovl_context *ctx, int32_t n, int32_t m, double mu, double delta, int32_t k,
                            const double *v_dev, const double *vD_dev)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(mu >= 0.0 && mu < 1.0 && delta > 0.0 && delta < 0.5, OVL_ERR_ARG, "need 0 <= mu < 1, 0 < delta < 1/2");
        OVL_REQUIRE(k >= 0 && k <= m, OVL_ERR_ARG, "need 0 <= k <= m");
        if (k > 0) OVL_REQUIRE(v_dev && vD_dev, OVL_ERR_ARG, "null eigenspace data");
        EigSpace &e = ctx->eig;
        e.mu = -1.0;   // force a fresh configuration
        eig_configure(*ctx, n, m, mu, delta, e.eps, e.krecalc);
        if (k > 0) {
            pack_spinor(*ctx, v_dev, e.V, k, OVL_F64);
            pack_spinor(*ctx, vD_dev, e.VD, k, OVL_F64);
        }
        e.k = k;
        e.ndiag = k > 0 ? 1 : 0;   // treat installed vectors as eigenvector estimates
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

// File layout of a saved eigenspace: the 8-byte tag "OVLEIG01", int32
// extents[4], n, m, k, ndiag, k_recalc, n_uv, n_ritz; double mu, delta, eps;
// double uv[n_uv], ritz[n_ritz], resid[n_ritz]; then the k vectors v and the
// k images v^D, each 12 V complex128 in the canonical layout.
static const char EIG_TAG[8] = {'O', 'V', 'L', 'E', 'I', 'G', '0', '1'};

ovl_status ovl_eigspace_save(ovl_context *ctx, const char *path)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(path != nullptr, OVL_ERR_ARG, "null path");
        const EigSpace &e = ctx->eig;
        OVL_REQUIRE(e.m > 0, OVL_ERR_STATE, "eigenspace not configured");
        std::FILE *fp = std::fopen(path, "wb");
        OVL_REQUIRE(fp != nullptr, OVL_ERR_ARG, std::string("cannot open ") + path + " for writing");
        bool ok = std::fwrite(EIG_TAG, 1, 8, fp) == 8;
        const int32_t hdr[11] = {ctx->g.L[0], ctx->g.L[1], ctx->g.L[2], ctx->g.L[3], e.n, e.m, e.k, e.ndiag,
                                 e.krecalc, (int32_t)e.uv_hist.size(), (int32_t)e.ritz.size()};
        const double par[3] = {e.mu, e.delta, e.eps};
        ok = ok && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 && std::fwrite(par, sizeof(par), 1, fp) == 1;
        auto wr = [&](const std::vector<double> &v) {
            ok = ok && (v.empty() || std::fwrite(v.data(), sizeof(double), v.size(), fp) == v.size());
        };
        wr(e.uv_hist);
        wr(e.ritz);
        wr(e.resid);
        const size_t FB = field_bytes(ctx->g, OVL_F64);
        double *canon = (double *)ctx->buf("eigio_canon", FB);
        void *host = ctx->host_stage(FB);
        for (int set = 0; set < 2 && ok; ++set)
            for (int i = 0; i < e.k && ok; ++i) {
                unpack_spinor(*ctx, (set ? e.VD : e.V) + (size_t)i * 12 * ctx->g.V, canon, 1, OVL_F64);
                OVL_HIP(hipMemcpyAsync(host, canon, FB, hipMemcpyDeviceToHost, ctx->stream));
                OVL_HIP(hipStreamSynchronize(ctx->stream));
                ok = std::fwrite(host, 1, FB, fp) == FB;
            }
        ok = (std::fclose(fp) == 0) && ok;
        OVL_REQUIRE(ok, OVL_ERR_ARG, std::string("write to ") + path + " failed");
    });
}

ovl_status ovl_eigspace_load(ovl_context *ctx, const char *path)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(path != nullptr, OVL_ERR_ARG, "null path");
        std::FILE *fp = std::fopen(path, "rb");
        OVL_REQUIRE(fp != nullptr, OVL_ERR_ARG, std::string("cannot open ") + path);
        struct Closer {
            std::FILE *f;
            ~Closer() { std::fclose(f); }
        } closer{fp};
        char tag[8];
        int32_t hdr[11];
        double par[3];
        OVL_REQUIRE(std::fread(tag, 1, 8, fp) == 8 && std::memcmp(tag, EIG_TAG, 8) == 0, OVL_ERR_ARG,
                    "not an eigenspace file");
        OVL_REQUIRE(std::fread(hdr, sizeof(hdr), 1, fp) == 1 && std::fread(par, sizeof(par), 1, fp) == 1, OVL_ERR_ARG,
                    "truncated eigenspace file");
        for (int mdim = 0; mdim < 4; ++mdim)
            OVL_REQUIRE(hdr[mdim] == ctx->g.L[mdim], OVL_ERR_ARG, "eigenspace file is for other lattice extents");
        const int n = hdr[4], m = hdr[5], k = hdr[6], nuv = hdr[9], nritz = hdr[10];
        OVL_REQUIRE(n >= 1 && m > n && m <= 512 && k >= 0 && k <= m && nuv >= 0 && nuv <= 10 && nritz >= 0 &&
                        nritz <= m && hdr[7] >= 0 && hdr[8] >= 1,
                    OVL_ERR_ARG, "eigenspace file header out of range");
        OVL_REQUIRE(par[0] >= 0.0 && par[0] < 1.0 && par[1] > 0.0 && par[1] < 0.5 && par[2] > 0.0, OVL_ERR_ARG,
                    "eigenspace file parameters out of range");
        std::vector<double> uv(nuv), ritz(nritz), resid(nritz);
        auto rd = [&](std::vector<double> &v) {
            OVL_REQUIRE(v.empty() || std::fread(v.data(), sizeof(double), v.size(), fp) == v.size(), OVL_ERR_ARG,
                        "truncated eigenspace file");
        };
        rd(uv);
        rd(ritz);
        rd(resid);
        EigSpace &e = ctx->eig;
        e.mu = -1.0;   // fresh configuration
        eig_configure(*ctx, n, m, par[0], par[1], par[2], hdr[8]);
        const size_t FB = field_bytes(ctx->g, OVL_F64);
        double *canon = (double *)ctx->buf("eigio_canon", FB);
        void *host = ctx->host_stage(FB);
        for (int set = 0; set < 2; ++set)
            for (int i = 0; i < k; ++i) {
                OVL_REQUIRE(std::fread(host, 1, FB, fp) == FB, OVL_ERR_ARG, "truncated eigenspace file");
                OVL_HIP(hipMemcpyAsync(canon, host, FB, hipMemcpyHostToDevice, ctx->stream));
                pack_spinor(*ctx, canon, (set ? e.VD : e.V) + (size_t)i * 12 * ctx->g.V, 1, OVL_F64);
                OVL_HIP(hipStreamSynchronize(ctx->stream));   // the staging buffer is reused
            }
        e.k = k;
        e.ndiag = hdr[7];
        e.uv_hist = uv;
        e.ritz = ritz;
        e.resid = resid;
        e.nsets = 0;
        e.defl_ready = false;
        e.spec_ready = false;
    });
}

ovl_status ovl_eigspace_diagonalise(ovl_context *ctx)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(ctx->eig.m > 0, OVL_ERR_STATE, "eigenspace not configured");
        eig_diagonalise(*ctx);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_eigspace_recompute(ovl_context *ctx, double rho, const ovl_zolo *zolo, double eta)
{
    return guard([&] {
        check_ctx(ctx);
        check_zolo(zolo);
        OVL_REQUIRE(eta > 0.0, OVL_ERR_ARG, "eta must be positive");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        eig_recompute(*ctx, rho, *zolo, eta, nullptr);
        OVL_HIP(hipStreamSynchronize(ctx->stream));
        ctx->prof_collect();
    });
}

ovl_status ovl_eigsumr_eigensolve(ovl_context *ctx, const ovl_zolo *zolo, const ovl_solver_params *params,
                                  const double *q0_dev, int32_t max_runs, int32_t diag_per_run, double eta_fixed,
                                  int32_t *runs_out, int64_t *applies_hist, double *maxres_hist, ovl_stats *stats)
{
    ovl_status res = OVL_OK;
    ovl_status st = guard([&] {
        check_ctx(ctx);
        check_zolo(zolo);
        OVL_REQUIRE(params != nullptr && q0_dev != nullptr, OVL_ERR_ARG, "bad eigensolver arguments");
        const ovl_solver_params &p = *params;
        OVL_REQUIRE(p.mu >= 0.0 && p.mu < 1.0 && p.eig_eps > 0.0 && p.norm_restart > 0.0 && p.max_mscg >= 1 &&
                        p.m_eig > p.n_eig && p.n_eig >= 1 && p.delta_split >= 0.0 && p.delta_split < 0.5,
                    OVL_ERR_ARG, "invalid eigensolver parameters");
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        if (stats) std::memset(stats, 0, sizeof(ovl_stats));
        double2 *q0 = (double2 *)ctx->buf("api_q0", field_bytes(ctx->g, OVL_F64));
        pack_spinor(*ctx, q0_dev, q0, 1, OVL_F64);
        int runs = 0;
        res = eig_eigensolve(*ctx, *zolo, p, q0, max_runs, diag_per_run, eta_fixed, &runs, applies_hist,
                             maxres_hist, stats);
        if (runs_out) *runs_out = runs;
        ctx->prof_collect();
        if (res != OVL_OK) set_error("eigensolver: residual target not reached within max_runs runs");
    });
    return st != OVL_OK ? st : res;
}

ovl_status ovl_deflate_project(ovl_context *ctx, const double *b_dev, double *x0_dev, double *Dx0_dev, int32_t nrhs)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(b_dev && x0_dev && Dx0_dev && nrhs >= 1 && nrhs <= MAX_NRHS, OVL_ERR_ARG, "bad field arguments");
        OVL_REQUIRE(ctx->eig.k >= 1, OVL_ERR_STATE, "the eigenspace is empty");
        const size_t FB = field_bytes(ctx->g, OVL_F64);
        double2 *b = (double2 *)ctx->buf("api_b64", FB);
        double2 *x = (double2 *)ctx->buf("api_x64", FB);
        double2 *d = (double2 *)ctx->buf("api_d64", FB);
        for (int f = 0; f < nrhs; ++f) {
            const size_t o = (size_t)f * ctx->g.V * 24;
            pack_spinor(*ctx, b_dev + o, b, 1, OVL_F64);
            eig_project(*ctx, b, x, d);
            unpack_spinor(*ctx, x, x0_dev + o, 1, OVL_F64);
            unpack_spinor(*ctx, d, Dx0_dev + o, 1, OVL_F64);
        }
        OVL_HIP(hipStreamSynchronize(ctx->stream));
    });
}

ovl_status ovl_profile_enable(ovl_context *ctx, int32_t on)
{
    return guard([&] {
        check_ctx(ctx);
        ctx->prof_collect();
        ctx->prof = on != 0;
        for (auto &row : ctx->slots)
            for (auto &s : row) s = ProfileSlot{};
    });
}

ovl_status ovl_profile_read(ovl_context *ctx, int32_t kernel, int32_t prec, int64_t *launches, double *milliseconds,
                            double *bytes)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(kernel >= 0 && kernel < KERN_COUNT && prec >= 0 && prec < 3, OVL_ERR_ARG, "bad slot");
        ctx->prof_collect();
        const ProfileSlot &s = ctx->slots[kernel][prec];
        if (launches) *launches = s.launches;
        if (milliseconds) *milliseconds = s.ms;
        if (bytes) *bytes = s.bytes;
    });
}

ovl_status ovl_sumr_gmresr_solve_many(ovl_instance *inst, int32_t n, const ovl_solver_params *params)
{
    ovl_status st = guard([&] {
        OVL_REQUIRE(inst != nullptr && n >= 1 && n <= 4096 && params != nullptr, OVL_ERR_ARG,
                    "bad instance list");
        std::vector<ovl_context *> seen;
        for (int i = 0; i < n; ++i) {
            OVL_REQUIRE(inst[i].ctx != nullptr, OVL_ERR_ARG, "null context in the instance list");
            seen.push_back(inst[i].ctx);
        }
        std::sort(seen.begin(), seen.end());
        OVL_REQUIRE(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), OVL_ERR_ARG,
                    "an instance list may hold each context once");
    });
    if (st != OVL_OK) return st;
    // a bounded pool of host threads takes instances from a shared counter;
    // each keeps its instance's error text (ovl_last_error is per thread)
    const int workers = std::min<int>(n, MAX_SOLVE_THREADS);
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    pool.reserve(workers);
    for (int w = 0; w < workers; ++w)
        pool.emplace_back([&next, n, inst, params] {
            for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
                ovl_instance &q = inst[i];
                q.message[0] = '\0';
                q.status = ovl_sumr_gmresr_solve(q.ctx, q.zolo, params, q.b_dev, q.x_dev, q.nrhs, q.stats);
                if (q.status != OVL_OK) {
                    std::strncpy(q.message, ovl::last_error(), sizeof(q.message) - 1);
                    q.message[sizeof(q.message) - 1] = '\0';
                }
            }
        });
    for (auto &t : pool) t.join();
    for (int i = 0; i < n; ++i)
        if (inst[i].status != OVL_OK) {
            set_error("instance " + std::to_string(i) + ": " + inst[i].message);
            return (ovl_status)inst[i].status;
        }
    return OVL_OK;
}

ovl_status ovl_stream_bench(ovl_context *ctx, int32_t kind, const void *src_dev, void *dst_dev, int64_t bytes,
                            int32_t reps, double *ms_host)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(kind == 0 || kind == 1, OVL_ERR_ARG, "kind must be 0 (copy) or 1 (read)");
        OVL_REQUIRE(src_dev && dst_dev && ms_host && reps >= 1, OVL_ERR_ARG, "bad arguments");
        OVL_REQUIRE(bytes >= 16 * 1024 * 1024 && bytes % 16 == 0, OVL_ERR_ARG,
                    "bytes must be a multiple of 16 and at least 16 MiB");
        OVL_REQUIRE(((uintptr_t)src_dev | (uintptr_t)dst_dev) % 16 == 0, OVL_ERR_ARG, "buffers must be 16-byte aligned");
        *ms_host = stream_bench(*ctx, kind, src_dev, dst_dev, bytes, reps);
    });
}

ovl_status ovl_set_option(ovl_context *ctx, int32_t option, int32_t value)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(value == 0 || value == 1, OVL_ERR_ARG, "option value must be 0 or 1");
        if (option == OVL_OPT_GRAPHS)
            ctx->use_graphs = value != 0;
        else if (option == OVL_OPT_AUTOTUNE)
            ctx->autotune = value;
        else if (option == OVL_OPT_ADAPTIVE_NZ)
            ctx->adaptive_nz = value != 0;
        else if (option == OVL_OPT_BOUND_PRINTED)
            ctx->eig.bound_printed = value != 0;
        else if (option == OVL_OPT_TWO_ROW_LINKS) {
            ctx->two_row_opt = value != 0;
            update_link_form(*ctx);
        } else if (option == OVL_OPT_OUTER_PRINTED)
            ctx->outer_printed = value != 0;
        else
            throw Error{OVL_ERR_ARG, "unknown option"};
    });
}

ovl_status ovl_gauge_info(ovl_context *ctx, double *su3_deviation, int32_t *two_row)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(ctx->have_gauge, OVL_ERR_STATE, "no gauge field loaded");
        if (su3_deviation) *su3_deviation = ctx->su3_dev;
        if (two_row) *two_row = ctx->g.two_row;
    });
}

ovl_status ovl_tuning_get(ovl_context *ctx, int32_t *keys, int32_t *variants, int32_t cap, int32_t *n)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(n != nullptr && cap >= 0 && (cap == 0 || (keys && variants)), OVL_ERR_ARG, "bad arguments");
        int i = 0;
        for (const auto &kv : ctx->tuned) {
            if (i < cap) {
                keys[i] = kv.first;
                variants[i] = kv.second;
            }
            ++i;
        }
        *n = i;
    });
}

ovl_status ovl_tuning_set(ovl_context *ctx, const int32_t *keys, const int32_t *variants, int32_t n)
{
    return guard([&] {
        check_ctx(ctx);
        OVL_REQUIRE(n >= 0 && (n == 0 || (keys && variants)), OVL_ERR_ARG, "bad arguments");
        for (int i = 0; i < n; ++i) {
            const int prec = keys[i] / 512;
            OVL_REQUIRE(keys[i] >= 0 && prec <= OVL_HALF && stencil_variant_ok(ctx->g, prec, variants[i]),
                        OVL_ERR_ARG, "tuning variant out of range for this lattice and precision");
        }
        for (int i = 0; i < n; ++i) ctx->tuned[keys[i]] = variants[i];
    });
}

}  // extern "C"
