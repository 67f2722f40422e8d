// C ABI entry points: set-up, operator apply, SL V-cycle, errors.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "handle.h"

namespace helm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

namespace {

using cd = std::complex<double>;

// In-place inverse of a dense k x k complex matrix (row-major) by
// Gauss-Jordan elimination with partial pivoting.  Returns false if singular.
bool invert_dense(std::vector<cd> &a, int k)
{
    std::vector<cd> inv(k * (size_t)k, 0.0);
    for (int i = 0; i < k; ++i) inv[(size_t)i * k + i] = 1.0;
    for (int c = 0; c < k; ++c) {
        int p = c;
        double best = std::abs(a[(size_t)c * k + c]);
        for (int r = c + 1; r < k; ++r)
            if (std::abs(a[(size_t)r * k + c]) > best) {
                best = std::abs(a[(size_t)r * k + c]);
                p = r;
            }
        if (best == 0.0) return false;
        if (p != c)
            for (int j = 0; j < k; ++j) {
                std::swap(a[(size_t)c * k + j], a[(size_t)p * k + j]);
                std::swap(inv[(size_t)c * k + j], inv[(size_t)p * k + j]);
            }
        cd piv = 1.0 / a[(size_t)c * k + c];
        for (int j = 0; j < k; ++j) {
            a[(size_t)c * k + j] *= piv;
            inv[(size_t)c * k + j] *= piv;
        }
        for (int r = 0; r < k; ++r) {
            if (r == c) continue;
            cd fct = a[(size_t)r * k + c];
            if (fct == 0.0) continue;
            for (int j = 0; j < k; ++j) {
                a[(size_t)r * k + j] -= fct * a[(size_t)c * k + j];
                inv[(size_t)r * k + j] -= fct * inv[(size_t)c * k + j];
            }
        }
    }
    a.swap(inv);
    return true;
}

// Dense inverse X of the coarsest-level shifted operator, computed in FP64.
// The operator is block tridiagonal over grid rows: diagonal blocks
// D_I = tridiag(-ih2, 4 ih2 - mass(I, .), -ih2), off-diagonal blocks -ih2 Id.
// Block elimination without block pivoting (the operator's imaginary part is
// positive definite, so every Schur complement is invertible):
//   S_0 = D_0,  S_I = D_I - ih2^2 S_{I-1}^-1,  T_I = S_I^-1.
// Column block c of X solves M X_c = E_c by the block forward/backward
// recurrences Y_I = E_I + ih2 T_{I-1} Y_{I-1},  X_I = T_I (Y_I + ih2 X_{I+1}).
bool coarse_inverse(int nl, double ih2, const std::vector<cd> &mass, std::vector<cd> &X)
{
    const int N = nl * nl;
    std::vector<std::vector<cd>> T(nl);
    std::vector<cd> prev;
    for (int I = 0; I < nl; ++I) {
        std::vector<cd> S((size_t)nl * nl, 0.0);
        for (int J = 0; J < nl; ++J) {
            S[(size_t)J * nl + J] = 4.0 * ih2 - mass[(size_t)I * nl + J];
            if (J > 0) S[(size_t)J * nl + J - 1] = -ih2;
            if (J < nl - 1) S[(size_t)J * nl + J + 1] = -ih2;
        }
        if (I > 0)
            for (size_t q = 0; q < S.size(); ++q) S[q] -= ih2 * ih2 * T[I - 1][q];
        if (!invert_dense(S, nl)) return false;
        T[I] = std::move(S);
    }
    X.assign((size_t)N * N, 0.0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&](int c0) {
        std::vector<cd> Y((size_t)nl * nl * nl), tmp((size_t)nl * nl);  // Y[I] is nl x nl
        for (int c = c0; c < nl; c += (int)nth) {
            // forward: Y_I = 0 for I < c, Y_c = Id, Y_I = ih2 T_{I-1} Y_{I-1}
            std::fill(Y.begin(), Y.end(), cd(0.0));
            for (int J = 0; J < nl; ++J) Y[(size_t)c * nl * nl + (size_t)J * nl + J] = 1.0;
            for (int I = c + 1; I < nl; ++I) {
                const cd *t = T[I - 1].data();
                const cd *yp = &Y[(size_t)(I - 1) * nl * nl];
                cd *yo = &Y[(size_t)I * nl * nl];
                for (int r = 0; r < nl; ++r)
                    for (int k = 0; k < nl; ++k) {
                        cd a = ih2 * t[(size_t)r * nl + k];
                        for (int q = 0; q < nl; ++q) yo[(size_t)r * nl + q] += a * yp[(size_t)k * nl + q];
                    }
            }
            // backward: X_I = T_I (Y_I + ih2 X_{I+1}); column block c of X
            for (int I = nl - 1; I >= 0; --I) {
                cd *yi = &Y[(size_t)I * nl * nl];
                if (I < nl - 1) {
                    const cd *xn = &Y[(size_t)(I + 1) * nl * nl];  // already holds X_{I+1}
                    for (size_t q = 0; q < (size_t)nl * nl; ++q) yi[q] += ih2 * xn[q];
                }
                std::fill(tmp.begin(), tmp.end(), cd(0.0));
                const cd *t = T[I].data();
                for (int r = 0; r < nl; ++r)
                    for (int k = 0; k < nl; ++k) {
                        cd a = t[(size_t)r * nl + k];
                        for (int q = 0; q < nl; ++q) tmp[(size_t)r * nl + q] += a * yi[(size_t)k * nl + q];
                    }
                std::copy(tmp.begin(), tmp.end(), yi);
                for (int r = 0; r < nl; ++r)
                    for (int q = 0; q < nl; ++q)
                        X[(size_t)(I * nl + r) * N + (size_t)c * nl + q] = yi[(size_t)r * nl + q];
            }
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t) pool.emplace_back(work, (int)t);
    for (auto &th : pool) th.join();
    return true;
}

template <typename T>
int dmalloc(T **p, size_t count)
{
    hipError_t e = dev_malloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        *p = nullptr;
        return HELM_E_NOMEM;
    }
    return HELM_OK;
}

}  // namespace

int ensure_vcycle_ws(helm_handle *h, int nb)
{
    if (nb <= h->ws_nb) return HELM_OK;
    for (auto p : h->wf) dev_free(p);
    for (auto p : h->wv) dev_free(p);
    dev_free(h->cpart);
    h->cpart = nullptr;
    h->wf.assign(h->levels, nullptr);
    h->wv.assign(h->levels, nullptr);
    h->ws_nb = 0;
    ++h->ws_gen;
    for (int l = 1; l < h->levels; ++l) {
        size_t Nl = (size_t)h->lv[l].n * h->lv[l].n;
        if (dmalloc(&h->wf[l], Nl * nb) || dmalloc(&h->wv[l], Nl * nb)) return HELM_E_NOMEM;
    }
    if (dmalloc(&h->cpart, coarse_ws(h, nb))) return HELM_E_NOMEM;
    h->ws_nb = nb;
    return HELM_OK;
}

int vcycle(helm_handle *h, const float2 *f, size_t fs, float2 *v, size_t vs, int nb,
           const int *active, hipStream_t s, const double *scale, int accumulate)
{
    int rc = ensure_vcycle_ws(h, nb);
    if (rc) return rc;
    VcycleWs ws;
    for (int l = 0; l < h->levels; ++l) {
        ws.wf[l] = h->wf[l];
        ws.wv[l] = h->wv[l];
    }
    ws.cpart = h->cpart;
    vcycle_with(h, ws, f, fs, v, vs, nb, active, s, scale, accumulate);
    return HELM_OK;
}

// complex elements of the coarsest solve's workspace for nb fields
size_t coarse_ws(const helm_handle *h, int nb)
{
    return h->coarse_gmres > 0 ? coarse_gmres_elems(h->Nc, h->coarse_gmres, nb) : coarse_scratch(h->Nc, nb);
}

size_t vcycle_ws_elems(const helm_handle *h, int nb)
{
    auto up = [](size_t e) { return (e + 31) & ~(size_t)31; };  // 256-byte aligned pieces
    size_t tot = 0;
    for (int l = 1; l < h->levels; ++l) tot += 2 * up((size_t)h->lv[l].n * h->lv[l].n * nb);
    return tot + up(coarse_ws(h, nb));
}

void vcycle_carve(const helm_handle *h, int nb, float2 *base, VcycleWs &ws)
{
    auto up = [](size_t e) { return (e + 31) & ~(size_t)31; };
    size_t off = 0;
    for (int l = 0; l < VcycleWs::MAXL; ++l) ws.wf[l] = ws.wv[l] = nullptr;
    for (int l = 1; l < h->levels; ++l) {
        const size_t e = up((size_t)h->lv[l].n * h->lv[l].n * nb);
        ws.wf[l] = base + off;
        off += e;
        ws.wv[l] = base + off;
        off += e;
    }
    ws.cpart = base + off;
}

void vcycle_with(helm_handle *h, const VcycleWs &ws, const float2 *f, size_t fs, float2 *v, size_t vs,
                 int nb, const int *active, hipStream_t s, const double *scale, int accumulate)
{
    const int L = h->levels;
    if (L == 1) {
        launch_coarse_solve(h->Xc, h->Nc, f, fs, v, vs, nb, active, s, scale, accumulate, ws.cpart);
        return;
    }
    const float sh = (float)h->beta, w = (float)h->jacobi_w;
    // restrict down to the coarsest level
    for (int l = 0; l < L - 1; ++l) {
        const float2 *src = l == 0 ? f : ws.wf[l];
        size_t ss = l == 0 ? fs : (size_t)h->lv[l].n * h->lv[l].n;
        size_t ds = (size_t)h->lv[l + 1].n * h->lv[l + 1].n;
        launch_down(h->lv[l], sh, w, src, ss, ws.wf[l + 1], ds, nb, active, s,
                    l == 0 ? scale : nullptr);
    }
    size_t Nc = (size_t)h->Nc;
    if (h->coarse_gmres > 0)
        launch_coarse_gmres(h->lv[L - 1], sh, w, h->coarse_gmres, ws.wf[L - 1], Nc, ws.wv[L - 1], Nc, nb, active, s,
                            ws.cpart);
    else
        launch_coarse_solve(h->Xc, h->Nc, ws.wf[L - 1], Nc, ws.wv[L - 1], Nc, nb, active, s, nullptr, 0,
                            ws.cpart);
    // prolongate and post-relax up to the finest level
    for (int l = L - 2; l >= 0; --l) {
        size_t Nl = (size_t)h->lv[l].n * h->lv[l].n;
        size_t Nn = (size_t)h->lv[l + 1].n * h->lv[l + 1].n;
        const float2 *src = l == 0 ? f : ws.wf[l];
        size_t ss = l == 0 ? fs : Nl;
        float2 *dst = l == 0 ? v : ws.wv[l];
        size_t dstr = l == 0 ? vs : Nl;
        launch_up(h->lv[l], sh, w, src, ss, ws.wv[l + 1], Nn, dst, dstr, nb, active, s,
                  l == 0 ? scale : nullptr, l == 0 ? accumulate : 0);
    }
}

}  // namespace helm

using namespace helm;

extern "C" {

const char *helm_last_error(void) { return g_err.c_str(); }

int helm_setup(const float *slowness, double omega, const float *gamma, int n,
               const helm_opts *opts, void *stream, helm_handle **out)
{
    if (!out || !slowness || !gamma) {
        set_error("helm_setup: null pointer argument");
        return HELM_E_INVALID;
    }
    *out = nullptr;
    if (!(omega > 0.0) || !std::isfinite(omega)) {
        set_error("helm_setup: omega must be a positive finite number");
        return HELM_E_INVALID;
    }
    if (n < 2 || (n % 2) != 0) {
        set_error("helm_setup: n must be even and >= 2");
        return HELM_E_SHAPE;
    }
    double beta = 0.5, jw = 0.8;
    int levels = 0, cgm = 0;
    if (opts) {
        beta = opts->beta;
        jw = opts->jacobi_weight;
        levels = opts->levels;
        cgm = opts->coarse_gmres;
    }
    if (cgm < 0 || cgm > 30) {
        set_error("helm_setup: coarse_gmres must be in [0, 30]");
        return HELM_E_INVALID;
    }
    if (!(jw > 0.0 && jw < 2.0) || !(beta >= 0.0) || !std::isfinite(beta)) {
        set_error("helm_setup: jacobi_weight must be in (0, 2) and beta >= 0");
        return HELM_E_INVALID;
    }
    if (levels <= 0) {
        levels = 1;
        while ((n >> (levels - 1)) > 64 && ((n >> (levels - 1)) % 2) == 0) ++levels;
    }
    if (levels > 12 || (n % (1 << (levels - 1))) != 0 || (n >> (levels - 1)) < 2) {
        set_error("helm_setup: n must be divisible by 2^(levels-1) with a coarsest size >= 2");
        return HELM_E_SHAPE;
    }
    const int nl = n >> (levels - 1);
    if (cgm > 0 && levels < 2) {
        set_error("helm_setup: a GMRES coarsest solver needs at least two levels");
        return HELM_E_SHAPE;
    }
    if (nl > 128) {
        set_error("helm_setup: coarsest grid larger than 128^2 (dense inverse too big); use more levels");
        return HELM_E_SHAPE;
    }
    hipStream_t s = (hipStream_t)stream;
    auto *h = new helm_handle();
    h->n = n;
    h->levels = levels;
    h->omega = omega;
    h->beta = beta;
    h->jacobi_w = jw;
    h->coarse_gmres = cgm;
    size_t N = (size_t)n * n;
    int rc = HELM_OK;
    auto fail = [&](int code) {
        helm_destroy(h);
        return code;
    };
    if ((rc = dmalloc(&h->kappa0, N)) || (rc = dmalloc(&h->gamma0, N))) return fail(rc);
    if (hipMemcpyAsync(h->kappa0, slowness, N * sizeof(float), hipMemcpyDeviceToDevice, s) ||
        hipMemcpyAsync(h->gamma0, gamma, N * sizeof(float), hipMemcpyDeviceToDevice, s)) {
        set_error("helm_setup: copying the medium failed");
        return fail(HELM_E_HIP);
    }
    h->lv.resize(levels);
    for (int l = 0; l < levels; ++l) {
        Level &L = h->lv[l];
        L.n = n >> l;
        L.ih2 = (float)((double)L.n * (double)L.n);
        if ((rc = dmalloc(&L.mass, (size_t)L.n * L.n))) return fail(rc);
        launch_level_mass(h->kappa0, h->gamma0, n, l, omega, L.mass, L.n, s);
    }
    // coarsest-level inverse on the host in FP64 from the float inputs
    std::vector<float> hk(N), hg(N);
    if (hipMemcpyAsync(hk.data(), h->kappa0, N * sizeof(float), hipMemcpyDeviceToHost, s) ||
        hipMemcpyAsync(hg.data(), h->gamma0, N * sizeof(float), hipMemcpyDeviceToHost, s) ||
        hipStreamSynchronize(s)) {
        set_error("helm_setup: reading the medium back failed");
        return fail(HELM_E_HIP);
    }
    for (size_t p = 0; p < N; ++p)
        if (!std::isfinite(hk[p]) || !std::isfinite(hg[p])) {
            set_error("helm_setup: slowness or gamma holds a non-finite value");
            return fail(HELM_E_INVALID);
        }
    h->Nc = nl * nl;
    if (cgm > 0) {  // no inverse: the coarsest level is solved by GMRES each cycle
        *out = h;
        return HELM_OK;
    }
    const int stp = 1 << (levels - 1);
    std::vector<std::complex<double>> mass((size_t)nl * nl);
    for (int I = 0; I < nl; ++I)
        for (int J = 0; J < nl; ++J) {
            size_t p = (size_t)(I * stp) * n + (size_t)J * stp;
            double k = hk[p], g = hg[p];
            double w2k2 = omega * omega * k * k;
            mass[(size_t)I * nl + J] = std::complex<double>(w2k2, -w2k2 * (g + beta));
        }
    std::vector<std::complex<double>> X;
    if (!coarse_inverse(nl, (double)nl * nl, mass, X)) {
        set_error("helm_setup: coarsest shifted operator is singular");
        return fail(HELM_E_INVALID);
    }
    h->Nc = nl * nl;
    size_t NN = (size_t)h->Nc * h->Nc;
    std::vector<float2> Xf(NN);
    for (size_t q = 0; q < NN; ++q) Xf[q] = make_float2((float)X[q].real(), (float)X[q].imag());
    if ((rc = dmalloc(&h->Xc, NN))) return fail(rc);
    if (hipMemcpyAsync(h->Xc, Xf.data(), NN * sizeof(float2), hipMemcpyHostToDevice, s) ||
        hipStreamSynchronize(s)) {
        set_error("helm_setup: uploading the coarse inverse failed");
        return fail(HELM_E_HIP);
    }
    *out = h;
    return HELM_OK;
}

void helm_destroy(helm_handle *h)
{
    if (!h) return;
    fgmres_free(h);
    dev_free(h->tw);
    dev_free(h->tx);
    dev_free(h->tpart);
    dev_free(h->txt);
    dev_free(h->kcoarse);
    for (auto p : h->wf) dev_free(p);
    for (auto p : h->wv) dev_free(p);
    for (auto &L : h->lv) dev_free(L.mass);
    dev_free(h->Xc);
    dev_free(h->cpart);
    dev_free(h->kappa0);
    dev_free(h->gamma0);
    delete h;
}

int helm_level_size(const helm_handle *h, int l)
{
    if (!h || l < 0 || l >= h->levels) return -1;
    return h->lv[l].n;
}

int helm_num_levels(const helm_handle *h) { return h ? h->levels : -1; }

int helm_apply(helm_handle *h, int op, const float *x, float *y, int nrhs, void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!x || !y)) || (op != HELM_OP_A && op != HELM_OP_M)) {
        set_error("helm_apply: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    size_t N = (size_t)h->n * h->n;
    float shift = op == HELM_OP_M ? (float)h->beta : 0.f;
    launch_apply(h->lv[0], shift, (const float2 *)x, N, (float2 *)y, N, nrhs, nullptr,
                 (hipStream_t)stream);
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

int helm_sl_vcycle(helm_handle *h, const float *f, float *v, int nrhs, void *stream)
{
    if (!h || nrhs < 0 || (nrhs > 0 && (!f || !v))) {
        set_error("helm_sl_vcycle: invalid argument");
        return HELM_E_INVALID;
    }
    if (nrhs == 0) return HELM_OK;
    size_t N = (size_t)h->n * h->n;
    int rc = vcycle(h, (const float2 *)f, N, (float2 *)v, N, nrhs, nullptr, (hipStream_t)stream);
    if (rc) return rc;
    HELM_HIP_CHECK(hipGetLastError());
    return HELM_OK;
}

}  // extern "C"
