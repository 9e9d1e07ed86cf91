// C-ABI entry points of the learned preconditioner network: validation on the
// host, then the launches of net.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace okinv {
namespace {

#define NET_TRY(expr)                    \
    do {                                 \
        int _r = (expr);                 \
        if (_r != OK_SUCCESS) return _r; \
    } while (0)

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

int check_fields(int nfields, int flags, bool allow_adjoint) {
    if (nfields < 1 || nfields > 65536) {
        set_error("nfields = %d outside [1, 65536]", nfields);
        return OK_EINVAL;
    }
    const int known = OK_SPINOR_RHS_INNER | (allow_adjoint ? OK_NET_ADJOINT : 0);
    if (flags & ~known) {
        set_error("unknown flags 0x%x", flags);
        return OK_EINVAL;
    }
    return OK_SUCCESS;
}

int check_layers(int n) {
    if (n < 1 || n > OK_NET_MAX_LAYERS) {
        set_error("n_layers = %d outside [1, %d]", n, OK_NET_MAX_LAYERS);
        return OK_EINVAL;
    }
    return OK_SUCCESS;
}

int check_net(const ok_net* net) {
    if (!net) {
        set_error("net is NULL");
        return OK_EINVAL;
    }
    NET_TRY(check_layers(net->n_layers));
    NET_TRY(check_ptr(net->d_params, "net->d_params"));
    return check_ptr(net->d_T, "net->d_T");
}

size_t field_bytes(const Geo& g, int nf) { return (size_t)g.V * 12 * 8 * nf; }

// Workspace of a training pass: every layer's output, then the gradient
// partials, then the loss scratch.
struct TrainWork {
    float* acts[OK_NET_MAX_LAYERS];
    float* wpart;
    void* loss;
};
size_t train_layout(const Geo& g, int n_layers, int nf, char* base, TrainWork* w) {
    size_t off = 0;
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off += align256(n);
        return p;
    };
    TrainWork tmp;
    TrainWork& W = w ? *w : tmp;
    for (int l = 0; l < n_layers; ++l) W.acts[l] = reinterpret_cast<float*>(take(field_bytes(g, nf)));
    W.wpart = reinterpret_cast<float*>(take(net_wgrad_partial_bytes(g, nf)));
    W.loss = take(net_loss_partial_bytes(nf));
    return off;
}

size_t workspace(const Geo& g, int n_layers, int nf, int training) {
    if (training == 1) return train_layout(g, n_layers, nf, nullptr, nullptr);
    if (training == 2) return align256(net_wgrad_partial_bytes(g, nf)) + align256(net_loss_partial_bytes(nf));
    return net_apply_work_bytes(g, n_layers, nf);
}

int loss_and_grad(const Geo& g, int n_layers, const float* params, const float* T, const float* xi,
                  const float* psi, int nf, bool inner, double* loss, float* grad, const TrainWork& W,
                  hipStream_t st) {
    constexpr int PL = 27 * 16 * 2;   // floats per layer
    for (int l = 0; l < n_layers; ++l)
        NET_TRY(launch_net_layer(g, nf, inner, false, params + (size_t)l * PL, T, l ? W.acts[l - 1] : xi,
                                 W.acts[l], st));
    float* gout = W.acts[n_layers - 1];
    NET_TRY(launch_net_loss_grad(g, nf, inner, gout, psi, gout, loss, W.loss, st));
    // backward: the gradient of layer l's output lives in acts[l]; the
    // adjoint of layer l writes the gradient of its input over acts[l - 1]
    // once layer l's weight gradient (which reads that input) is done
    for (int l = n_layers - 1; l >= 0; --l) {
        const float* in = l ? W.acts[l - 1] : xi;
        NET_TRY(launch_net_wgrad(g, nf, inner, T, W.acts[l], in, W.wpart, grad + (size_t)l * PL, st));
        if (l)
            NET_TRY(launch_net_layer(g, nf, inner, true, params + (size_t)l * PL, T, W.acts[l], W.acts[l - 1], st));
    }
    return OK_SUCCESS;
}

int check_training_args(const Geo& G, int n_layers, const float* d_xi, const float* d_psi, int nfields, int flags,
                        double* d_loss, float* d_grad, void* d_work, size_t work_bytes) {
    NET_TRY(check_layers(n_layers));
    NET_TRY(check_fields(nfields, flags, false));
    NET_TRY(check_ptr(d_xi, "d_xi"));
    NET_TRY(check_ptr(d_psi, "d_psi"));
    NET_TRY(check_ptr(d_grad, "d_grad"));
    NET_TRY(check_ptr(d_work, "d_work"));
    if (!d_loss) {
        set_error("d_loss is NULL");
        return OK_EINVAL;
    }
    const size_t need = workspace(G, n_layers, nfields, 1);
    if (work_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", work_bytes, need);
        return OK_ESIZE;
    }
    if (overlaps(d_work, need, d_xi, field_bytes(G, nfields)) || overlaps(d_work, need, d_psi, field_bytes(G, nfields))) {
        set_error("d_work must not overlap d_xi or d_psi");
        return OK_EINVAL;
    }
    return OK_SUCCESS;
}

}  // namespace

size_t net_apply_work_bytes(const Geo& g, int n_layers, int nf) {
    return (size_t)std::min(n_layers - 1, 2) * align256(field_bytes(g, nf));
}

int net_apply(const Geo& g, int n_layers, const float* params, const float* T, const float* in, float* out, int nf,
              bool inner, void* work, hipStream_t st) {
    constexpr int PL = 27 * 16 * 2;
    float* tmp[2] = {reinterpret_cast<float*>(work),
                     reinterpret_cast<float*>(reinterpret_cast<char*>(work) + align256(field_bytes(g, nf)))};
    const float* src = in;
    for (int l = 0; l < n_layers; ++l) {
        float* dst = l == n_layers - 1 ? out : tmp[l & 1];
        NET_TRY(launch_net_layer(g, nf, inner, false, params + (size_t)l * PL, T, src, dst, st));
        src = dst;
    }
    return OK_SUCCESS;
}

}  // namespace okinv

using namespace okinv;

extern "C" {

int ok_net_param_count(int n_layers, size_t* n_floats) {
    NET_TRY(check_layers(n_layers));
    if (!n_floats) {
        set_error("n_floats is NULL");
        return OK_EINVAL;
    }
    *n_floats = (size_t)n_layers * 27 * 16 * 2;
    return OK_SUCCESS;
}

int ok_net_transports_bytes(const ok_geom* g, size_t* bytes) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    if (!bytes) {
        set_error("bytes is NULL");
        return OK_EINVAL;
    }
    *bytes = net_T_bytes(G);
    return OK_SUCCESS;
}

int ok_net_transports(const ok_geom* g, const double* d_links, float* d_T, size_t T_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_ptr(d_links, "d_links"));
    NET_TRY(check_ptr(d_T, "d_T"));
    if (T_bytes < net_T_bytes(G)) {
        set_error("transport buffer has %zu bytes, needs %zu", T_bytes, net_T_bytes(G));
        return OK_ESIZE;
    }
    if (overlaps(d_T, net_T_bytes(G), d_links, (size_t)G.V * 4 * 9 * 16)) {
        set_error("d_T must not overlap d_links");
        return OK_EINVAL;
    }
    return launch_net_transports(G, d_links, d_T, reinterpret_cast<hipStream_t>(stream));
}

int ok_net_layer(const ok_geom* g, const float* d_A, const float* d_T, const float* d_in, float* d_out,
                 int nfields, int flags, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_fields(nfields, flags, true));
    NET_TRY(check_ptr(d_A, "d_A"));
    NET_TRY(check_ptr(d_T, "d_T"));
    NET_TRY(check_ptr(d_in, "d_in"));
    NET_TRY(check_ptr(d_out, "d_out"));
    if (overlaps(d_in, field_bytes(G, nfields), d_out, field_bytes(G, nfields))) {
        set_error("d_out must not overlap d_in");
        return OK_EINVAL;
    }
    return launch_net_layer(G, nfields, flags & OK_SPINOR_RHS_INNER, flags & OK_NET_ADJOINT, d_A, d_T, d_in, d_out,
                            reinterpret_cast<hipStream_t>(stream));
}

int ok_net_workspace_bytes(const ok_geom* g, int n_layers, int nfields, int training, size_t* bytes) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_layers(n_layers));
    NET_TRY(check_fields(nfields, 0, false));
    if (training < 0 || training > 2 || !bytes) {
        set_error("training must be 0, 1 or 2 and bytes non-NULL");
        return OK_EINVAL;
    }
    *bytes = std::max<size_t>(256, workspace(G, n_layers, nfields, training));
    return OK_SUCCESS;
}

int ok_net_apply(const ok_geom* g, const ok_net* net, const float* d_in, float* d_out, int nfields, int flags,
                 void* d_work, size_t work_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_net(net));
    NET_TRY(check_fields(nfields, flags, false));
    NET_TRY(check_ptr(d_in, "d_in"));
    NET_TRY(check_ptr(d_out, "d_out"));
    const size_t need = net_apply_work_bytes(G, net->n_layers, nfields);
    if (need) {
        NET_TRY(check_ptr(d_work, "d_work"));
        if (work_bytes < need) {
            set_error("workspace has %zu bytes, needs %zu", work_bytes, need);
            return OK_ESIZE;
        }
    }
    const size_t fb = field_bytes(G, nfields);
    if (overlaps(d_in, fb, d_out, fb) || (need && (overlaps(d_work, need, d_in, fb) || overlaps(d_work, need, d_out, fb)))) {
        set_error("d_in, d_out and d_work must not overlap");
        return OK_EINVAL;
    }
    return net_apply(G, net->n_layers, net->d_params, net->d_T, d_in, d_out, nfields, flags & OK_SPINOR_RHS_INNER,
                     d_work, reinterpret_cast<hipStream_t>(stream));
}

int ok_net_layer_wgrad(const ok_geom* g, const float* d_T, const float* d_gout, const float* d_in, float* d_gA,
                       int nfields, int flags, void* d_work, size_t work_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_fields(nfields, flags, false));
    NET_TRY(check_ptr(d_T, "d_T"));
    NET_TRY(check_ptr(d_gout, "d_gout"));
    NET_TRY(check_ptr(d_in, "d_in"));
    NET_TRY(check_ptr(d_gA, "d_gA"));
    NET_TRY(check_ptr(d_work, "d_work"));
    if (work_bytes < net_wgrad_partial_bytes(G, nfields)) {
        set_error("workspace has %zu bytes, needs %zu", work_bytes, net_wgrad_partial_bytes(G, nfields));
        return OK_ESIZE;
    }
    return launch_net_wgrad(G, nfields, flags & OK_SPINOR_RHS_INNER, d_T, d_gout, d_in,
                            reinterpret_cast<float*>(d_work), d_gA, reinterpret_cast<hipStream_t>(stream));
}

int ok_net_loss_grad(const ok_geom* g, const float* d_out, const float* d_psi, float* d_gout, double* d_loss,
                     int nfields, int flags, void* d_work, size_t work_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_fields(nfields, flags, false));
    NET_TRY(check_ptr(d_out, "d_out"));
    NET_TRY(check_ptr(d_psi, "d_psi"));
    NET_TRY(check_ptr(d_gout, "d_gout"));
    NET_TRY(check_ptr(d_work, "d_work"));
    if (!d_loss) {
        set_error("d_loss is NULL");
        return OK_EINVAL;
    }
    if (work_bytes < net_loss_partial_bytes(nfields)) {
        set_error("workspace has %zu bytes, needs %zu", work_bytes, net_loss_partial_bytes(nfields));
        return OK_ESIZE;
    }
    const size_t fb = field_bytes(G, nfields);
    if (d_gout != d_out && overlaps(d_gout, fb, d_out, fb)) {
        set_error("d_gout must equal d_out or not overlap it");
        return OK_EINVAL;
    }
    return launch_net_loss_grad(G, nfields, flags & OK_SPINOR_RHS_INNER, d_out, d_psi, d_gout, d_loss, d_work,
                                reinterpret_cast<hipStream_t>(stream));
}

int ok_net_loss_and_grad(const ok_geom* g, const ok_net* net, const float* d_xi, const float* d_psi, int nfields,
                         int flags, double* d_loss, float* d_grad, void* d_work, size_t work_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_net(net));
    NET_TRY(check_training_args(G, net->n_layers, d_xi, d_psi, nfields, flags, d_loss, d_grad, d_work, work_bytes));
    TrainWork W;
    train_layout(G, net->n_layers, nfields, reinterpret_cast<char*>(d_work), &W);
    return loss_and_grad(G, net->n_layers, net->d_params, net->d_T, d_xi, d_psi, nfields, flags & OK_SPINOR_RHS_INNER,
                         d_loss, d_grad, W, reinterpret_cast<hipStream_t>(stream));
}

int ok_cast_f64_to_f32(const double* d_in, float* d_out, size_t n, void* stream) {
    NET_TRY(check_ptr(d_in, "d_in"));
    NET_TRY(check_ptr(d_out, "d_out"));
    if (n == 0 || n > (size_t)1 << 40) {
        set_error("n = %zu outside [1, 2^40]", n);
        return OK_EINVAL;
    }
    if (overlaps(d_in, n * 8, d_out, n * 4)) {
        set_error("d_out must not overlap d_in");
        return OK_EINVAL;
    }
    return launch_cast((long)n, d_in, d_out, reinterpret_cast<hipStream_t>(stream));
}

int ok_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, size_t n, const ok_adam_cfg* cfg, int step,
                 void* stream) {
    NET_TRY(check_ptr(d_p, "d_p"));
    NET_TRY(check_ptr(d_g, "d_g"));
    NET_TRY(check_ptr(d_m, "d_m"));
    NET_TRY(check_ptr(d_v, "d_v"));
    if (!cfg || step < 1 || n == 0 || n > (size_t)1 << 40) {
        set_error("cfg must be non-NULL, step >= 1 and 0 < n");
        return OK_EINVAL;
    }
    if (!(cfg->lr >= 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) ||
        !(cfg->eps > 0) || !std::isfinite(cfg->lr)) {
        set_error("invalid Adam settings (lr >= 0, 0 <= beta < 1, eps > 0)");
        return OK_EINVAL;
    }
    return launch_adam((long)n, d_p, d_g, d_m, d_v, *cfg, step, reinterpret_cast<hipStream_t>(stream));
}

int ok_net_train_step(const ok_geom* g, int n_layers, float* d_params, float* d_m, float* d_v, const float* d_T,
                      const float* d_xi, const float* d_psi, int nfields, int flags, const ok_adam_cfg* cfg, int step,
                      double* d_loss, float* d_grad, void* d_work, size_t work_bytes, void* stream) {
    Geo G;
    NET_TRY(make_geo(g, &G));
    NET_TRY(check_training_args(G, n_layers, d_xi, d_psi, nfields, flags, d_loss, d_grad, d_work, work_bytes));
    NET_TRY(check_ptr(d_params, "d_params"));
    NET_TRY(check_ptr(d_m, "d_m"));
    NET_TRY(check_ptr(d_v, "d_v"));
    NET_TRY(check_ptr(d_T, "d_T"));
    if (!cfg || step < 1) {
        set_error("cfg must be non-NULL and step >= 1");
        return OK_EINVAL;
    }
    const size_t np = (size_t)n_layers * 27 * 16 * 2;
    if (overlaps(d_grad, np * 4, d_params, np * 4)) {
        set_error("d_grad must not overlap d_params");
        return OK_EINVAL;
    }
    TrainWork W;
    train_layout(G, n_layers, nfields, reinterpret_cast<char*>(d_work), &W);
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    NET_TRY(loss_and_grad(G, n_layers, d_params, d_T, d_xi, d_psi, nfields, flags & OK_SPINOR_RHS_INNER, d_loss,
                          d_grad, W, st));
    return ok_adam_step(d_params, d_grad, d_m, d_v, np, cfg, step, stream);
}

}  // extern "C"
