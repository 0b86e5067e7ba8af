// sos.hip -- cascades of second-order sections (biquads), the structure the
// paper's experiments name for higher orders (Sec. 4: higher-order filters
// are usually built from second-order sections to keep rounding errors
// small), with SciPy's sosfilt semantics: section s filters the output of
// section s - 1 in the transposed direct form II with its own initial state.
//
// Every section runs the transposed-form path of tdf.hip over the whole
// signal.  The backward recomputes the sections' inputs (the forward outputs
// of sections 0 .. S-2) into the workspace and then runs the sections'
// backward passes from the last to the first; the input gradient of section
// s is the output gradient of section s - 1 (chain rule).
#include "common.h"

namespace filt_detail {
namespace {

filt_status sos_check(const filt_problem *p, int32_t nsec)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    if (nsec < 1)
        return fail(FILT_EINVAL, "at least one section is needed (got %d)", (int)nsec);
    if (p->M != 2 || p->N != 2)
        return fail(FILT_EINVAL, "sections are biquads: M and N must be 2 (got %d, %d)", p->M,
                    p->N);
    return FILT_OK;
}

size_t sig_bytes(const filt_problem *p)
{
    return align256((size_t)(p->B * p->T) * sizeof(float));
}

}  // namespace
}  // namespace filt_detail

using namespace filt_detail;

extern "C" {

filt_status filt_sos_workspace_bytes(const filt_problem *p, int32_t nsec, size_t *bytes)
{
    filt_status s = sos_check(p, nsec);
    if (s != FILT_OK)
        return s;
    if (bytes == nullptr)
        return fail(FILT_EINVAL, "bytes is NULL");
    size_t inner = 0;
    s = filt_tdf_workspace_bytes(p, &inner);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0) {
        *bytes = 0;
        return FILT_OK;
    }
    // backward: the inputs of sections 1 .. S-1 and two gradient signals;
    // the forward needs two of those signals
    *bytes = 256 + (size_t)(nsec + 1) * sig_bytes(p) + align256(inner);
    return FILT_OK;
}

filt_status filt_sos_forward(const filt_problem *p, int32_t nsec, const float *x, const float *b,
                             const float *a, const float *zi, float *y, void *ws, size_t ws_bytes,
                             void *stream)
{
    size_t need = 0;
    filt_status s = filt_sos_workspace_bytes(p, nsec, &need);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (x == nullptr || b == nullptr || a == nullptr || y == nullptr)
        return fail(FILT_EINVAL, "x, b, a and y are required");
    if (ws == nullptr || ws_bytes < need)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const size_t sb = sig_bytes(p);
    float *buf[2] = {(float *)base, (float *)(base + sb)};
    char *inner = base + (size_t)(nsec + 1) * sb;
    const size_t inner_bytes = ws_bytes - (size_t)(inner - (char *)ws);
    const int64_t B = p->B;
    for (int32_t k = 0; k < nsec && s == FILT_OK; ++k) {
        const float *in = k == 0 ? x : buf[(k - 1) & 1];
        float *out = k == nsec - 1 ? y : buf[k & 1];
        s = filt_tdf_forward(p, in, b + k * B * 3, a + k * B * 2,
                             zi != nullptr ? zi + k * B * 2 : nullptr, out, inner, inner_bytes,
                             stream);
    }
    return s;
}

filt_status filt_sos_backward(const filt_problem *p, int32_t nsec, const float *gy,
                              const float *x, const float *y, const float *b, const float *a,
                              const float *zi, float *gx, float *gb, float *ga, float *gzi,
                              void *ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    filt_status s = filt_sos_workspace_bytes(p, nsec, &need);
    if (s != FILT_OK)
        return s;
    if (p->B == 0)
        return FILT_OK;
    const int64_t B = p->B;
    if (p->T == 0) {
        // no output: every per-section gradient is zero
        for (int32_t k = 0; k < nsec && s == FILT_OK; ++k)
            s = filt_tdf_backward(p, gy, x, y, b, a, zi, nullptr,
                                  gb != nullptr ? gb + k * B * 3 : nullptr,
                                  ga != nullptr ? ga + k * B * 2 : nullptr,
                                  gzi != nullptr ? gzi + k * B * 2 : nullptr, nullptr, 0, stream);
        return s;
    }
    if (gy == nullptr || x == nullptr || y == nullptr || b == nullptr || a == nullptr)
        return fail(FILT_EINVAL, "gy, x, y, b and a are required");
    if (ws == nullptr || ws_bytes < need)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const size_t sb = sig_bytes(p);
    // inputs of sections 1 .. S-1, then two gradient signals
    auto input_of = [&](int32_t k) -> float * { return (float *)(base + (size_t)(k - 1) * sb); };
    float *gbuf[2] = {(float *)(base + (size_t)(nsec - 1) * sb),
                      (float *)(base + (size_t)nsec * sb)};
    char *inner = base + (size_t)(nsec + 1) * sb;
    const size_t inner_bytes = ws_bytes - (size_t)(inner - (char *)ws);
    for (int32_t k = 0; k + 1 < nsec && s == FILT_OK; ++k)
        s = filt_tdf_forward(p, k == 0 ? x : input_of(k), b + k * B * 3, a + k * B * 2,
                             zi != nullptr ? zi + k * B * 2 : nullptr, input_of(k + 1), inner,
                             inner_bytes, stream);
    const float *g = gy;
    for (int32_t k = nsec - 1; k >= 0 && s == FILT_OK; --k) {
        const float *in = k == 0 ? x : input_of(k);
        const float *out = k == nsec - 1 ? y : input_of(k + 1);
        float *gin = k == 0 ? gx : gbuf[k & 1];
        s = filt_tdf_backward(p, g, in, out, b + k * B * 3, a + k * B * 2,
                              zi != nullptr ? zi + k * B * 2 : nullptr, gin,
                              gb != nullptr ? gb + k * B * 3 : nullptr,
                              ga != nullptr ? ga + k * B * 2 : nullptr,
                              gzi != nullptr ? gzi + k * B * 2 : nullptr, inner, inner_bytes,
                              stream);
        g = gin;
    }
    return s;
}

}  // extern "C"
