// C-ABI entry points of the material field on its own: evaluation at a batch
// of points and the pull-back of output gradients onto its parameters (the
// kernels are in field.h, shared with the renderer's field material mode).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "field.h"
#include "runtime.h"

namespace mrs {
namespace {

#define HIPTRY_F(x, what) do { mrs_status st_ = hip_check((x), what); if (st_ != MRS_OK) return st_; } while (0)

mrs_status field_args(const mrs_field *field, const float *d_x, int64_t n, FieldDev &fd) {
    const char *why = nullptr;
    if (!make_field_dev(field, fd, &why)) return fail(MRS_EINVAL, "%s", why);
    if (n < 0) return fail(MRS_EINVAL, "n < 0");
    if (n > 0 && !d_x) return fail(MRS_EINVAL, "d_x is NULL");
    if ((uint64_t)n > (1ull << 40)) return fail(MRS_EOVERFLOW, "more than 2^40 points");
    return MRS_OK;
}

}  // namespace
}  // namespace mrs

using namespace mrs;

extern "C" mrs_status mrs_field_eval(const mrs_field *field, const float *d_x, int64_t n, float *d_m, void *stream) {
    clear_error();
    FieldDev fd;
    mrs_status st = field_args(field, d_x, n, fd);
    if (st != MRS_OK) return st;
    if (n > 0 && !d_m) return fail(MRS_EINVAL, "d_m is NULL");
    if (n == 0) return MRS_OK;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t tiles = ((uint64_t)n + kFieldTile - 1) / kFieldTile;
    if (tiles > 0x7FFFFFFFull) return fail(MRS_EOVERFLOW, "too many points for one launch");
    k_field_eval<PointsArray><<<(unsigned)tiles, 64, 0, s>>>(fd, PointsArray{d_x, (uint64_t)n}, d_m);
    HIPTRY_F(hipGetLastError(), "k_field_eval launch");
    return MRS_OK;
}

extern "C" mrs_status mrs_field_backward(const mrs_field *field, const float *d_x, const float *d_grad_m, int64_t n,
                                         const mrs_field_grads *grads, void *stream) {
    clear_error();
    FieldDev fd;
    mrs_status st = field_args(field, d_x, n, fd);
    if (st != MRS_OK) return st;
    if (!grads) return fail(MRS_EINVAL, "grads is NULL");
    if (n > 0 && !d_grad_m) return fail(MRS_EINVAL, "d_grad_m is NULL");
    if (n == 0) return MRS_OK;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t tiles = ((uint64_t)n + kFieldTile - 1) / kFieldTile;
    FieldGrads g{grads->table, grads->w1, grads->b1, grads->w2, grads->b2};
    k_field_backward<PointsArray><<<field_backward_blocks(tiles), 64, 0, s>>>(fd, PointsArray{d_x, (uint64_t)n},
                                                                              d_grad_m, g);
    HIPTRY_F(hipGetLastError(), "k_field_backward launch");
    return MRS_OK;
}
