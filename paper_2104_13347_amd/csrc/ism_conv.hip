// Source convolution + sensor noise (placeholder until the MFMA path lands).
#include <hip/hip_runtime.h>

#include "../../include/ism.h"
#include "ism_host.h"

void ism_conv_release(ism_handle *h) { (void)h; }
void ism_serve_release(ism_handle *h) { (void)h; }

extern "C" int ism_convolve_batch(ism_handle *h, int n_rooms, int M, const float *rirs, const int64_t *rir_offset,
                                  const int32_t *rir_len, const float *src, int src_len, int out_len,
                                  const float *snr_db, const float *z, int use_mfma, float *out, ism_stream stream)
{
    (void)n_rooms; (void)M; (void)rirs; (void)rir_offset; (void)rir_len; (void)src; (void)src_len;
    (void)out_len; (void)snr_db; (void)z; (void)use_mfma; (void)out; (void)stream;
    if (h) ism_set_error(h, "not implemented");
    return ISM_EINVAL;
}
