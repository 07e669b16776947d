// Stand-ins for the device launch functions of the HIP kernel files, so that
// the library's host logic (amber_api.cpp) links into a CPU-only harness.
// None of them is reached by the harness; each reports "not implemented".
#include "../../paper_2109_10375_amd/csrc/internal.h"

int fft_radiation(const amber_plan_s*, const float*, const double*, int, float* const*, unsigned char*,
                  const WsLayout&, hipStream_t) { return AMBER_E_UNIMPL; }
int fft_forward(const amber_plan_s*, const float*, float2*, float2*, hipStream_t) { return AMBER_E_UNIMPL; }
int fft_from_spectrum(const amber_plan_s*, float2*, float2*, const double*, int, float* const*, float2*, float2*,
                      hipStream_t) { return AMBER_E_UNIMPL; }
int fft_schedule_count(int, int* a, int* b) { *a = *b = 1; return AMBER_OK; }
int fft_schedule_info(int, int, int, int* a, int* b) { *a = *b = 1; return AMBER_OK; }
int halo_source_spectrum(const amber_plan_s*, const float*, const float*, long long, int, int, unsigned char*,
                         const WsLayout&, hipStream_t) { return AMBER_E_UNIMPL; }
int spectra_bins(const amber_plan_s*, const float2*, const float2*, int, const float2*, const float2*, int, int,
                 double*, hipStream_t) { return AMBER_E_UNIMPL; }
int rank_sort(const amber_plan_s*, const float*, const float*, unsigned char*, const WsLayout&, hipStream_t, int,
              uint32_t*) { return AMBER_E_UNIMPL; }
int match_scan(const amber_plan_s*, const amber_weibull*, int, float* const*, unsigned char*, const WsLayout&,
               hipStream_t) { return AMBER_E_UNIMPL; }
int status_collect(const amber_plan_s*, unsigned char*, const WsLayout&, unsigned*, bool, hipStream_t) {
    return AMBER_E_UNIMPL;
}
int noalloc_scratch_address(int, void** out) {
    *out = nullptr;
    return AMBER_E_HIP;
}
