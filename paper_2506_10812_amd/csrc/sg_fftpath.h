// sg_fftpath.h -- internal entry points of the FFT path.
#pragma once
#include "sg_internal.h"

size_t sg_fft_disc_ws_bytes(const sg_disc &d);
sg_status sg_fft_run(const sg_disc *discs, int n, void *ws, hipStream_t s);
void sg_fft_release();
int sg_fft_cache_entries();
sg_status sg_fft_profile(const sg_disc *discs, int n, void *ws, hipStream_t s, int reps, float *ms);
sg_status sg_fft_tune(const sg_disc *discs, int n, void *ws, hipStream_t s, sg_tune_result *res, int cap,
                      int *nres);
