// Host-side launchers of the device kernels (all asynchronous on `st`).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.h"

namespace matnc {

// complex64
hipError_t launch_stream(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st);
int mfma_config_count();
int mfma_config_tn(int cfg);  // complex N columns of a tile configuration
bool mfma_config_fits(int cfg, int mbits, int nbits, int kbits);
hipError_t launch_mfma(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st);
// fan-out tiles (d.fan_off / d.n_fan describe the grouping)
bool mfma_fan_config_fits(int cfg, int mbits, int nbits, int kbits, int fan_tn);
hipError_t launch_mfma_fan(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st);
// the same, also recording each output instance's maximum (its scale slot
// must have been cleared)
hipError_t launch_mfma_fan_rec(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st);
// adds the root instances of slices sigma0 .. sigma0+nb-1 into rows[0..nrows)
// of amps (root.gmap_off: local root instance of each row position)
hipError_t launch_slice_sum(const OpDesc& root, uint64_t ws, const int64_t* sig, int nb, int64_t nrows,
                            const int32_t* rows, int open_bits, double* amps, hipStream_t st);

// complex-half
bool chalf_available();
hipError_t launch_stream_h(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st);
int mfma_h_config_count();
int mfma_h_config_tn(int cfg);
bool mfma_h_config_fits(int cfg, int mbits, int nbits, int kbits);
hipError_t launch_mfma_h(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st);
bool mfma_h_fan_config_fits(int cfg, int mbits, int nbits, int kbits, int fan_tn);
hipError_t launch_mfma_h_fan(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st);
hipError_t launch_slice_sum_h(const OpDesc& root, uint64_t ws, const int64_t* sig, int nb, int64_t nrows,
                              const int32_t* rows, int open_bits, double* amps, hipStream_t st);

hipError_t launch_zero(uint64_t ptr, uint64_t bytes, hipStream_t st);
// records max |re|, |im| of each FP32 output instance of d into its scale
// slot (atomic max; the slot must have been cleared)
hipError_t launch_absmax(const NodeDesc& d, uint64_t ws, hipStream_t st);

// shared
hipError_t launch_xeb(const double* amps, int64_t count, int n_qubits, double* out, hipStream_t st);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st);

}  // namespace matnc
