// launch.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include "device.h"

namespace pclaunch {
using pcdev::Params;
using pcdev::Soa;
using pcdev::Soa32;
using pcdev::SoaIO;

// t0/t1 (optional, both or neither): events that take the start and end
// timestamps of the launch itself (hipExtLaunchKernelGGL), so that their
// elapsed time is the kernel's duration without the queue gaps around it
hipError_t advance(const Params& P, int species, const Soa& sp, int64_t* rho, uint8_t* ev, int64_t evlen,
                   int grid, hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t advance(const Params& P, int species, const Soa32& sp, int64_t* rho, uint8_t* ev, int64_t evlen,
                   int grid, hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t finish(const Params& P, const Soa& se, const Soa& si, int64_t* rho_e, int64_t* rho_i,
                  int64_t* zero_a, int64_t* zero_b, hipStream_t st);
hipError_t finish(const Params& P, const Soa32& se, const Soa32& si, int64_t* rho_e, int64_t* rho_i,
                  int64_t* zero_a, int64_t* zero_b, hipStream_t st);
hipError_t field(const Params& P, const int64_t* rho_e, const int64_t* rho_i, double* E, double* phi,
                 int ghost, hipStream_t st);
hipError_t scale_field(const Params& P, hipStream_t st);
hipError_t load(const Params& P, int species, const Soa& sp, int64_t n0, double sig, hipStream_t st);
hipError_t load(const Params& P, int species, const Soa32& sp, int64_t n0, double sig, hipStream_t st);
hipError_t halfstep(const Params& P, const Soa& sp, int64_t n, double hq, hipStream_t st);
hipError_t halfstep(const Params& P, const Soa32& sp, int species, int64_t n, hipStream_t st);
hipError_t to64(const Params& P, const Soa32& src, const SoaIO& dst, int64_t n, int species, hipStream_t st);
hipError_t from64(const Params& P, const SoaIO& src, const Soa32& dst, int64_t n, int species, hipStream_t st);
hipError_t vt_split(const double2* vt, double* vy, double* vz, int64_t n, hipStream_t st);
hipError_t vt_join(const double* vy, const double* vz, double2* vt, int64_t n, hipStream_t st);
hipError_t fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t deposit(const Params& P, const double* x, int64_t n, int64_t* rho, hipStream_t st);
hipError_t deposit(const Params& P, const Soa32& sp, int64_t n, int64_t* rho, hipStream_t st);
hipError_t copy_soa(const Soa& dst, const Soa& src, int64_t n, hipStream_t st);
hipError_t stream_copy(const double* src, double* dst, int64_t n, int blocks, hipStream_t st);
hipError_t moments(const Params& P, const Soa& se, const Soa& si, int32_t cpg, int reset, int64_t* out,
                   int64_t out_len, hipStream_t st);
hipError_t moments(const Params& P, const Soa32& se, const Soa32& si, int32_t cpg, int reset, int64_t* out,
                   int64_t out_len, hipStream_t st);
hipError_t sort(const Params& P, int species, const Soa& src, const Soa& dst, int grid, hipStream_t st);
hipError_t sort(const Params& P, int species, const Soa32& src, const Soa32& dst, int grid, hipStream_t st);
hipError_t batch_push_e(const pcdev::ColumnDev* cols, int fp32, const pcdev::BatchItem* items, int n,
                        const pcdev::BatchStep& b, hipStream_t st, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
hipError_t batch_advance_i(const pcdev::ColumnDev* cols, int fp32, const pcdev::BatchItem* items, int n,
                           const pcdev::BatchStep& b, hipStream_t st);
hipError_t batch_finish(const pcdev::ColumnDev* cols, int n_cols, int fp32, const pcdev::BatchStep& b,
                        hipStream_t st);
hipError_t batch_sort(const pcdev::ColumnDev* cols, int n_cols, int fp32, int species, const pcdev::BatchItem* items,
                      int n, int cur, hipStream_t st);
hipError_t slot_map(const Params& P, const Soa& se, const Soa& si, hipStream_t st);
hipError_t slot_map(const Params& P, const Soa32& se, const Soa32& si, hipStream_t st);
int max_nodes();

}  // namespace pclaunch
