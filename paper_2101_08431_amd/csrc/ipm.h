// Stage 2 of the two-stage NMF (Sec. III, IV, Alg. 3): transition and the
// primal-dual line-search interior-point iterations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nmf.h"
#include "nmf_internal.h"

namespace nmfk {

struct IpmState {
    bool bound = false;
    std::string err;
};

size_t ipm_workspace_bytes(int64_t n, int64_t m_cap, int K);
nmf_status ipm_bind(IpmState &s, uint8_t *base, int64_t n, int64_t m_cap, int K);
nmf_status ipm_transition(IpmState &s, const AnlsParams &p, const nmf_options &o, hipStream_t st);
nmf_status ipm_iterate(IpmState &s, const AnlsParams &p, const nmf_options &o, int iters, hipStream_t st);
nmf_status ipm_report(IpmState &s, nmf_report *r, double ms1, double ms2);
nmf_status ipm_export(IpmState &s, const AnlsParams &p, hipStream_t st);
const char *ipm_last_error(const IpmState &s);

}  // namespace nmfk
