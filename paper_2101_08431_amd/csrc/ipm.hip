#include "ipm.h"

namespace nmfk {

size_t ipm_workspace_bytes(int64_t, int64_t, int) { return 0; }
nmf_status ipm_bind(IpmState &s, uint8_t *, int64_t, int64_t, int) { s.bound = true; return NMF_OK; }
nmf_status ipm_transition(IpmState &s, const AnlsParams &, const nmf_options &, hipStream_t) {
    s.err = "stage 2 not available";
    return NMF_ESTATE;
}
nmf_status ipm_iterate(IpmState &s, const AnlsParams &, const nmf_options &, int, hipStream_t) {
    s.err = "stage 2 not available";
    return NMF_ESTATE;
}
nmf_status ipm_report(IpmState &, nmf_report *, double, double) { return NMF_ESTATE; }
nmf_status ipm_export(IpmState &, const AnlsParams &, hipStream_t) { return NMF_OK; }
const char *ipm_last_error(const IpmState &s) { return s.err.c_str(); }

}  // namespace nmfk
