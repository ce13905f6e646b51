// Fused kernels of the padded rule sizes (QXA_FORM_CASES_PADDED): the same
// source as kernels_fused.hip, built as a second translation unit so that the
// two sets of kernels compile in parallel.
#define QXA_FUSED_PADDED
#include "kernels_fused.hip"
