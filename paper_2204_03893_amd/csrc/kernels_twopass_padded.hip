// Two-pass and formation kernels of the padded rule sizes
// (QXA_FORM_CASES_PADDED): the same source as kernels_twopass.hip, built as a
// second translation unit so that the two sets of kernels compile in parallel.
#define QXA_TWOPASS_PADDED
#include "kernels_twopass.hip"
