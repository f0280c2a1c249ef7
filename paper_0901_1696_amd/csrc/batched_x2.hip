// The batched solver's persistent loop built for two workgroups per compute
// unit (batched_kernel_x2 and its launcher only; everything else of the
// batched solver is in batched.hip).  A separate translation unit, so that
// every device function the loop calls is compiled under that kernel's
// register budget.
#define RFP_BATCHED_X2 1
#include "batched.hip"
