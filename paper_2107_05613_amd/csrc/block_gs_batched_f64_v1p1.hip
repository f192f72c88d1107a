// Batched block Gauss-Seidel launches of one shape: double vector blocks, 1 column(s) per lane,
// 1 lane(s) per row.
#define BGS_SHAPE_T double
#define BGS_SHAPE_V 1
#define BGS_SHAPE_P 1
#include "block_gs_batched.inl"
