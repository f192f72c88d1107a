// Batched block Gauss-Seidel launches of one shape: float vector blocks, 8 column(s) per lane,
// 4 lane(s) per row.
#define BGS_SHAPE_T float
#define BGS_SHAPE_V 8
#define BGS_SHAPE_P 4
#include "block_gs_batched.inl"
