// Layout constants shared by host precompute and device kernels.
#pragma once
namespace hopu {
// per-element geometry record (doubles): J row-major (d x d), det J,
// |N_F| per local facet, outward unit normal per local facet, |det J|^{(d-1)/d}
enum { GEO_STRIDE = 32, GEO_DET = 9, GEO_NFN = 10, GEO_NRM = 14, GEO_SI = 26 };
}  // namespace hopu
