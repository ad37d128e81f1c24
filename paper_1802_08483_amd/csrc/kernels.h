// Launchers for the gfx950 kernels (implemented in kernels.hip).
#pragma once

#include "mapdec_internal.h"

namespace mapdec {

// fp64 != 0 selects the double-precision instantiation of each kernel.
hipError_t launch_init(const FrameDesc *fd, int nframes, hipStream_t st);
hipError_t launch_pack(const FrameDesc *fd, const Work *tab, int nblocks, hipStream_t st);
hipError_t launch_lattice(int fp64, int mn, int imode, const FrameDesc *fd, const Work *tab,
                          int nblocks, hipStream_t st);
hipError_t launch_gamma(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                        hipStream_t st);
hipError_t launch_chain(int fp64, const FrameDesc *fd, const int *frames, int nchains,
                        size_t lds_bytes, hipStream_t st);
hipError_t launch_app(int fp64, const FrameDesc *fd, const Work *tab, int nblocks,
                      size_t lds_bytes, hipStream_t st);

// Block sizes the host uses to build work tables.
constexpr int kPackWords = 8;      // packed words per pack workgroup (256 threads)
constexpr int kLatticeLanes = 64;  // start indices per lattice workgroup
constexpr int kGammaLanes = 256;   // drift states per Gamma workgroup
constexpr int kChainThreads = 256;
constexpr int kAppThreads = 64;

}  // namespace mapdec
