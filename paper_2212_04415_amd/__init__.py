"""MI355X-native peridynamic MC/MLMC hot path (arXiv 2212.04415).

The solve runs in libpdmi.so (HIP kernels for gfx950, C ABI in
include/pd.h); `pd` binds it one-to-one and `beam` adds argument marshalling
for beam workloads.  Importing the package does not load the library, so the
build step can run without a GPU; the first call into `pd` loads it and fails
loudly if it has not been built."""

__all__ = ["pd", "beam", "build"]
