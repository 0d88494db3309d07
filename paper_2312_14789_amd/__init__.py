"""MI355X-native meshless lattice Boltzmann step (arXiv 2312.14789).

`mlbm` binds the C ABI of libmlbm.so (include/mlbm.h); `units` holds the
paper's unit conversions and memory model.  Importing `mlbm` fails when the
library is not built: there is no fallback path.
"""
