"""MI355X (gfx950) implementation of the Alternating Metropolis-Hastings sampler
(arXiv 2211.03193): HIP kernels behind the C ABI of libamh.so, with a thin
Python binding in :mod:`paper_2211_03193_amd.amh`."""
