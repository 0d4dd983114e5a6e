"""MI355X-native Huffman encoder (histogram -> parallel canonical codebook ->
chunked reduce/shuffle-merge encoding), after Tian et al., arXiv 2010.10039.

`paper_2010_10039_amd.hf` is the Python binding of the C-ABI library
`libhf.so` (HIP kernels for gfx950); `paper_2010_10039_amd.workloads` holds
the seeded input generators.
"""
