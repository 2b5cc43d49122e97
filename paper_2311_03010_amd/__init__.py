"""MI355X-native EECMG image restoration (arXiv 2311.03010).

The HIP library is loaded on first use by ``paper_2311_03010_amd.eecmg``;
importing the package (for example for the synthetic workload generator)
does not touch the GPU.
"""
