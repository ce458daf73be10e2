"""MI355X-native sequential multi-view deconvolution (arXiv 1308.0730)."""
