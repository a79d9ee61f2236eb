"""MI355X-native runtime for QoS-aware GPU microservice pipelines (Camelot, arXiv 2005.02088).

The product is the C-ABI library libcamelot.so (include/camelot.h); ``camelot`` is
its Python binding.
"""
