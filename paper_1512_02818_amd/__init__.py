"""MI355X-native first-stage Feynman-Kac nodal solver (probabilistic domain
decomposition). The HIP library is loaded lazily by ``paper_1512_02818_amd.pdd``."""
