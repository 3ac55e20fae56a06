"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds input generators only: byte streams shaped like fixed-width
HEP record files and seeded initial weights for the byte-level Mamba
predictor.  It contains none of the compressor's arithmetic (no model step, no
probability quantisation, no range coding), so both the CPU oracle and the GPU
path can draw their inputs from it without sharing any of the method.

The paper evaluates on CERN open-data files (Methodology, Dataset) that are not
available here; the generators below stand in for them with the same kind of
structure: little-endian, row-major serialised records of float32 / int32 /
float16 / counter fields.
"""
from .records import (  # noqa: F401
    records_f32_mix, records_structured64, raw_normal_f32,
    chunk_lengths_uniform, chunk_lengths_heavy, split_fixed, mixed_chunks,
)
from .weights import ModelConfig, param_layout, param_count, init_weights  # noqa: F401
