"""Python access to the plain CPU compactor in ``luda_oracle.c``.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.
"""
from .oracle import (  # noqa: F401
    build, lib, RefError, RefResult, STATUS_NAMES, WHERE_NAMES, PHASE_NAMES,
    crc32c, crc32c_bitwise, crc32c_extend, mask_crc, unmask_crc, xxh64,
    put_varint64, get_varint32, get_varint64,
    bloom_build, bloom_may_match, bloom_size,
    build_tables, build_input_tables, decode_table, compact, compact_job,
    snappy_compress, snappy_decompress, STATUS_CODES,
)
