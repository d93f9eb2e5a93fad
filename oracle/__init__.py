"""FP64 CPU oracle for the MTPT step -- test infrastructure, not the product.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
this package.  See mtpt_oracle.c for what each function computes and the
passage of the paper it follows.
"""
