"""Hash of the HIP sources and build flags, to tie recorded hardware-counter results to the
kernel code they were taken on."""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    with open(os.path.join(HERE, "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(kernel_source_hash())
