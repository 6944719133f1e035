// Text reports for verdicts, in the shape of the wrapper's report in Sec. 4.5
// (Listing 6): a one-line diagnosis naming the copy direction, followed by
// the byte count the copy needs and the bytes the device allocation offers.
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/xfercheck.h"

namespace {

const char *direction(uint32_t kind)
{
    switch (kind) {
    case CG_H2D: return "host->device";
    case CG_D2H: return "device->host";
    case CG_D2D: return "device->device";
    default: return "unknown";
    }
}

void line(std::string &s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void line(std::string &s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (!s.empty()) s += '\n';
    s += buf;
}

}  // namespace

extern "C" int cg_format_verdict(const cg_transfer *rec, const cg_verdict *v, char *buf, uint64_t len)
{
    if (!rec || !v || (!buf && len)) return CG_EINVAL;
    std::string s;
    const uint32_t f = v->flags;
    const char *dir = direction(rec->kind);
    if (f & CG_BAD_KIND) {
        line(s, "Error: Unknown copy kind %u.", rec->kind);
    } else {
        if (f & (CG_SRC_UNALLOC | CG_DST_UNALLOC)) {
            line(s, "Error: %s of %s copy is not in allocated device memory.",
                 (f & CG_SRC_UNALLOC) ? ((f & CG_DST_UNALLOC) ? "Source and destination" : "Source") : "Destination",
                 dir);
        }
        if (f & (CG_SRC_OVERRUN | CG_DST_OVERRUN)) {
            line(s, "Error: Allocated device memory too small for %s copy.", dir);
            line(s, "Expected %" PRIu64 " allocated bytes but only found %" PRIu64 ".", rec->n, v->avail);
        }
        if (f & CG_SRC_UNADDR)
            line(s, "Error: Source of %s copy is not addressable host memory (first bad byte at offset %" PRIu64 ").",
                 dir, v->first_bad);
        if (f & CG_DST_UNADDR)
            line(s, "Error: Destination of %s copy is not addressable host memory.", dir);
        if (f & CG_SRC_UNDEF) {
            // undefined host data sent to the device is the error class of
            // Sec. 2; from a device source the definedness is only carried on
            line(s, "%s: %" PRIu64 " undefined byte%s in %s copy.",
                 rec->kind == CG_H2D ? "Error" : "Note", v->undef_bytes, v->undef_bytes == 1 ? "" : "s", dir);
        }
        if (f & CG_OVERLAP)
            line(s, "Warning: Source and destination of %s copy overlap; definedness not propagated.", dir);
    }
    if (f & CG_ROWS_LIMIT) line(s, "Note: not every row of the pitched %s copy was checked.", dir);
    if (len) {
        const size_t k = s.size() < len - 1 ? s.size() : (size_t)len - 1;
        s.copy(buf, k);
        buf[k] = '\0';
    }
    return (int)s.size();
}
