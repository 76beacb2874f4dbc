// debug.hip -- host-side self-check entry points (include/pentago_debug.h).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/pentago_debug.h"
#include "internal.h"

using namespace pg;

static Set256 from_abi(const pentago_set256 *s)
{
    Set256 r;
    memcpy(r.w, s->w, 32);
    return r;
}

static void to_abi(const Set256 &s, pentago_set256 *out) { memcpy(out->w, s.w, 32); }

extern "C" {

int pentago_debug_five(pentago_board board, int color, pentago_set256 *out)
{
    if (!out || (color != 1 && color != 2)) return fail(PENTAGO_EINVAL, "invalid arguments");
    const HostTables &H = host_tables();
    LineMasks lm[4];
    for (int j = 0; j < 4; j++) {
        if (board.q[j] >= 19683) return fail(PENTAGO_EINVAL, "invalid quadrant code");
        unsigned m = 0;
        int x = board.q[j];
        for (int l = 0; l < 9; l++, x /= 3)
            if (x % 3 == color) m |= 1u << l;
        lm[j] = H.lm[j * 512 + m];
    }
    to_abi(five_set(lm[0], lm[1], lm[2], lm[3]), out);
    return 0;
}

int pentago_debug_rmax(const pentago_set256 *in, pentago_set256 *out)
{
    if (!in || !out) return fail(PENTAGO_EINVAL, "NULL argument");
    to_abi(rmax(from_abi(in)), out);
    return 0;
}

int pentago_debug_shift(const pentago_set256 *in, int d, int k, pentago_set256 *out)
{
    if (!in || !out || d < 0 || d > 3) return fail(PENTAGO_EINVAL, "invalid arguments");
    to_abi(shift_dim(from_abi(in), d, k), out);
    return 0;
}

int pentago_debug_swap3(const pentago_set256 *in, int d, pentago_set256 *out)
{
    if (!in || !out || d < 0 || d > 3) return fail(PENTAGO_EINVAL, "invalid arguments");
    Set256 x = from_abi(in);
    swap_with3_rt(x, d);
    to_abi(x, out);
    return 0;
}

int pentago_debug_sym(const pentago_set256 *in, int sym, const int h[4], pentago_set256 *out)
{
    if (!in || !out || !h || sym < 0 || sym > 7) return fail(PENTAGO_EINVAL, "invalid arguments");
    Set256 x = from_abi(in);
    sym_apply_rt(x, sym, h);
    to_abi(x, out);
    return 0;
}

int pentago_debug_sym_pattern(int sym, int black, int white, int index, int *src_index, int *h)
{
    const HostTables &H = host_tables();
    if (sym < 0 || sym > 7 || black < 0 || white < 0 || black + white > 9 || !src_index || !h)
        return fail(PENTAGO_EINVAL, "invalid arguments");
    if (index < 0 || index >= H.class_size[black][white]) return fail(PENTAGO_EINVAL, "index out of range");
    const uint16_t e = H.symmap[sym * kPatterns + H.class_start[black][white] + index];
    *src_index = e & 0xfff;
    *h = e >> 12;
    return 0;
}

int pentago_debug_canon(int code, int *index, int *k)
{
    if (code < 0 || code >= 19683 || !index || !k) return fail(PENTAGO_EINVAL, "invalid arguments");
    const uint16_t c = host_tables().canon[code];
    *index = c & 0xfff;
    *k = c >> 12;
    return 0;
}

}  // extern "C"
